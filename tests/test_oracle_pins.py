"""Pins of the paper-form fluxes, the explicit step bound, the Marangoni
face-force stencil and the periodic face arrays (the checks live in
tests/oracle_pins.py, where tests/test_oracle_mutations.py also runs them on
copies of the oracle with planted mistakes)."""
import pytest

from tests import oracle_pins as PINS


@pytest.mark.parametrize("dim,axis", [(2, 0), (2, 1), (3, 2)])
def test_paper_form_flux_vanishes_on_equilibrium_profiles(dim, axis):
    PINS.paper_form_zero_flux_residuals(dim, axis)


def test_paper_form_flux_vanishes_about_a_cylinder_on_rings():
    PINS.paper_form_zero_flux_residuals(2, 0, axisym=True)


def test_paper_form_upwinding_keeps_positivity_at_high_cell_peclet():
    PINS.paper_form_upwind_positivity()


@pytest.mark.parametrize("dim", [2, 3])
def test_step_bound_weighted_diffusion(dim):
    PINS.bound_weighted_diffusion(dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_step_bound_paper_diffusion(dim):
    PINS.bound_paper_diffusion(dim)


def test_step_bound_adsorption_term():
    PINS.bound_adsorption()


def test_step_bound_desorption_term():
    PINS.bound_desorption()


@pytest.mark.parametrize("dim", [2, 3])
def test_force_stencil_exact_for_quadratic_fields(dim):
    PINS.force_stencil_exact_for_quadratics(dim)


def test_periodic_last_face_is_never_read():
    PINS.periodic_last_face_unread()


@pytest.mark.parametrize("kinetics", [0, 1])
@pytest.mark.parametrize("axisym", [False, True], ids=["cartesian", "rings"])
def test_implicit_paper_form_satisfies_its_equations(kinetics, axisym):
    PINS.paper_implicit_residual(kinetics=kinetics, axisym=axisym)

"""The pins of tests/oracle_pins.py are sharp: each plausible mistake in the
oracle (a flipped normal, swapped anti-diffusion weights, the wrong upwind
side, a term dropped from the step bound, a wrong transverse stencil of the
face force, a periodic last face read) is planted, once, in a copy of the
oracle's source compiled on the CPU, and the pin that guards that part must
fail on the copy while it holds on the oracle itself."""
import contextlib
import ctypes
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O
from tests import oracle_pins as PINS

MUTANTS = {
    # section 2.6 / 3.2: n = grad phi/|grad phi| = -grad chi/|grad chi|
    "paper-normal-flipped": [("double n_d = -g[d] / nrm;", "double n_d = g[d] / nrm;")],
    # B_F carries (1 - phi), B_psi (1 - 2 phi): swap them
    "paper-weights-swapped": [
        ("double w = is_bulk ? omega[c] : (omega[c] - phi[c]);",
         "double w = is_bulk ? (omega[c] - phi[c]) : omega[c];")],
    # the anti-diffusive flux taken from the downwind cell of -B
    "paper-downwind": [("double up = Bf < 0.0 ? xs[L] : xs[R];",
                        "double up = Bf < 0.0 ? xs[R] : xs[L];")],
    # the weighted-form neighbour excess cosh(h/eps) - 1 dropped
    "bound-no-cosh": [("(2.0 * nd - 1.0 + cosh(p.h / p.eps))", "(2.0 * nd)")],
    # the k_a Gamma_inf / eps adsorption term dropped
    "bound-no-adsorption": [("lam += p.ka * p.ginf / p.eps + ", "lam += ")],
    # k_d dropped from the interfacial term
    "bound-no-desorption": [("(cmax > 0 ? cmax : 0.0) + p.kd;", "(cmax > 0 ? cmax : 0.0);")],
    # the paper-form anti-diffusion term without sqrt(N_d)
    "bound-paper-no-sqrt": [("sqrt(nd) / (p.eps * p.h)", "1.0 / (p.eps * p.h)")],
    # transverse centred differences not averaged over the two cells
    "force-transverse-left-only": [("g[e] = (tl + tr) / (4.0 * p->h);",
                                    "g[e] = (tl + tl) / (4.0 * p->h);")],
    # transverse differences taken over one cell instead of two
    "force-transverse-factor": [("g[e] = (tl + tr) / (4.0 * p->h);",
                                 "g[e] = (tl + tr) / (2.0 * p->h);")],
    # the cell-mean velocity of a periodic axis read from the literal last face
    "periodic-last-face-read": [
        ("if (a[t] == p->n[t] && p->bc[t][0] == BC_PERIODIC) a[t] = 0;", "")],
    "periodic-last-face-in-bound": [
        ("if (p.bc[d][1] == BC_PERIODIC && a[d] == p.n[d]) a[d] = 0; /* face n_d is face 0 */", "")],
}

# which pin guards which mutant
GUARDS = {
    "paper-normal-flipped": [lambda: PINS.paper_form_zero_flux_residuals(2, 0)],
    "paper-weights-swapped": [lambda: PINS.paper_form_zero_flux_residuals(2, 1)],
    "paper-downwind": [PINS.paper_form_upwind_positivity],
    "bound-no-cosh": [lambda: PINS.bound_weighted_diffusion(2)],
    "bound-no-adsorption": [PINS.bound_adsorption],
    "bound-no-desorption": [PINS.bound_desorption],
    "bound-paper-no-sqrt": [lambda: PINS.bound_paper_diffusion(3)],
    "force-transverse-left-only": [lambda: PINS.force_stencil_exact_for_quadratics(3)],
    "force-transverse-factor": [lambda: PINS.force_stencil_exact_for_quadratics(2)],
    "periodic-last-face-read": [PINS.periodic_last_face_unread],
    "periodic-last-face-in-bound": [PINS.periodic_last_face_unread],
}


# mistakes planted in the implicit oracle (a Python module), each with the
# pin that guards it
PY_MUTANTS = {
    # the anti-diffusive term with the wrong sign in the implicit operator
    "implicit-paper-sign": ("oracle/implicit.py",
                            [("-Bf / h * wL, Bf / h * wR]", "Bf / h * wL, -Bf / h * wR]")],
                            PINS.paper_implicit_residual),
    # the ring weight of a radial face taken from the wrong cell
    "implicit-paper-ring-weight": ("oracle/implicit.py",
                                   [("wR = rhi / np.roll(rmid, -1, axis=ax)", "wR = rhi / rmid")],
                                   lambda I=None: PINS.paper_implicit_residual(I, axisym=True)),
    # the downwind cell of -B
    "implicit-paper-downwind": ("oracle/implicit.py",
                                [("up = np.where(Bf < 0.0, L, R)", "up = np.where(Bf < 0.0, R, L)")],
                                PINS.paper_implicit_residual),
    # the azimuthal curvature of the rings with the wrong sign
    "rings-azimuthal-sign": ("oracle/capillary.py",
                             [("kap -= mx / math.hypot(mx, my) / ring_radius(q, i)",
                               "kap += mx / math.hypot(mx, my) / ring_radius(q, i)")],
                             PINS.rings_capillary),
    # the rings' delta_m without the swept radius (the 2D chord per ring)
    "rings-swept-radius": ("oracle/capillary.py",
                           [("* rm / ring_radius(q, i)", "* 1.0")],
                           PINS.rings_capillary),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_pin_fails_on_planted_mistake(name):
    import importlib.util
    path, edits, check = PY_MUTANTS[name]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, path)).read()
    for a, b in edits:
        assert src.count(a) == 1, (name, a)
        src = src.replace(a, b)
    check()  # holds on the oracle
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "oracle_mutant_%s.py" % name.replace("-", "_"))
        with open(f, "w") as fh:
            # the module imports its sibling with a relative import
            fh.write(src.replace("from . import oracle as O", "from oracle import oracle as O"))
        spec = importlib.util.spec_from_file_location("oracle_mutant", f)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        with pytest.raises(AssertionError):
            check(mod)


@contextlib.contextmanager
def planted(name):
    src = open(O._SRC).read()
    for a, b in MUTANTS[name]:
        assert src.count(a) == 1, (name, a)
        src = src.replace(a, b)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mutant.c")
        so = os.path.join(d, "mutant.so")
        with open(c, "w") as f:
            f.write(src)
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-fopenmp", "-o", so, c, "-lm"])
        old = O._lib
        O._lib = ctypes.CDLL(so)
        try:
            yield
        finally:
            O._lib = old


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_fails_on_planted_mistake(name):
    for check in GUARDS[name]:
        check()  # holds on the oracle
    with planted(name):
        for check in GUARDS[name]:
            with pytest.raises(AssertionError):
                check()

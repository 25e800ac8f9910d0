"""Writes the FP64 oracle's results for the full-size workloads at their
stated step counts, for the GPU parity tests of tests/test_gpu_full_length.py.

    python tests/golden/make_full_length.py [c1 c1i c2 c3 c4]

Only the oracle (oracle/) and the seeded input generators run here: no value
comes from the HIP library.  A full field at these sizes is too large to
keep, so each file holds the oracle's values on a fixed sample of cells
(uniform over the grid plus cells in the interface band of the final level
set), each field's max-norm over the whole grid (the denominator of the
relative max-norm), and the totals of every tenth step.  Each file records
a digest of the workload recipe and of the oracle's source, which the tests
check, so that a changed workload or oracle cannot be compared against a
stale file.

Workloads (paper_2605_27534_amd/configs.py):
  c1  expanding circle 1024^2 (soluble), 2000 steps;
  c1i the insoluble variant, 2000 steps;
  c2  translating sphere 256^3, 50 moving steps (the level set built by the
      oracle's own sweeps from the initial VoF, then warm-started), inputs
      from the torch generators of synth_dev on the host CPU;
  c3  the 64-instance ensemble, 500 steps each;
  c4  the adjoint sphere 128^3: the sigma history at the target parameters,
      then the loss and its gradient at the nominal ones over 100 steps.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2605_27534_amd import configs as C  # noqa: E402

C1_STEPS, C2_STEPS, C3_STEPS, C4_STEPS, C4_CHECKPOINT = 2000, 50, 500, 100, 50
HIST_EVERY = 10


def oracle_digest():
    with open(O._SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recipe_digest(obj):
    def enc(x):
        if isinstance(x, dict):
            return {k: enc(v) for k, v in sorted(x.items()) if not callable(v)}
        if isinstance(x, (list, tuple)):
            return [enc(v) for v in x]
        if isinstance(x, (np.integer,)):
            return int(x)
        if isinstance(x, (np.floating,)):
            return float(x)
        return x
    return hashlib.sha256(json.dumps(enc(obj), sort_keys=True).encode()).hexdigest()[:16]


def c1_recipe():
    cfg = C.c1_expanding_circle()
    return cfg, dict(cfg, steps=C1_STEPS)


def c1i_recipe():
    cfg = C.c1_expanding_circle(soluble=False)
    return cfg, dict(cfg, steps=C1_STEPS)


def c2_recipe():
    cfg = C.c2_translating_sphere()
    return cfg, dict(cfg, steps=C2_STEPS, inputs="synth_dev fp64")


def c3_recipe():
    ens = C.c3_ensemble()
    return ens, [dict(e, steps=C3_STEPS) for e in ens]


def c4_recipe():
    cfg = C.c4_adjoint()
    return cfg, dict(cfg, steps=C4_STEPS, checkpoint_used=C4_CHECKPOINT)


def sample_cells(chi, eps, seed, n_uniform, n_band):
    rng = np.random.default_rng(seed)
    flat = chi.ravel()
    idx_u = rng.choice(flat.size, n_uniform, replace=False)
    band = np.flatnonzero(np.abs(flat) < 8 * eps)
    idx_b = rng.choice(band, min(n_band, band.size), replace=False)
    return np.unique(np.concatenate([idx_u, idx_b])).astype(np.int64)


def fields_record(prefix, idx, **fields):
    out = {prefix + "idx": idx}
    for k, v in fields.items():
        if v is None:
            continue
        v = np.asarray(v).ravel()
        out[prefix + k] = v[idx]
        out[prefix + k + "_maxabs"] = np.array(np.max(np.abs(v)))
    return out


def save(name, rec, recipe):
    rec["oracle_digest"] = np.array(oracle_digest())
    rec["recipe_digest"] = np.array(recipe_digest(recipe))
    path = os.path.join(HERE, "full_length_%s.npz" % name)
    np.savez_compressed(path, **rec)
    print("wrote", path, "%.0f KB" % (os.path.getsize(path) / 1024), flush=True)


def make_c1():
    cfg, recipe = c1_recipe()
    prob, dt = cfg["prob"], cfg["dt"]
    u = cfg["u"]()
    chi = O.geometry(prob, cfg["vof0"](), 72)
    F, P = O.init_state(prob, chi, c0=cfg["c0"](), gamma0=cfg["gamma0"])
    tot = np.zeros(16)
    hist = []
    t0 = time.time()
    for k in range(C1_STEPS):
        chi = O.geometry(prob, cfg["vof_seq"](k), cfg["hj_step"], chi=chi)
        F, P, S, tot = O.step(prob, chi, u, F, P, dt, tot)
        if (k + 1) % HIST_EVERY == 0:
            hist.append(tot.copy())
        if (k + 1) % 200 == 0:
            print("c1 step %d  %.0f s" % (k + 1, time.time() - t0), flush=True)
    eps = 1.5 * prob["h"]
    idx = sample_cells(chi, eps, 101, 2048, 2048)
    rec = fields_record("", idx, chi=chi, F=F, psi=P, sigma=S)
    rec["hist"] = np.array(hist)
    save("c1", rec, recipe)


def make_c1i():
    cfg, recipe = c1i_recipe()
    prob, dt = cfg["prob"], cfg["dt"]
    u = cfg["u"]()
    chi = O.geometry(prob, cfg["vof0"](), 72)
    F, P = O.init_state(prob, chi, gamma0=cfg["gamma0"])
    tot = np.zeros(16)
    hist = []
    t0 = time.time()
    for k in range(C1_STEPS):
        chi = O.geometry(prob, cfg["vof_seq"](k), cfg["hj_step"], chi=chi)
        F, P, S, tot = O.step(prob, chi, u, F, P, dt, tot)
        if (k + 1) % HIST_EVERY == 0:
            hist.append(tot.copy())
        if (k + 1) % 200 == 0:
            print("c1i step %d  %.0f s" % (k + 1, time.time() - t0), flush=True)
    idx = sample_cells(chi, 1.5 * prob["h"], 105, 2048, 2048)
    rec = fields_record("", idx, chi=chi, psi=P, sigma=S)
    rec["hist"] = np.array(hist)
    save("c1i", rec, recipe)


def make_c2():
    import torch
    cfg, recipe = c2_recipe()
    prob, dt = cfg["prob"], cfg["dt"]
    dev = torch.device("cpu")
    chi = O.geometry(prob, cfg["vof0_dev"](dev).numpy(), 108)
    F, P = O.init_state(prob, chi, c0_const=cfg["c0_const"], gamma0=cfg["gamma0"])
    tot = np.zeros(16)
    hist = []
    t0 = time.time()
    for k in range(C2_STEPS):
        chi = O.geometry(prob, cfg["vof_seq_dev"](k, dev).numpy(), cfg["hj_step"], chi=chi)
        u = [x.numpy() for x in cfg["u_seq_dev"](k, dev)]
        F, P, S, tot = O.step(prob, chi, u, F, P, dt, tot)
        if (k + 1) % HIST_EVERY == 0:
            hist.append(tot.copy())
        print("c2 step %d  %.0f s" % (k + 1, time.time() - t0), flush=True)
    eps = 1.5 * prob["h"]
    idx = sample_cells(chi, eps, 102, 2048, 2048)
    rec = fields_record("", idx, chi=chi, F=F, psi=P, sigma=S)
    rec["hist"] = np.array(hist)
    save("c2", rec, recipe)


def make_c3():
    ens, recipe = c3_recipe()
    rec = {}
    t0 = time.time()
    for i, e in enumerate(ens):
        prob, dt = e["prob"], e["dt"]
        chi = O.geometry(prob, e["vof0"](), 72)
        F, P = O.init_state(prob, chi, c0_const=e["c0_const"], gamma0=e["gamma0"])
        chi, F, P, S, hist = O.run(prob, chi, None, F, P, dt, C3_STEPS)
        idx = sample_cells(chi, 1.5 * prob["h"], 300 + i, 64, 64)
        rec.update(fields_record("i%02d_" % i, idx, F=F, psi=P, sigma=S))
        rec["i%02d_tot" % i] = hist[-1]
        print("c3 instance %d (%d^2)  %.0f s" % (i, prob["n"][0], time.time() - t0), flush=True)
    save("c3", rec, recipe)


def make_c4():
    cfg, recipe = c4_recipe()
    prob, dt = cfg["prob"], cfg["dt"]
    chi = O.geometry(prob, cfg["vof0"](), 108)
    u = cfg["u"]()
    c0 = cfg["c0"]()
    t0 = time.time()
    _, target = O.rollout(prob, chi, u, c0, cfg["gamma0"], dt, C4_STEPS, cfg["theta_target"])
    print("c4 target  %.0f s" % (time.time() - t0), flush=True)
    loss, dth, gc0 = O.sigma_history_grad(prob, chi, u, c0, cfg["gamma0"], dt, C4_STEPS,
                                          cfg["theta_nominal"], target)
    print("c4 gradient  %.0f s" % (time.time() - t0), flush=True)
    idx = sample_cells(chi, 1.5 * prob["h"], 104, 2048, 2048)
    rec = fields_record("", idx, gc0=gc0)
    rec["target"] = target
    rec["loss"] = np.array(loss)
    rec["dtheta"] = dth
    save("c4", rec, recipe)


def load(name):
    path = os.path.join(HERE, "full_length_%s.npz" % name)
    return dict(np.load(path, allow_pickle=False))


def current_digests(name):
    recipe = {"c1": c1_recipe, "c1i": c1i_recipe, "c2": c2_recipe, "c3": c3_recipe,
              "c4": c4_recipe}[name]()[1]
    return oracle_digest(), recipe_digest(recipe)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c1i", "c2", "c3", "c4"]
    for w in which:
        {"c1": make_c1, "c1i": make_c1i, "c2": make_c2, "c3": make_c3, "c4": make_c4}[w]()

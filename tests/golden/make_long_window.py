"""Write the long-window parity goldens from the CPU oracle (one-off runs).

Every value stored here comes from the oracle (oracle/) on the seeded
workloads (workloads/); nothing else is imported.  Two files:

* ``c1_fields_20steps.npz`` -- the 82,944-element order-4 FP64 workload
  (layered medium, explosive Ricker source at (5.1, 4.9, 9.1), 64 surface
  receivers) after its first 20 LSERK4 steps from zero fields.  The fields
  are nonzero only near the source, and their size falls steeply with the
  distance from it.  For every element whose largest value is at least
  ``KEEP`` times the global largest value (all other elements are below
  it) the file keeps per-field checksums (the L2 norm over the nodes and a
  sum with seeded +-1 node weights); the elements above ``FULL`` times the
  global largest value, which carry nearly all of the field's norm, are
  stored in full.  Also stored: the full field's norms and the traces.
* ``c3_traces_1500steps.npz`` -- the 24,576-element order-3 FP64 workload
  (true layered medium, same source and receivers) over the full 1500 steps:
  the receiver traces [64][3][1500], and the final fields of 64 seeded
  elements plus the full final field's norms.

The time step is the oracle's CFL formula at 0.5 on the true medium and is
stored with the data; the parity tests hand the same value to the library.

Usage (CPU, minutes for c1, about half an hour for c3 on 8 cores):
    python tests/golden/make_long_window.py [c1] [c3]
"""

import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W                     # noqa: E402
from oracle import solver as O            # noqa: E402

KEEP = 1e-17           # element checked if max |q_e| >= KEEP * max |q|
FULL = 1e-3            # element stored in full if max |q_e| >= FULL * max |q|
C1_WEIGHT_SEED = 20
C1_STEPS = 20
C3_STEPS = 1500
C3_SAMPLE_SEED = 1500
C3_SAMPLE_ELEMENTS = 64


def _setup(name):
    w = W.build_workload(name)
    P = O.Problem(w["mesh"], w["N"])
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
    rho, lam, mu = t(w["rho"]), t(w["lam"]), t(w["mu"])
    P.set_source(w["source"], w["f0"], w["t0"], w["amp"])
    P.set_receivers(w["receivers"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    return w, P, rho, lam, mu, dt


def _norms(q):
    return dict(l2=float(torch.linalg.norm(q)), maxabs=float(q.abs().max()),
                field_l2=np.array([float(torch.linalg.norm(q[:, c])) for c in range(9)]))


def _run(P, rho, lam, mu, dt, nsteps, label):
    q = torch.zeros(P.K, 9, P.Np, dtype=torch.float64)
    traces = []
    t0 = time.time()
    for s in range(nsteps):
        q = O.lserk_step(P, q, s * dt, dt, rho, lam, mu)
        traces.append(O.sample_receivers(P, q))
        if (s + 1) % 10 == 0 or s + 1 == nsteps:
            print("%s: step %d/%d, %.1f s" % (label, s + 1, nsteps, time.time() - t0),
                  flush=True)
    return q, torch.stack(traces, dim=2)


def make_c1():
    w, P, rho, lam, mu, dt = _setup("c1_layered_n24")
    q, tr = _run(P, rho, lam, mu, dt, C1_STEPS, "c1")
    emax = q.abs().amax(dim=(1, 2))
    gmax = float(emax.max())
    keep = torch.nonzero(emax >= KEEP * gmax).reshape(-1)
    full = torch.nonzero(emax >= FULL * gmax).reshape(-1)
    rest = float(emax[emax < KEEP * gmax].max()) if len(keep) < P.K else 0.0
    # per-element, per-field checksums of every kept element: the L2 norm
    # and a sum with seeded +-1 weights over the nodes (catches sign errors)
    wts = np.random.default_rng(C1_WEIGHT_SEED).choice([-1.0, 1.0], size=P.Np)
    qk = q[keep]
    n = _norms(q)
    np.savez_compressed(
        os.path.join(HERE, "c1_fields_20steps.npz"),
        workload=np.array("c1_layered_n24"), steps=C1_STEPS, dt=dt,
        keep_threshold=KEEP, elements=keep.numpy().astype(np.int32),
        field_norms=torch.linalg.norm(qk, dim=2).numpy(),
        weights=wts, field_wsums=(qk.numpy() * wts).sum(axis=2),
        full_threshold=FULL, full_elements=full.numpy().astype(np.int32),
        full_fields=q[full].numpy(), rest_maxabs=rest, l2=n["l2"],
        maxabs=n["maxabs"], field_l2=n["field_l2"], traces=tr.numpy())
    print("c1: %d elements with checksums, %d with full values, max of the rest "
          "%.3e (global max %.3e)" % (len(keep), len(full), rest, gmax), flush=True)


def make_c3():
    w, P, rho, lam, mu, dt = _setup("c3_adjoint")
    q, tr = _run(P, rho, lam, mu, dt, C3_STEPS, "c3")
    rng = np.random.default_rng(C3_SAMPLE_SEED)
    sample = np.sort(rng.choice(P.K, size=C3_SAMPLE_ELEMENTS, replace=False))
    n = _norms(q)
    np.savez_compressed(
        os.path.join(HERE, "c3_traces_1500steps.npz"),
        workload=np.array("c3_adjoint (true medium)"), steps=C3_STEPS, dt=dt,
        traces=tr.numpy(), sample_elements=sample.astype(np.int32),
        sample_fields=q[torch.as_tensor(sample)].numpy(), l2=n["l2"],
        maxabs=n["maxabs"], field_l2=n["field_l2"])
    print("c3: traces max %.3e, final field l2 %.3e" % (float(tr.abs().max()), n["l2"]),
          flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c3"]
    if "c1" in which:
        make_c1()
    if "c3" in which:
        make_c3()

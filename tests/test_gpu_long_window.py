"""Long-window parity of the library against stored oracle runs.

The expected values were written once by tests/golden/make_long_window.py,
which runs only the CPU oracle on the seeded workloads:

* the 82,944-element order-4 workload (layered medium, explosive Ricker
  source, 64 surface receivers) after its first 20 steps from zero fields:
  the elements above 1e-3 of the global largest value in full, per-field
  checksums (norm and a +-1-weighted node sum) of every element above 1e-17
  of it (all others are below), and the full field's norms;
* the 24,576-element order-3 workload (true layered medium, same source and
  receivers) over its full 1500 steps: all receiver traces, the final fields
  of 64 seeded elements and the full final field's norms.

FP64 must match to 1e-12 relative L2, globally and per receiver; per
element the checksums must agree to 1e-10 of the element's own largest field
norm, so an error in a low-amplitude element cannot hide under the global
norm.  The FP32 error on the same data is printed and held to the
short-window bar of 1e-5 on the 20-step window; over 1500 steps it is
reported and held to 1e-4.
"""

import os

import numpy as np
import pytest

import workloads as W
from gpu_helpers import rel_l2, say
from paper_2205_11052_amd import Solver

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("golden %s not generated" % name)
    return np.load(path)


def _run(w, dt, precision, nsteps, launch=None):
    s = Solver(w["N"], precision, 1)
    s.set_mesh_dict(w["mesh"])
    s.set_material(w["rho"], w["lam"], w["mu"])
    s.set_dt(float(dt))
    s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
    s.set_receivers(0, w["receivers"], nsteps)
    if launch is None:
        shape = s.autotune()
    else:
        s.set_launch(*launch)
        shape = launch
    s.zero_fields()
    s.step(nsteps)
    out = s.get_fields(0), s.read_traces(0), shape
    s.close()
    return out


@pytest.mark.parametrize("launch", [None, (0, 7, 0)])
def test_c1_fields_after_20_steps(launch):
    g = _load("c1_fields_20steps.npz")
    w = W.build_workload("c1_layered_n24")
    keep, full = g["elements"], g["full_elements"]
    gmax = float(g["maxabs"])
    norms, wsums, wts = g["field_norms"], g["field_wsums"], g["weights"]
    for prec in (64, 32):
        say("case c1 20 steps, precision %d, launch %s" % (prec, launch))
        q, tr, shape = _run(w, g["dt"], prec, int(g["steps"]), launch)
        err = rel_l2(q[full], g["full_fields"])
        rest = np.ones(w["K"], bool)
        rest[keep] = False
        rest_max = float(np.abs(q[rest]).max()) if rest.any() else 0.0
        total = float(np.linalg.norm(q))
        nerr = abs(total - float(g["l2"])) / float(g["l2"])
        # per element and field: norm and weighted sum, relative to the
        # element's own largest field norm (fields far below it are noise
        # next to its round-off)
        qk = q[keep]
        scale = norms.max(axis=1, keepdims=True)
        dn = np.abs(np.linalg.norm(qk, axis=2) - norms) / scale
        dw = np.abs((qk * wts).sum(axis=2) - wsums) / (scale * np.sqrt(len(wts)))
        say("  shape %s: %d elements in full, rel L2 %.3e, full-norm diff %.3e, "
            "worst per-element norm %.3e and weighted-sum %.3e over %d elements, "
            "largest elsewhere %.3e of the maximum"
            % (shape, len(full), err, nerr, dn.max(), dw.max(), len(keep), rest_max / gmax))
        assert rest_max <= 1e-12 * gmax
        if prec == 64:
            assert err <= 1e-12
            assert nerr <= 1e-12
            assert dn.max() <= 1e-10 and dw.max() <= 1e-10
            tref = g["traces"]
            assert np.abs(tr - tref).max() <= 1e-12 * np.abs(tref).max() + 1e-300
        else:
            assert err <= 1e-5


def test_c3_traces_over_1500_steps():
    g = _load("c3_traces_1500steps.npz")
    w = W.build_workload("c3_adjoint")
    tref = g["traces"]
    peak = np.abs(tref).max(axis=(1, 2))
    live = np.nonzero(peak >= 1e-3 * peak.max())[0]
    sample = g["sample_elements"]
    for prec in (64, 32):
        say("case c3 1500 steps, precision %d" % prec)
        q, tr, shape = _run(w, g["dt"], prec, int(g["steps"]))
        err = rel_l2(tr, tref)
        worst = max(rel_l2(tr[r], tref[r]) for r in live)
        ferr = rel_l2(q[sample], g["sample_fields"])
        nerr = abs(float(np.linalg.norm(q)) - float(g["l2"])) / float(g["l2"])
        say("  shape %s: traces rel L2 %.3e, worst of %d live receivers %.3e, "
            "sampled fields %.3e, full-norm diff %.3e" % (shape, err, len(live), worst,
                                                          ferr, nerr))
        if prec == 64:
            assert err <= 1e-12
            assert worst <= 1e-12
            assert ferr <= 1e-12
            assert nerr <= 1e-12
        else:
            assert err <= 1e-4
            assert ferr <= 1e-4

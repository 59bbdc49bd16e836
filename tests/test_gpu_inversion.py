"""The inversion loop on the GPU.

* Parity: three L-BFGS iterations (lambda and mu inverted, two shots) driven
  by the library's batched forward and adjoint follow the oracle's inversion
  (its own L-BFGS over its reverse-mode gradients) on the same seeded
  problem: misfit history to 1e-10 and model to 1e-9, relative.
* On a reduced version of the adjoint workload (1296 elements, order 3,
  four shots, layered truth, blob-perturbed start) the misfit falls
  monotonically, in FP64 and FP32.
"""

import numpy as np
import pytest

import workloads as W
from oracle import inversion as OI
from paper_2205_11052_amd import Solver
from paper_2205_11052_amd.inversion import invert
from gpu_helpers import say
from test_inversion import tiny_inversion_problem

pytestmark = pytest.mark.gpu


def test_inversion_matches_oracle():
    T = tiny_inversion_problem(N=2, nsteps=60)
    say("case inversion parity K=%d N=%d shots=%d" % (T["K"], T["N"], len(T["shots"])))
    s = Solver(T["N"], 64, len(T["shots"]))
    s.set_mesh_dict(T["mesh"])
    s.set_material(*T["start"])
    s.set_dt(T["dt"])
    for i, (pos, f0, t0, amp, moment) in enumerate(T["shots"]):
        s.set_source(i, pos, f0, t0, amp, moment=moment)
        s.set_receivers(i, T["rec"], T["nsteps"])
    model, hist, obj = invert(s, T["d_obs"], T["nsteps"], 20, T["start"], 3,
                              which=("lam", "mu"))
    fg = OI.shots_objective(T["P"], T["shots"], T["d_obs"], T["start"], (1, 2),
                            T["dt"], T["nsteps"], 20)
    x_o, h_o = OI.minimise(fg, np.zeros(2 * T["K"]), 3)
    f_gpu = [h["f"] for h in hist]
    say("inversion misfits gpu %s oracle %s" % (f_gpu, h_o))
    assert len(f_gpu) == len(h_o) == 4
    for a, b in zip(f_gpu, h_o):
        assert abs(a - b) <= 1e-10 * abs(b)
    K = T["K"]
    for c in (1, 2):
        ref = T["start"][c] * (1.0 + np.asarray(x_o[(c - 1) * K:c * K]))
        err = np.max(np.abs(model[c] - ref)) / np.max(np.abs(ref))
        say("component %d model rel diff %.3e" % (c, err))
        assert err <= 1e-9
    assert np.array_equal(model[0], T["start"][0])   # rho held
    assert all(b < a for a, b in zip(f_gpu, f_gpu[1:]))


@pytest.mark.parametrize("prec", [64, 32])
def test_inversion_lowers_misfit_reduced_adjoint_workload(prec):
    wt = W.build_workload("c3_adjoint", n=6)
    ws = W.build_workload("c3_adjoint", n=6, medium="blob")
    shots = [np.array([2.5 + 5 * i, 2.5 + 5 * j, 9.1]) for i in (0, 1) for j in (0, 1)]
    nsteps = 300
    say("case inversion reduced c3 fp%d K=%d" % (prec, wt["K"]))
    st = Solver(wt["N"], 64, len(shots))
    st.set_mesh_dict(wt["mesh"])
    st.set_material(wt["rho"], wt["lam"], wt["mu"])
    dt = st.suggest_dt(wt["cfl"])
    st.set_dt(dt)
    for i, pos in enumerate(shots):
        st.set_source(i, pos, wt["f0"], wt["t0"], wt["amp"])
        st.set_receivers(i, wt["receivers"], nsteps)
    st.zero_fields()
    st.step(nsteps)
    d_obs = np.stack([st.read_traces(i) for i in range(len(shots))])
    st.close()
    s = Solver(ws["N"], prec, len(shots))
    s.set_mesh_dict(ws["mesh"])
    s.set_material(ws["rho"], ws["lam"], ws["mu"])
    s.set_dt(dt)
    for i, pos in enumerate(shots):
        s.set_source(i, pos, ws["f0"], ws["t0"], ws["amp"])
        s.set_receivers(i, ws["receivers"], nsteps)
    model, hist, obj = invert(s, d_obs, nsteps, 100,
                              (ws["rho"], ws["lam"], ws["mu"]), 4)
    f = [h["f"] for h in hist]
    say("fp%d misfits %s (evaluations %d, gradients %d)" % (prec, f, obj.evaluations,
                                                           obj.gradients))
    assert len(f) == 5
    assert all(b < a for a, b in zip(f, f[1:]))
    assert f[-1] < 0.8 * f[0]

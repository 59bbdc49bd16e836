"""GPU parity of the forward solver (FP64 and FP32) against the CPU oracle.

All calls go through the C ABI (libdgw.so) via the ctypes binding.  Bars:
FP64 relative L2 <= 1e-12, FP32 relative L2 <= 1e-5 against the FP64 oracle
on the same seeded inputs.
"""

import functools

import numpy as np
import pytest
import torch

import workloads as W
from paper_2205_11052_amd.dgw import DGWError
from gpu_helpers import (gpu_solver, oracle_problem, oracle_run, rel_l2,
                         random_fields, say)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def _random_medium(K, seed):
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    cs = cp / rng.uniform(1.5, 2.2, K)
    rho = rng.uniform(1.0, 3.0, K)
    return W.lame_from_velocities(cp, cs, rho)


def test_c0_periodic_plane_wave_fp64():
    w = W.build_workload("c0_periodic_pwave")
    say("case c0_periodic_pwave fp64 K=%d N=%d" % (w["K"], w["N"]))
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt)
    assert abs(s.suggest_dt(w["cfl"]) - dt) <= 1e-14 * dt
    s.set_fields(0, w["q0"])
    s.step(w["steps"])
    q_gpu = s.get_fields(0)
    q_ora, _ = oracle_run(P, w["q0"], w["rho"], w["lam"], w["mu"], dt,
                          w["steps"])
    err = rel_l2(q_gpu, q_ora)
    say("c0 fp64 rel L2 vs oracle", err)
    assert err <= FP64_TOL
    # discrete energy on the device equals the oracle's
    from oracle import solver as O
    t = lambda a: torch.as_tensor(np.asarray(a))
    e_ora = O.energy(P, t(q_ora), t(w["rho"]), t(w["lam"]), t(w["mu"])).item()
    assert abs(s.energy(0) - e_ora) <= 1e-13 * e_ora
    s.check_finite()


# stage kernel variants: 0 = one thread per node on the vector ALUs,
# 1 = volume and lift as one GEMM on the matrix cores, 2 = the minimal-form
# matrix-core kernel (orders 1-4 in FP64, 1-6 in FP32; 32 elements per
# work-group, no persistent grid)
KERNELS = (0, 1, 2)


def supported(kernel, N, precision=64):
    return kernel != 2 or N <= (4 if precision == 64 else 6)


@pytest.mark.parametrize("N,kernel", [(N, kv) for kv in KERNELS for N in range(1, 7)
                                      if supported(kv, N)])
def test_all_orders_all_boundaries_fp64(N, kernel):
    mesh = W.kuhn_cube(2, 1.0)          # free-surface top, absorbing sides
    K = mesh["etov"].shape[0]
    rho, lam, mu = _random_medium(K, 100 + N)
    say("case orders fp64 N=%d K=%d kernel=%d" % (N, K, kernel))
    P = oracle_problem(mesh, N)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    q0 = random_fields(K, P.Np, 200 + N)
    src = np.array([0.37, 0.52, 0.61])
    moment = (1.0, -0.5, 0.25, 0.3, -0.2, 0.1)
    rec = np.array([[0.2, 0.3, 1.0], [0.8, 0.6, 0.5], [0.1, 0.9, 0.0]])
    P.set_source(src, 3.0, 0.1, 2.0, moment=moment)
    P.set_receivers(rec)
    s = gpu_solver(mesh, N, rho, lam, mu, dt, kernel=kernel)
    s.set_source(0, src, 3.0, 0.1, 2.0, moment=moment)
    s.set_receivers(0, rec, 16)
    s.set_fields(0, q0)
    nst = 7
    s.step(nst)
    q_ora, tr_ora = oracle_run(P, q0, rho, lam, mu, dt, nst, record=True)
    err = rel_l2(s.get_fields(0), q_ora)
    terr = rel_l2(s.read_traces(0), tr_ora)
    say("N=%d fields %.3e traces %.3e" % (N, err, terr))
    assert err <= FP64_TOL and terr <= FP64_TOL
    assert s.shot_steps(0) == nst


def _reduced_c1(n=6, N=4, t0=0.35):
    w = W.build_workload("c1_layered_n24", n=n, N=N)
    w["t0"] = t0
    return w


def test_reduced_layered_source_receivers_fp64():
    w = _reduced_c1()
    say("case reduced c1 fp64 K=%d" % w["K"])
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    P.set_source(w["source"], w["f0"], w["t0"], w["amp"])
    P.set_receivers(w["receivers"])
    nst = 40
    s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt)
    s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
    s.set_receivers(0, w["receivers"], nst)
    s.step(nst)
    q_ora, tr_ora = oracle_run(P, np.zeros((w["K"], 9, P.Np)), w["rho"],
                               w["lam"], w["mu"], dt, nst, record=True)
    err = rel_l2(s.get_fields(0), q_ora)
    tr = s.read_traces(0)
    terr = np.abs(tr - tr_ora).max() / np.abs(tr_ora).max()
    say("reduced c1 fields %.3e traces %.3e" % (err, terr))
    assert np.abs(q_ora).max() > 0 and np.abs(tr_ora).max() > 0
    assert err <= FP64_TOL and terr <= FP64_TOL


@functools.lru_cache(maxsize=1)
def _full_c1_oracle():
    """The full 82944-element order-4 mesh with random fields everywhere
    (every face type and element exercised), source and receivers active:
    two oracle steps, shared by the full-size tests."""
    w = W.build_workload("c1_layered_n24")
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    P.set_source(w["source"], w["f0"], 0.05, w["amp"])
    P.set_receivers(w["receivers"])
    q0 = random_fields(w["K"], P.Np, 7)
    q_ora, tr_ora = oracle_run(P, q0, w["rho"], w["lam"], w["mu"], dt, 2,
                               record=True)
    return w, dt, q0, q_ora, tr_ora


def test_full_size_layered_fp64_bench_launch():
    """Full 82944-element mesh at order 4 in every launch shape the
    benchmark's autotuner can pick, two steps against the oracle."""
    w, dt, q0, q_ora, tr_ora = _full_c1_oracle()
    say("case full c1 fp64 K=%d" % w["K"])
    shapes = [(kv, be, wpc) for kv in (0, 1) for be in (7, 3)
              for wpc in (0, 1, 2, 3, 4, 8, 16)] + [(2, 32, 0)]
    s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt)
    s.set_source(0, w["source"], w["f0"], 0.05, w["amp"])
    s.set_receivers(0, w["receivers"], 8)
    for shape in shapes:
        s.set_launch(*shape)
        s.set_fields(0, q0)
        s.step(2)
        err = rel_l2(s.get_fields(0), q_ora)
        terr = rel_l2(s.read_traces(0), tr_ora)
        say("full c1 shape %s fields %.3e traces %.3e" % (shape, err, terr))
        assert err <= FP64_TOL and terr <= FP64_TOL


@pytest.mark.parametrize("kernel", KERNELS)
def test_full_size_layered_fp32_bench_launch(kernel):
    """The FP32 form on the full 82944-element order-4 mesh in the shapes
    the benchmark times, against the FP64 oracle."""
    w, dt, q0, q_ora, tr_ora = _full_c1_oracle()
    say("case full c1 fp32 kernel=%d" % kernel)
    s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt, 32)
    s.set_source(0, w["source"], w["f0"], 0.05, w["amp"])
    s.set_receivers(0, w["receivers"], 8)
    # the FP32 block choices: kernel 0 (7, 3), kernel 1 (14, 7: two column
    # tiles per wave, then one), kernel 2 (32)
    for be in {0: (7, 3), 1: (14, 7), 2: (32,)}[kernel]:
        s.set_launch(kernel, be, 0)
        s.set_fields(0, q0)
        s.step(2)
        err = rel_l2(s.get_fields(0), q_ora)
        terr = rel_l2(s.read_traces(0), tr_ora)
        say("full c1 fp32 kernel %d be %d fields %.3e traces %.3e" % (kernel, be, err, terr))
        assert err <= FP32_TOL and terr <= FP32_TOL


@pytest.mark.parametrize("N", [5, 6])
def test_order5_6_fp64_matrix_core_shapes(N):
    """Orders 5 and 6 in FP64, where the matrix-core variant loads its
    operator fragments through a register ring: every block size and a
    persistent grid give bitwise the same fields, which match the oracle to
    the FP64 bar."""
    mesh = W.kuhn_cube(2, 1.0)
    K = mesh["etov"].shape[0]
    rho, lam, mu = _random_medium(K, 300 + N)
    P = oracle_problem(mesh, N)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    q0 = random_fields(K, P.Np, 400 + N)
    q_ora, _ = oracle_run(P, q0, rho, lam, mu, dt, 4)
    blocks = {5: (6, 3), 6: (4, 2)}[N]
    outs = []
    for be in blocks:
        for wpc in (0, 2):
            say("case order %d fp64 matrix-core shape (1, %d, %d)" % (N, be, wpc))
            s = gpu_solver(mesh, N, rho, lam, mu, dt)
            s.set_launch(1, be, wpc)
            s.set_fields(0, q0)
            s.step(4)
            outs.append(s.get_fields(0))
            s.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    err = rel_l2(outs[0], q_ora)
    say("order %d matrix-core fields vs oracle %.3e" % (N, err))
    assert err <= FP64_TOL


def test_full_size_order6_variants_agree_and_dissipate():
    """Order 6 (84 nodes) on the full 82944-element mesh, where the oracle
    is too slow for a full run: the two kernel variants agree to the FP64
    bar, the discrete energy does not grow over the steps (no source; the
    upwind flux and the absorbing and free-surface boundaries only
    dissipate; checked in FP64), and FP32 agrees with FP64 to the FP32
    bar.  Oracle parity
    at order 6 is covered on smaller meshes."""
    w = W.build_workload("c1_layered_n24", N=6)
    say("case full order 6 K=%d" % w["K"])
    q0 = random_fields(w["K"], 84, 17)
    dt = None
    outs = {}
    for prec, kernel in ((64, 0), (64, 1), (32, 1)):
        from paper_2205_11052_amd import Solver
        s = Solver(6, prec, 1)
        s.set_mesh_dict(w["mesh"])
        s.set_material(w["rho"], w["lam"], w["mu"])
        if dt is None:
            dt = s.suggest_dt(w["cfl"])
        s.set_dt(dt)
        s.set_launch(kernel)
        s.set_fields(0, q0)
        e = [s.energy(0)]
        for _ in range(3):
            s.step(1)
            e.append(s.energy(0))
        outs[(prec, kernel)] = s.get_fields(0)
        say("order 6 fp%d kernel %d energies %s" % (prec, kernel, e))
        if prec == 64:
            for a, b in zip(e[:-1], e[1:]):
                assert b <= a * (1 + 1e-10)
        s.close()
    assert rel_l2(outs[(64, 1)], outs[(64, 0)]) <= FP64_TOL
    assert rel_l2(outs[(32, 1)], outs[(64, 0)]) <= FP32_TOL


def test_full_size_batched_32_shots():
    """The benchmark's batched form at full size: 32 FP32 shots of uneven
    length on the 82944-element mesh, one launch per stage over all shots;
    the first and last shots equal single-shot runs bitwise."""
    w = W.build_workload("c1_layered_n24")
    pos, lens = W.batched_shots()
    lens = np.minimum(lens, 4)
    lens[0] = 2                         # one shot stops early
    say("case full batched 32 shots")
    from paper_2205_11052_amd import Solver
    b = Solver(4, 32, len(pos))
    b.set_mesh_dict(w["mesh"])
    b.set_material(w["rho"], w["lam"], w["mu"])
    dt = b.suggest_dt(w["cfl"])
    b.set_dt(dt)
    for i in range(len(pos)):
        b.set_source(i, pos[i], w["f0"], w["t0"], w["amp"], nsteps=int(lens[i]))
        b.set_receivers(i, w["receivers"], 8)
    b.set_launch(1, 7, 0)
    b.step(4)
    for i in (0, len(pos) - 1):
        assert b.shot_steps(i) == lens[i]
        one = Solver(4, 32, 1)
        one.set_mesh_dict(w["mesh"])
        one.set_material(w["rho"], w["lam"], w["mu"])
        one.set_dt(dt)
        one.set_source(0, pos[i], w["f0"], w["t0"], w["amp"], nsteps=int(lens[i]))
        one.set_receivers(0, w["receivers"], 8)
        one.set_launch(1, 7, 0)
        one.step(4)
        assert np.array_equal(b.get_fields(i), one.get_fields(0))
        assert np.array_equal(b.read_traces(i), one.read_traces(0))
        one.close()
    b.close()


@pytest.mark.parametrize("kernel", KERNELS)
def test_fp32_error_against_fp64_oracle(kernel):
    w = W.build_workload("c0_periodic_pwave")
    say("case c0 fp32 kernel=%d" % kernel)
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt, 32,
                   kernel=kernel)
    s.set_fields(0, w["q0"])
    s.step(w["steps"])
    q_ora, _ = oracle_run(P, w["q0"], w["rho"], w["lam"], w["mu"], dt,
                          w["steps"])
    err = rel_l2(s.get_fields(0), q_ora)
    say("c0 fp32 rel L2 vs fp64 oracle %.3e" % err)
    assert err <= FP32_TOL


@pytest.mark.parametrize("N,kernel", [(N, kv) for kv in KERNELS for N in (4, 6)
                                      if supported(kv, N, 32)])
def test_fp32_reduced_layered(N, kernel):
    w = _reduced_c1(n=4, N=N)
    say("case reduced c2 fp32 N=%d K=%d kernel=%d" % (N, w["K"], kernel))
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    P.set_source(w["source"], w["f0"], w["t0"], w["amp"])
    P.set_receivers(w["receivers"])
    q0 = random_fields(w["K"], P.Np, 31)
    nst = 10
    s = gpu_solver(w["mesh"], N, w["rho"], w["lam"], w["mu"], dt, 32,
                   kernel=kernel)
    s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
    s.set_receivers(0, w["receivers"], nst)
    s.set_fields(0, q0)
    s.step(nst)
    q_ora, tr_ora = oracle_run(P, q0, w["rho"], w["lam"], w["mu"], dt, nst,
                               record=True)
    err = rel_l2(s.get_fields(0), q_ora)
    terr = rel_l2(s.read_traces(0), tr_ora)
    say("fp32 N=%d fields %.3e traces %.3e" % (N, err, terr))
    assert err <= FP32_TOL and terr <= FP32_TOL


def test_graph_replay_equals_eager_and_block_shapes_agree():
    w = _reduced_c1(n=4)
    say("case graph vs eager")
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
    q0 = random_fields(w["K"], P.Np, 5)
    outs = []
    shapes = ((False, 0, 0, 0), (True, 0, 0, 0), (False, 0, 3, 0),
              (False, 0, 7, 4), (False, 0, 3, 1))
    mma_shapes = ((False, 1, 0, 0), (True, 1, 0, 0), (False, 1, 3, 2))
    for timing, kernel, block, wpc in shapes:
        s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt)
        s.set_launch(kernel, block, wpc)
        s.enable_timing(timing)
        s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
        s.set_fields(0, q0)
        s.step(23)
        outs.append(s.get_fields(0))
        if timing:
            ms, n = s.stage_kernel_ms()
            assert n == 5 * 23 and ms > 0
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    # the matrix-core variant: bitwise stable over its own shapes and
    # graph/eager, equal to variant 0 to rounding
    mouts = []
    for timing, kernel, block, wpc in mma_shapes:
        s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt)
        s.set_launch(kernel, block, wpc)
        s.enable_timing(timing)
        s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
        s.set_fields(0, q0)
        s.step(23)
        mouts.append(s.get_fields(0))
    for o in mouts[1:]:
        assert np.array_equal(mouts[0], o)
    assert rel_l2(mouts[0], outs[0]) <= FP64_TOL
    # the minimal-form kernel: graph replay equals eager bitwise, and it
    # equals variant 0 to rounding
    souts = []
    for timing in (False, True):
        s = gpu_solver(w["mesh"], w["N"], w["rho"], w["lam"], w["mu"], dt)
        s.set_launch(2, 32, 0)
        s.enable_timing(timing)
        s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
        s.set_fields(0, q0)
        s.step(23)
        souts.append(s.get_fields(0))
    assert np.array_equal(souts[0], souts[1])
    assert rel_l2(souts[0], outs[0]) <= FP64_TOL
    # a kernel variant or shape this build does not provide is refused
    for bad in ((3, 0, 0), (0, 5, 0), (1, 5, 0), (0, 7, 65), (2, 7, 0), (2, 32, 2)):
        with pytest.raises(DGWError) as ei:
            s.set_launch(*bad)
        assert ei.value.status == "DGW_EINVAL"


@pytest.mark.parametrize("precision,kernel", [(p, kv) for kv in KERNELS for p in (64, 32)])
def test_batched_shots_match_single_shot_runs(precision, kernel):
    mesh = W.kuhn_cube(3, 1.0)
    K = mesh["etov"].shape[0]
    rho, lam, mu = _random_medium(K, 3)
    N = 3
    dt = 0.5 * 2 * (1 / 3) / (2 * (1 + np.sqrt(2))) / np.sqrt(
        np.max((lam + 2 * mu) / rho)) / 16
    srcs = np.array([[0.2, 0.3, 0.4], [0.7, 0.6, 0.5], [0.5, 0.5, 0.9]])
    lens = [7, 12, 3]
    rec = np.array([[0.4, 0.4, 1.0], [0.6, 0.2, 1.0]])
    say("case batched shots precision=%d kernel=%d" % (precision, kernel))
    b = gpu_solver(mesh, N, rho, lam, mu, dt, precision, nshots=3)
    # persistent grid looping over (shot, block) items (kernel 2: one
    # work-group per (shot, block) item)
    b.set_launch(kernel, 0, 2 if kernel < 2 else 0)
    for i in range(3):
        b.set_source(i, srcs[i], 6.0, 0.1, 1.0, nsteps=lens[i])
        b.set_receivers(i, rec, 20)
    b.step(15)
    for i in range(3):
        assert b.shot_steps(i) == lens[i]
        one = gpu_solver(mesh, N, rho, lam, mu, dt, precision, kernel=kernel)
        one.set_source(0, srcs[i], 6.0, 0.1, 1.0, nsteps=lens[i])
        one.set_receivers(0, rec, 20)
        one.step(15)
        assert np.array_equal(b.get_fields(i), one.get_fields(0))
        tb, to = b.read_traces(i), one.read_traces(0)
        assert tb.shape == (2, 3, lens[i]) and np.array_equal(tb, to)
    # a shot extended after it stopped resumes from its own state
    b.set_source(2, srcs[2], 6.0, 0.1, 1.0, nsteps=5)
    b.step(2)
    assert b.shot_steps(2) == 5 and b.shot_steps(0) == 7


@pytest.mark.parametrize("kernel", KERNELS)
def test_compacted_batch_with_graph_replays(kernel):
    """Shots of lengths 5, 27 and 40 in one 40-step call: after step 5 the
    launches cover two shots, after step 27 one (each segment long enough
    for captured-graph replays of its own active set); every shot equals its
    single-shot run bitwise."""
    if not supported(kernel, 3, 64):
        pytest.skip("kernel not built for this order")
    mesh = W.kuhn_cube(3, 1.0)
    K = mesh["etov"].shape[0]
    rho, lam, mu = _random_medium(K, 21)
    N = 3
    P = oracle_problem(mesh, N)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    srcs = np.array([[0.2, 0.3, 0.4], [0.7, 0.6, 0.5], [0.5, 0.5, 0.9]])
    lens = [5, 27, 40]
    rec = np.array([[0.4, 0.4, 1.0], [0.6, 0.2, 1.0]])
    say("case compacted batch kernel=%d" % kernel)
    b = gpu_solver(mesh, N, rho, lam, mu, dt, 64, nshots=3, kernel=kernel)
    q0 = [random_fields(K, P.Np, 70 + i) for i in range(3)]
    for i in range(3):
        b.set_source(i, srcs[i], 6.0, 0.1, 1.0, nsteps=lens[i])
        b.set_receivers(i, rec, 40)
        b.set_fields(i, q0[i])
    b.step(40)
    for i in range(3):
        assert b.shot_steps(i) == lens[i]
        one = gpu_solver(mesh, N, rho, lam, mu, dt, 64, kernel=kernel)
        one.set_source(0, srcs[i], 6.0, 0.1, 1.0, nsteps=lens[i])
        one.set_receivers(0, rec, 40)
        one.set_fields(0, q0[i])
        one.step(40)
        assert np.array_equal(b.get_fields(i), one.get_fields(0))
        assert np.array_equal(b.read_traces(i), one.read_traces(0))
        one.close()
    b.close()


def test_resume_at_own_time():
    """A source-driven run saved at step 12 and resumed there
    (dgw_set_fields, then dgw_set_shot_step) continues exactly as the
    uninterrupted run: fields and the traces from step 12 on, bitwise."""
    mesh = W.kuhn_cube(3, 1.0)
    K = mesh["etov"].shape[0]
    rho, lam, mu = _random_medium(K, 31)
    N = 3
    P = oracle_problem(mesh, N)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    src, rec = np.array([0.4, 0.45, 0.55]), np.array([[0.3, 0.6, 1.0], [0.7, 0.2, 0.5]])
    say("case resume")

    def solver():
        s = gpu_solver(mesh, N, rho, lam, mu, dt, 64, kernel=1)
        s.set_source(0, src, 8.0, 0.05, 1.0, nsteps=30)
        s.set_receivers(0, rec, 30)
        s.zero_fields()
        return s

    a = solver()
    a.step(20)
    b = solver()
    b.step(12)
    q12 = b.get_fields(0)
    b.close()
    c = solver()
    c.set_fields(0, q12)
    c.set_shot_step(0, 12)
    c.step(8)
    assert c.shot_steps(0) == 20
    assert np.array_equal(c.get_fields(0), a.get_fields(0))
    ta, tc = a.read_traces(0), c.read_traces(0)
    assert np.array_equal(tc[:, :, 12:20], ta[:, :, 12:20])
    assert not tc[:, :, :12].any()
    for bad in (-1, 31):
        with pytest.raises(DGWError) as e:
            c.set_shot_step(0, bad)
        assert e.value.code == -6
    a.close()
    c.close()


def test_tiny_mesh_smaller_than_a_block_and_zero_steps():
    mesh = W.kuhn_cube(1, 1.0)
    K = mesh["etov"].shape[0]
    rho, lam, mu = _random_medium(K, 8)
    say("case tiny mesh")
    for N, kernel in ((1, 0), (4, 0), (1, 2), (4, 2)):
        P = oracle_problem(mesh, N)
        dt = P.suggest_dt(rho, lam, mu, 0.5)
        q0 = random_fields(K, P.Np, 9)
        s = gpu_solver(mesh, N, rho, lam, mu, dt, kernel=kernel)
        s.set_fields(0, q0)
        s.step(0)
        assert np.array_equal(s.get_fields(0), q0)
        s.step(3)
        q_ora, _ = oracle_run(P, q0, rho, lam, mu, dt, 3)
        assert rel_l2(s.get_fields(0), q_ora) <= FP64_TOL

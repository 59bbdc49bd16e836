"""Benchmark of the fused nodal-DG elastic RHS + LSERK4 stage on one MI355X.

Workload (the headline configuration): the [0,10]^3 cube split into
6*24^3 = 82944 tetrahedra, order 4 (35 nodes, 9 fields = 26,127,360 DOF),
FP64, layered noisy medium, free-surface top and absorbing sides, explosive
Ricker point source and 64 surface receivers.  One "step" is one LSERK4 time
step: five fused stage launches plus one receiver-sampling launch.  Fields are
resident in HBM before the timed region; the timed region replays captured
HIP graphs on a torch stream bracketed by torch.cuda.synchronize() and HIP
events.

Metric: GDOF-stage/s = 9 * Np * K * 5 * steps / seconds / 1e9.

Timing: W warm-up steps, then one graph's worth of steps (so the captured
graph is built and replayed once before any window), then 5 windows of K
steps; the median window gives `value` and `ms_per_step`.

Extra forms reported beside the headline (same GPU, same mesh and medium):
FP32 fields and arithmetic, a batch of 32 FP32 shots advanced together, and
order 6 in FP64 and FP32.  The FP32 error against the FP64 run is stated on
the receiver traces and the final fields after the full 2000 steps from
zero fields.  The adjoint form
reports seconds per shot of the misfit gradient on the 24576-element order-3
workload, with its error against central differences measured in the run.

Roofline: the stage kernel's algorithmic HBM bytes per launch (read q and
res, write res and q', read the per-element data and connectivity) divided by
its average launch duration, timed with HIP events around each launch on the
library's stream, against 8 TB/s.  "traffic" is the HBM bytes per launch the
hardware counters measured for this kernel source and launch shape (null
when either differs).

The roofline also states the algorithmic FLOP rate (minimal operation
count per element, `stage_flops`) against the FP64 peak of 78.6 TFLOP/s.

CPU baseline: the CPU oracle (plain PyTorch FP64) on one pinned host core,
timed on a bounded sample of the same workload (one LSERK4 step of the full
mesh), with the CPU model and the host's core count.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--no-forms] [--no-adjoint] [--shape K,E,W]
                       [--copy-probe]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
META_BYTES = 48 * 8 + 4 * 4        # per-element data + packed connectivity
ANI_BYTES = 120 * 8                # anisotropic per-element data (DGW_ANI doubles)


# HBM traffic of the order-4 FP64 stage kernel on this workload, measured
# with rocprofv3 (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the
# factors a plain 1 GiB copy gives for the same counters: 2.0 and 1.0).  It
# is reported only while the kernel source hashes to the value it was
# measured for and the same launch shape runs; otherwise traffic is null.
MEASURED_TRAFFIC = {
    "kernel_source_sha256": "15ccbb7cd79ebddaf7cbef16a22f6fb1a79ea6045fe05cdc11048a4db2d08f6f",
    "launch_shape": (1, 7, 0),
    "bytes_per_launch": 983367987,
}


def measured_traffic(shape):
    m = MEASURED_TRAFFIC
    if kernel_source_sha() != m["kernel_source_sha256"] or tuple(shape) != m["launch_shape"]:
        return None
    return m["bytes_per_launch"]


# Matrix-pipe and vector-ALU busy fractions of the same kernel, from
# rocprofv3 counters (SQ_VALU_MFMA_BUSY_CYCLES and SQ_ACTIVE_INST_VALU over
# SQ_BUSY_CYCLES x SIMDs), reported under the same source-hash and
# launch-shape condition as the traffic.
MEASURED_COUNTERS = {
    "kernel_source_sha256": MEASURED_TRAFFIC["kernel_source_sha256"],
    "launch_shape": MEASURED_TRAFFIC["launch_shape"],
    "values": {"mfma_busy": 0.446, "valu_busy": 0.211, "wave_wait_frac": 0.268},
}


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("stage.hip", "stage_common.h", "dgw_internal.h"):
        with open(os.path.join(ROOT, "paper_2205_11052_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_counters(shape):
    m = MEASURED_COUNTERS
    if kernel_source_sha() != m["kernel_source_sha256"] or tuple(shape) != m["launch_shape"]:
        return None
    return dict(m["values"])


FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
FULL_STEPS = 2000      # the full run length of the order-4 and order-6 workloads


def stage_flops(K, N, nshots=1):
    """Algorithmic floating-point operations of one stage launch, minimal
    form per element: 18 reference matrix-vector products (9 for the stress
    divergence, 9 for the velocity gradient), 6 lifted components per face,
    about 150 operations per face node for the Riemann solve, and the RK
    update (2 operations per value per register)."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    per = 2 * 18 * Np * Np + 2 * 6 * 4 * Np * Nfp + 150 * 4 * Nfp + 4 * 9 * Np
    return nshots * K * per


def full_length_run(s, nsteps):
    """Run shot 0 from zero fields for nsteps steps; traces and final fields."""
    s.zero_fields()
    s.step(nsteps)
    return {"traces": s.read_traces(0), "fields": s.get_fields(0), "steps": nsteps}


def full_length_errors(a, b):
    """Errors of run a against run b (traces over all receivers, components
    and samples; final fields over all nodal values)."""
    ta, tb = np.asarray(a["traces"]), np.asarray(b["traces"])
    fa, fb = np.asarray(a["fields"]), np.asarray(b["fields"])
    peak = np.abs(tb).max(axis=(1, 2))
    live = peak >= 1e-3 * peak.max()
    per_rec = [float(np.linalg.norm(ta[r] - tb[r]) / np.linalg.norm(tb[r]))
               for r in np.nonzero(live)[0]]
    return {"steps": b["steps"],
            "traces_rel_l2": rel_l2(ta, tb),
            "traces_worst_receiver_rel_l2": max(per_rec),
            "receivers_compared": len(per_rec),
            "fields_rel_l2": rel_l2(fa, fb),
            "fields_per_component_rel_l2": [rel_l2(fa[:, c], fb[:, c]) for c in range(9)],
            "fields_max_abs_err_over_max": float(np.abs(fa - fb).max() / np.abs(fb).max()),
            "note": "both runs from zero fields with the source active, same dt; "
                    "per-receiver error over receivers whose peak is >= 1e-3 of "
                    "the largest"}


def stage_bytes(K, Np, real_bytes, nshots=1):
    """Algorithmic HBM bytes of one stage launch: q and res read, res and q'
    written (4 field streams), per-element data and connectivity read once."""
    return nshots * K * 4 * 9 * Np * real_bytes + K * META_BYTES


def build_solver(w, precision, nshots=1, stream=None, shots=None, shape=None):
    from paper_2205_11052_amd import Solver
    s = Solver(w["N"], precision, nshots, stream=stream)
    s.set_mesh_dict(w["mesh"])
    s.set_material(w["rho"], w["lam"], w["mu"])
    dt = s.suggest_dt(w["cfl"])
    s.set_dt(dt)
    for i in range(nshots):
        pos = w["source"] if shots is None else shots[0][i]
        n = 0 if shots is None else int(shots[1][i])
        s.set_source(i, pos, w["f0"], w["t0"], w["amp"], nsteps=n)
        s.set_receivers(i, w["receivers"], 4096)
    # launch shape (elements per work-group, persistent grid): given, or
    # chosen by the library's autotuner on this very workload
    if shape is None:
        s.shape = s.autotune()
    else:
        s.set_launch(*shape)
        s.shape = tuple(shape)
    return s


def copy_probe(torch, nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size (reads and writes nbytes
    per launch); profiling it calibrates the HBM byte counters."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": nbytes, "launches": reps}),
          flush=True)


_T0 = time.perf_counter()


def progress(msg):
    """One progress line on stderr (the JSON result goes to stdout)."""
    print("[bench %7.1f s] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr,
          flush=True)


GRAPH_STEPS = 10      # steps per captured HIP graph in the library
REPEATS = 5           # timed windows; the median is reported


def timed_steps(torch, s, stream, steps, warmup, repeats=REPEATS):
    """Seconds for `steps` steps: the median of `repeats` windows, each timed
    with events on the solver's stream.  Before timing, `warmup` steps run
    and then one more graph's worth of steps, so the graph the timed windows
    replay is already captured, instantiated and replayed once (its capture
    is never inside a window).  Returns (median seconds, all window seconds)."""
    s.step(warmup)
    s.step(GRAPH_STEPS)
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        s.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        times.append(t0.elapsed_time(t1) / 1000.0)
    return float(np.median(times)), times


def kernel_avg_ms(s, steps=10):
    s.enable_timing(True)
    s.step(steps)
    ms, n = s.stage_kernel_ms()
    s.enable_timing(False)
    return ms, n


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def adjoint_form(torch, stream, nsteps=1500, ckpt=100, n_fd=2):
    """Gradient of the receiver misfit with respect to per-element rho,
    lambda, mu on the 24576-element order-3 workload (layered true medium,
    blob-perturbed start, dt fixed from the true medium), 1500 steps,
    checkpoint every 100 steps.  Seconds per shot = forward with checkpoints
    + reverse sweep, FP64 and FP32; the FP64 gradient is checked live against
    central differences of the FP64 forward (step 1e-6 relative) on n_fd
    seeded elements, all three parameters, and the FP32 gradient against the
    FP64 one."""
    import workloads as W
    from paper_2205_11052_amd import Solver
    wt = W.build_workload("c3_adjoint")
    ws = W.build_workload("c3_adjoint", medium="blob")

    def make(prec, w, dt=None):
        s = Solver(w["N"], prec, 1, stream=stream.cuda_stream)
        s.set_mesh_dict(w["mesh"])
        s.set_material(w["rho"], w["lam"], w["mu"])
        s.set_dt(dt if dt is not None else s.suggest_dt(w["cfl"]))
        s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
        s.set_receivers(0, w["receivers"], nsteps)
        s.autotune()
        return s

    with torch.cuda.stream(stream):
        st = make(64, wt)
        dt = st.dt
        st.zero_fields()
        st.step(nsteps)
        d = st.read_traces(0)[None]          # observed data [1][R][3][nsteps]
        st.close()
        res, grads = {}, {}
        for prec in (64, 32):
            s = make(prec, ws, dt)
            s.zero_fields()
            s.forward_checkpointed(nsteps, ckpt, d)      # warm-up
            s.adjoint()
            s.zero_fields()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mis = s.forward_checkpointed(nsteps, ckpt, d)
            g = s.adjoint()
            torch.cuda.synchronize()
            res["fp%d_s_per_shot" % prec] = round(time.perf_counter() - t0, 4)
            res["fp%d_misfit" % prec] = float(mis[0])
            grads[prec] = [x[0] for x in g]
            if prec == 64:
                s64 = s
            else:
                s.close()
        g = grads[64]
        gmax = max(np.abs(x).max() for x in g)
        eligible = np.nonzero(np.maximum.reduce([np.abs(x) for x in g])
                              >= 1e-3 * gmax)[0]
        elems = np.random.default_rng(52).choice(eligible, size=n_fd, replace=False)
        base = [np.array(ws["rho"]), np.array(ws["lam"]), np.array(ws["mu"])]
        worst, nfd = 0.0, 0
        for k in elems:
            for p in range(3):
                if abs(g[p][k]) < 1e-3 * gmax:
                    continue
                delta = 1e-6 * base[p][k]
                vals = []
                for sgn in (1, -1):
                    m = [b.copy() for b in base]
                    m[p][k] += sgn * delta
                    s64.set_material(*m)
                    s64.zero_fields()
                    vals.append(s64.forward_checkpointed(nsteps, nsteps, d)[0])
                fd = (vals[0] - vals[1]) / (2 * delta)
                worst = max(worst, abs(fd - g[p][k]) / abs(fd))
                nfd += 1
        s64.close()
    res["fd_max_rel_error_fp64"] = worst
    res["fd_entries"] = nfd
    res["kernels"] = adjoint_kernel_times(torch, stream, make, ws, dt, d)
    res["fp32_grad_rel_l2_vs_fp64"] = rel_l2(np.concatenate(grads[32]),
                                             np.concatenate(grads[64]))
    res["workload"] = ("c3_adjoint: 6*16^3 = 24576 tetrahedra, order 3, %d steps, "
                       "checkpoint every %d, one shot" % (nsteps, ckpt))
    return res


def adjoint_probe(torch, stream, nsteps=200, ckpt=100):
    """One gradient of the order-3 gradient workload (24576 tetrahedra) over
    a short window, FP64 then FP32, for counter runs of the reverse-sweep
    kernels: observed data from the true layered medium, gradient at the
    blob-perturbed start, checkpoints every 100 steps."""
    import workloads as W
    from paper_2205_11052_amd import Solver
    wt = W.build_workload("c3_adjoint")
    ws = W.build_workload("c3_adjoint", medium="blob")

    def make(prec, w, dt=None):
        s = Solver(w["N"], prec, 1, stream=stream.cuda_stream)
        s.set_mesh_dict(w["mesh"])
        s.set_material(w["rho"], w["lam"], w["mu"])
        s.set_dt(dt if dt is not None else s.suggest_dt(w["cfl"]))
        s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
        s.set_receivers(0, w["receivers"], nsteps)
        # the autotuner's picks for this workload, fixed for the counters
        if prec == 64:
            s.set_launch(1, 7, 0)
        else:
            s.set_launch(0, 12, 0)
        return s

    out = {"probe": "adjoint", "steps": nsteps, "checkpoint_every": ckpt}
    with torch.cuda.stream(stream):
        st = make(64, wt)
        dt = st.dt
        st.zero_fields()
        st.step(nsteps)
        d = st.read_traces(0)[None]
        st.close()
        for prec in (64, 32):
            s = make(prec, ws, dt)
            s.zero_fields()
            mis = s.forward_checkpointed(nsteps, ckpt, d)
            g = s.adjoint()
            out["fp%d_misfit" % prec] = float(mis[0])
            out["fp%d_grad_finite" % prec] = bool(all(np.isfinite(x).all() for x in g))
            s.close()
        torch.cuda.synchronize()
    return out


def reverse_stage_bytes(K, Np, real_bytes):
    """Algorithmic HBM bytes of one reverse (adjoint) stage: the stage input
    q read, the adjoint states lam_q and lam_r read and written, the
    per-element data and connectivity read, the FP64 gradient (3 values per
    element) read and written."""
    return K * (5 * 9 * Np * real_bytes + META_BYTES + 2 * 3 * 8)


# HBM traffic of one reverse stage of the order-3 gradient workload (the
# main kernel plus a fifth of a lift, per dispatch, calibrated FETCH_SIZE x
# 2.0 and WRITE_SIZE x 1.0, from `bench.py --adjoint-probe`), reported only
# while the reverse-sweep kernel source hashes to the value it was measured
# for.
MEASURED_ADJ_TRAFFIC = {
    "kernel_source_sha256": "1a2535ab18bda86aa257e174f0261d8e5d03a9fb37df74b379dff2408999f276",
    "bytes_per_reverse_stage": {64: 365032528 + 132779902 // 5,
                                32: 188583377 + 70089743 // 5},
}


def adjoint_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("adjoint_kernels.hip", "dgw_internal.h"):
        with open(os.path.join(ROOT, "paper_2205_11052_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def adjoint_kernel_times(torch, stream, make, ws, dt, d, nsteps=100):
    """Average duration of one reverse stage (its two launches) and of one
    forward stage launch, timed with HIP events on the library's stream in a
    short checkpointed run (timing on; the timed seconds per shot above are
    measured with timing off), and the reverse stage's HBM roofline."""
    out = {}
    K, N = ws["K"], ws["N"]
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    with torch.cuda.stream(stream):
        for prec in (64, 32):
            s = make(prec, ws, dt)
            s.enable_timing(True)
            s.zero_fields()
            s.forward_checkpointed(nsteps, 20, d[..., :nsteps])
            fms, _ = s.stage_kernel_ms()
            s.adjoint()
            rms, nrev = s.adjoint_stage_ms()
            s.close()
            b = reverse_stage_bytes(K, Np, prec // 8)
            out["fp%d" % prec] = {
                "forward_stage_ms": round(fms, 5), "reverse_stage_ms": round(rms, 5),
                "reverse_over_forward": round(rms / fms, 3),
                "reverse_stages_timed": nrev,
                "reverse_bytes_per_stage": b,
                "reverse_hbm_frac": round(b / (rms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "forward_hbm_frac": round(stage_bytes(K, Np, prec // 8) / (fms / 1e3) / 1e9
                                          / HBM_PEAK_GBS, 4)}
            m = MEASURED_ADJ_TRAFFIC
            if m["kernel_source_sha256"] == adjoint_source_sha():
                t = m["bytes_per_reverse_stage"][prec]
                out["fp%d" % prec]["reverse_traffic_per_stage"] = t
                out["fp%d" % prec]["reverse_traffic_hbm_frac"] = round(
                    t / (rms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def order6_form(torch, stream, w, steps, warmup, full_steps=FULL_STEPS):
    """FP32 and FP64 at order 6 (84 nodes) on the same mesh and medium:
    throughput, and the FP32 run's error against the FP64 run on the
    receiver traces and final fields after the full run from zero fields
    (dt from the CFL formula at order 6)."""
    import workloads as W
    w6 = W.build_workload("c1_layered_n24", N=6)
    out = {}
    runs = {}
    for prec in (64, 32):
        with torch.cuda.stream(stream):
            s = build_solver(w6, prec, stream=stream.cuda_stream)
            sec, _ = timed_steps(torch, s, stream, steps, warmup)
            kms, _ = kernel_avg_ms(s)
            runs[prec] = full_length_run(s, full_steps)
            shape = s.shape
            s.close()
        Np = 84
        peak = FP64_PEAK_TFLOPS if prec == 64 else FP32_PEAK_TFLOPS
        out["fp%d" % prec] = {
            "value": round(9 * Np * w6["K"] * 5 * steps / sec / 1e9, 3),
            "ms_per_step": round(sec / steps * 1e3, 4),
            "kernel_avg_ms": round(kms, 5),
            "hbm_frac": round(stage_bytes(w6["K"], Np, prec // 8) / (kms / 1e3) / 1e9
                              / HBM_PEAK_GBS, 4),
            "flops_frac": round(stage_flops(w6["K"], 6) / (kms / 1e3) / 1e12 / peak, 4),
            "launch_shape": list(shape)}
    out["fp32"]["speedup_vs_fp64"] = round(out["fp32"]["value"] / out["fp64"]["value"], 3)
    out["fp32"]["error_vs_fp64"] = full_length_errors(runs[32], runs[64])
    return out


def general_mesh_form(torch, stream, w, steps, warmup, structured_ms):
    """The workload's size (82944 elements, order 4, FP64) on a general mesh
    (jittered vertices, random element and vertex numbering, random vertex
    order per element) in three numberings: as generated (shuffled), Morton
    and reverse Cuthill-McKee (dgw_order_elements).  Stage-kernel time with
    the autotuned launch shape of each."""
    import workloads as W
    from paper_2205_11052_amd import order_elements, permute_mesh
    g = W.general_mesh(w["mesh"]["n"], w["mesh"]["L"], seed=3)
    K = g["etov"].shape[0]
    Np = 35
    out = {"elements": K, "structured_kernel_avg_ms": round(structured_ms, 5)}
    for name in ("shuffled", "morton", "rcm"):
        mesh = g if name == "shuffled" else permute_mesh(
            g, order_elements(g["vxyz"], g["etov"], name))
        rho, lam, mu, _ = W.layered_medium(W.element_centroids(mesh))
        wg = dict(w, mesh=mesh, rho=rho, lam=lam, mu=mu)
        with torch.cuda.stream(stream):
            s = build_solver(wg, 64, stream=stream.cuda_stream)
            sec, _ = timed_steps(torch, s, stream, steps, warmup)
            kms, _ = kernel_avg_ms(s)
            shape = s.shape
            s.close()
        out[name] = {
            "value": round(9 * Np * K * 5 * steps / sec / 1e9, 3),
            "kernel_avg_ms": round(kms, 5),
            "hbm_frac": round(stage_bytes(K, Np, 8) / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "vs_structured": round(structured_ms / kms, 3),
            "launch_shape": list(shape)}
    return out


def pml_bytes(n, Np, real_bytes):
    """Algorithmic bytes of one layer-kernel launch over n layer elements:
    the stage input read once (9 Np), the residual and output state read and
    written (4 x 9 Np), the memory variables and their residual read and
    written (4 x 18 Np), the per-node profile (6 Np, FP64) and the
    per-element data (DGW_META doubles); neighbour traces are not counted."""
    return n * (real_bytes * Np * (9 + 36 + 72) + 8 * 6 * Np + META_BYTES)


def variants_form(torch, stream, w, steps, warmup, plain_ms):
    """Method variants on the workload's mesh (82944 elements, order 4,
    FP64), each with the launch shape the autotuner picks for it: the
    layered medium with an absorbing sponge one unit thick on the five
    absorbing sides; the same medium with a convolutional perfectly matched
    layer of the same width (quadratic profile, nominal reflection 1e-3,
    frequency shift pi f0), whose kernel runs after each stage over the
    layer's elements; and a fully anisotropic heterogeneous medium (seeded
    random stiffness per element; node-per-thread form).  Algorithmic bytes
    add the per-element anisotropic data (DGW_ANI doubles) read once."""
    import workloads as W
    K, Np = w["K"], 35
    cen = W.element_centroids(w["mesh"])
    out = {}
    for name in ("sponge", "pml", "anisotropic"):
        progress("variant %s" % name)
        with torch.cuda.stream(stream):
            from paper_2205_11052_amd import Solver
            s = Solver(w["N"], 64, 1, stream=stream.cuda_stream)
            s.set_mesh_dict(w["mesh"])
            extra = 0
            nlayer = 0
            if name == "sponge":
                s.set_material(w["rho"], w["lam"], w["mu"])
                s.set_damping(W.sponge_profile(cen, width=1.0, sigma_max=3.0))
            elif name == "pml":
                s.set_material(w["rho"], w["lam"], w["mu"])
                cp_max = float(np.sqrt((w["lam"] + 2 * w["mu"]) / w["rho"]).max())
                el, prof, _, _ = W.pml_layer(w["mesh"], w["N"], width=1.0, cp_max=cp_max,
                                             reflection=1e-3, f0=w["f0"])
                s.set_pml(el, prof)
                nlayer = len(el)
            else:
                rho, C = W.random_stiffness(K, 2205)
                s.set_material(rho, np.ones(K), np.ones(K))
                s.set_stiffness(C)
                extra = K * ANI_BYTES
            s.set_dt(s.suggest_dt(w["cfl"]))
            s.set_source(0, w["source"], w["f0"], w["t0"], w["amp"])
            s.set_receivers(0, w["receivers"], 4096)
            shape = s.autotune()
            sec, _ = timed_steps(torch, s, stream, steps, warmup)
            kms, _ = kernel_avg_ms(s)
            pms = s.pml_kernel_ms()[0] if nlayer else 0.0
            s.close()
        out[name] = {
            "value": round(9 * Np * K * 5 * steps / sec / 1e9, 3),
            "ms_per_step": round(sec / steps * 1e3, 4),
            "kernel_avg_ms": round(kms, 5),
            "hbm_frac": round((stage_bytes(K, Np, 8) + extra) / (kms / 1e3) / 1e9
                              / HBM_PEAK_GBS, 4),
            "vs_plain": round(plain_ms / kms, 3),
            "launch_shape": list(shape)}
        if nlayer:
            out[name].update({
                "layer_elements": nlayer,
                "layer_kernel_avg_ms": round(pms, 5),
                "layer_kernel_hbm_frac": round(pml_bytes(nlayer, Np, 8) / (pms / 1e3) / 1e9
                                               / HBM_PEAK_GBS, 4)})
    return out


def batched_gradients_form(torch, stream, w, nshots=8, ckpt=100, t0=0.1):
    """Per-shot gradients of the batched workload at full length: shots 0-7
    of the 32 (seeded positions in the upper half, uneven lengths 752-1906
    steps), on the benchmark's mesh (82944 elements, order 4), all in one
    batch, each shot over its own length, checkpoints every 100 steps.  The
    observed data are the library's FP64 traces of the true layered medium
    (one batched forward); the gradients are taken at the blob-perturbed
    starting medium (cp -10% Gaussian blob), with dt fixed from the true
    medium.  At this time step the shots last 0.62-1.57 time units, so the
    Ricker wavelet is fired early (delay t0 = 0.1 instead of 1/f0) for the
    waves to reach the surface receivers inside the windows; a shot whose
    window still ends before the first arrival has a misfit at round-off
    level and is left out of shots_with_signal.  FP32 and FP64 gradients
    are both computed and timed; the FP32 error against FP64 is stated per
    shot.  Seconds for each batch and
    milliseconds per shot-step (forward with checkpoints, recomputation and
    reverse sweep all included)."""
    import workloads as W
    from paper_2205_11052_amd import Solver
    pos, lens = W.batched_shots()
    pos, lens = pos[:nshots], lens[:nshots]
    nsteps = int(lens.max())
    wb = W.build_workload("c1_layered_n24", medium="blob")

    def make(prec, m, dt=None):
        s = Solver(w["N"], prec, nshots, stream=stream.cuda_stream)
        s.set_mesh_dict(w["mesh"])
        s.set_material(m["rho"], m["lam"], m["mu"])
        s.set_dt(dt if dt is not None else s.suggest_dt(w["cfl"]))
        for i in range(nshots):
            s.set_source(i, pos[i], w["f0"], t0, w["amp"], nsteps=int(lens[i]))
            s.set_receivers(i, w["receivers"], nsteps)
        s.autotune()
        return s

    R = len(w["receivers"])
    out = {"shots": nshots, "lengths": [int(x) for x in lens],
           "shot_steps": int(lens.sum()), "checkpoint_every": ckpt,
           "elements": w["K"], "order": w["N"],
           "ricker_delay_t0": t0,
           "observed_data": "library FP64 traces of the true layered medium",
           "start_medium": "blob-perturbed (cp -10% Gaussian blob)"}
    grads = {}
    with torch.cuda.stream(stream):
        st = make(64, w)
        dt = st.dt
        st.zero_fields()
        st.step(nsteps)
        d = np.zeros((nshots, R, 3, nsteps))
        for i in range(nshots):
            tr = st.read_traces(i)
            d[i, :, :, :tr.shape[2]] = tr
        st.close()
        torch.cuda.empty_cache()
        progress("batched gradients: observed data done")
        for prec in (32, 64):
            s = make(prec, wb, dt)
            s.zero_fields()
            torch.cuda.synchronize()
            tstart = time.perf_counter()
            mis = s.forward_checkpointed(nsteps, ckpt, d)
            progress("batched gradients fp%d: forward with checkpoints done" % prec)
            g = s.adjoint()
            progress("batched gradients fp%d: reverse sweep done" % prec)
            torch.cuda.synchronize()
            sec = time.perf_counter() - tstart
            s.close()
            torch.cuda.empty_cache()      # the FP64 batch needs ~210 GB
            grads[prec] = g
            out["fp%d" % prec] = {
                "s_total": round(sec, 3),
                "ms_per_shot_step": round(1e3 * sec / float(lens.sum()), 3),
                "misfit_per_shot": [float(m) for m in mis],
                "gradients_finite": bool(all(np.isfinite(x).all() for x in g))}
    m64 = np.array(out["fp64"]["misfit_per_shot"])
    out["shots_with_signal"] = [int(i) for i in np.nonzero(m64 >= 1e-8 * m64.max())[0]]
    out["fp32_grad_rel_l2_vs_fp64_per_shot"] = [
        rel_l2(np.concatenate([grads[32][p][i] for p in range(3)]),
               np.concatenate([grads[64][p][i] for p in range(3)])) for i in range(nshots)]
    return out


def fwi_form(torch, stream, nsteps=600, iterations=3, prec=32):
    """The inversion loop (L-BFGS over the batched per-shot gradients) on
    the 24576-element order-3 workload: four shots in one batch, layered
    truth, blob-perturbed start, all of rho, lambda, mu inverted; seconds
    per iteration (each: forward sweeps of the line search, one reverse
    sweep) and the misfit history."""
    import workloads as W
    from paper_2205_11052_amd import Solver
    from paper_2205_11052_amd.inversion import invert
    wt = W.build_workload("c3_adjoint")
    ws = W.build_workload("c3_adjoint", medium="blob")
    shots = [np.array([2.5 + 5 * i, 2.5 + 5 * j, 9.1]) for i in (0, 1) for j in (0, 1)]

    def make(w, precision, dt=None):
        s = Solver(w["N"], precision, len(shots), stream=stream.cuda_stream)
        s.set_mesh_dict(w["mesh"])
        s.set_material(w["rho"], w["lam"], w["mu"])
        s.set_dt(dt if dt is not None else s.suggest_dt(w["cfl"]))
        for i, pos in enumerate(shots):
            s.set_source(i, pos, w["f0"], w["t0"], w["amp"])
            s.set_receivers(i, w["receivers"], nsteps)
        s.autotune()
        return s

    with torch.cuda.stream(stream):
        st = make(wt, 64)
        dt = st.dt
        st.zero_fields()
        st.step(nsteps)
        d_obs = np.stack([st.read_traces(i) for i in range(len(shots))])
        st.close()
        s = make(ws, prec, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist, obj = invert(s, d_obs, nsteps, 100, (ws["rho"], ws["lam"], ws["mu"]),
                              iterations)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        s.close()
    f = [h["f"] for h in hist]
    return {"precision": "fp%d" % prec, "shots": len(shots), "steps": nsteps,
            "elements": wt["K"], "iterations": len(f) - 1,
            "s_per_iteration": round(sec / max(1, len(f) - 1), 3),
            "forward_sweeps": obj.evaluations, "reverse_sweeps": obj.gradients,
            "misfit_history": [float("%.6e" % v) for v in f],
            "misfit_ratio": round(f[-1] / f[0], 4)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps=1):
    """The oracle (plain PyTorch FP64, never tuned for speed) on ONE host
    core: torch intra-op threads set to 1 and the process pinned to one
    core in-process for the measurement (both restored afterwards).  Sample:
    one warm-up right-hand side, then `steps` full LSERK4 steps (5 stages
    each) of the full 82944-element order-4 workload from zero fields."""
    import torch
    from oracle import solver as O
    threads = torch.get_num_threads()
    affinity = os.sched_getaffinity(0)
    core = min(affinity)
    torch.set_num_threads(1)
    os.sched_setaffinity(0, {core})
    try:
        P = O.Problem(w["mesh"], w["N"])
        t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
        P.set_source(w["source"], w["f0"], w["t0"], w["amp"])
        q = torch.zeros(w["K"], 9, P.Np, dtype=torch.float64)
        dt = P.suggest_dt(w["rho"], w["lam"], w["mu"], w["cfl"])
        rho, lam, mu = t(w["rho"]), t(w["lam"]), t(w["mu"])
        O.rhs(P, q, rho, lam, mu)                      # warm-up
        t0 = time.perf_counter()
        for s_ in range(steps):
            q = O.lserk_step(P, q, s_ * dt, dt, rho, lam, mu)
        sec = time.perf_counter() - t0
    finally:
        torch.set_num_threads(threads)
        os.sched_setaffinity(0, affinity)
    dof = 9 * P.Np * w["K"]
    return {"value": dof * 5 * steps / sec / 1e9, "unit": "GDOF-stage/s",
            "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "cores_available": len(affinity), "pinned_core": core,
            "torch_threads": 1,
            "sample": "%d LSERK4 step(s) (%d stages) of the full 82944-element "
                      "order-4 FP64 workload on one pinned core, %.2f s"
                      % (steps, 5 * steps, sec)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--shape", default=None,  # kernel,elements,wgs_per_cu
                    help="launch shape 'kernel,elements,wgs_per_cu' (skips the autotuner)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--fp32-probe", action="store_true",
                    help="only time the FP32 form on the headline workload "
                         "(counter runs; with --shape)")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="only one short gradient of the order-3 workload, "
                         "FP64 then FP32 (counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (the mesh-partition design is documented, not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(torch)
        return
    if args.adjoint_probe:
        print(json.dumps(adjoint_probe(torch, torch.cuda.Stream())))
        return
    shape = tuple(int(x) for x in args.shape.split(",")) if args.shape else None
    stream = torch.cuda.Stream()
    w = W.build_workload("c1_layered_n24")
    K, N = w["K"], w["N"]
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    dof = 9 * Np * K

    if args.fp32_probe:
        with torch.cuda.stream(stream):
            s = build_solver(w, 32, stream=stream.cuda_stream, shape=shape)
            sec, _ = timed_steps(torch, s, stream, args.steps, args.warmup)
            kms, nl = kernel_avg_ms(s)
            shp = s.shape
            s.close()
        print(json.dumps({"probe": "fp32", "ms_per_step": round(sec / args.steps * 1e3, 4),
                          "kernel_avg_ms": round(kms, 5), "launches_timed": nl,
                          "launch_shape": list(shp)}))
        return
    with torch.cuda.stream(stream):
        progress("headline: building and autotuning")
        s = build_solver(w, 64, stream=stream.cuda_stream, shape=shape)
        sec, windows = timed_steps(torch, s, stream, args.steps, args.warmup)
        kms, nl = kernel_avg_ms(s)
        s.check_finite()
        shape64 = s.shape
        full64 = None if args.no_forms else full_length_run(s, FULL_STEPS)
    del s
    progress("headline done")
    value = dof * 5 * args.steps / sec / 1e9
    bytes_launch = stage_bytes(K, Np, 8)
    achieved = bytes_launch / (kms / 1e3) / 1e9
    flops = stage_flops(K, N)
    ms_step = sec / args.steps * 1e3
    out = {
        "metric": "GDOF-stage/s", "value": round(value, 3),
        "unit": "GDOF-stage/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c1_layered_n24", "elements": K, "order": N,
                   "nodes_per_element": Np, "dof": dof, "shots": 1,
                   "stages_per_step": 5, "parallelism": "none (1 GPU)"},
        "timing": {"windows": len(windows), "statistic": "median",
                   "window_ms_per_step": [round(t / args.steps * 1e3, 4)
                                          for t in windows],
                   "graph_warmup_steps": GRAPH_STEPS,
                   "five_stage_kernels_ms": round(5 * kms, 4),
                   "step_over_kernels": round(ms_step / (5 * kms), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(shape64),
                     "kernel": "stage_kernel<4,double>",
                     "kernel_avg_ms": round(kms, 5),
                     "launches_timed": nl,
                     "bytes_per_launch": bytes_launch,
                     "flops_per_launch": flops,
                     "flops_achieved_tflops": round(flops / (kms / 1e3) / 1e12, 3),
                     "flops_peak_tflops": FP64_PEAK_TFLOPS,
                     "flops_frac": round(flops / (kms / 1e3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                     "counters": measured_counters(shape64),
                     "launch_shape": {"kernel": shape64[0],
                                      "elements_per_workgroup": shape64[1],
                                      "persistent_wgs_per_cu": shape64[2]}},
    }
    if not args.no_forms:
        forms = {}
        with torch.cuda.stream(stream):
            # the FP32 form's own autotuned shape (its block choices differ:
            # two column tiles per wave fit its LDS)
            s32 = build_solver(w, 32, stream=stream.cuda_stream)
            sec32, _ = timed_steps(torch, s32, stream, args.steps, args.warmup)
            k32, _ = kernel_avg_ms(s32)
            shape32 = s32.shape
            full32 = full_length_run(s32, FULL_STEPS)
        del s32
        forms["fp32"] = {
            "value": round(dof * 5 * args.steps / sec32 / 1e9, 3),
            "ms_per_step": round(sec32 / args.steps * 1e3, 4),
            "speedup_vs_fp64": round(sec / sec32, 3),
            "kernel_avg_ms": round(k32, 5),
            "hbm_frac": round(stage_bytes(K, Np, 4) / (k32 / 1e3) / 1e9
                              / HBM_PEAK_GBS, 4),
            "flops_frac": round(flops / (k32 / 1e3) / 1e12 / FP32_PEAK_TFLOPS, 4),
            "launch_shape": list(shape32),
            "error_vs_fp64": full_length_errors(full32, full64)}
        del full64, full32
        pos, lens = W.batched_shots()
        nb = len(pos)
        bsteps = max(10, args.steps // 10)
        with torch.cuda.stream(stream):
            sb = build_solver(w, 32, nshots=nb, stream=stream.cuda_stream,
                              shots=(pos, lens), shape=shape32)
            secb, _ = timed_steps(torch, sb, stream, bsteps, 2)
            kb, _ = kernel_avg_ms(sb, 2)
            shapeb = sb.shape
            # the whole uneven batch from rest to its last step: shots drop
            # out as they reach their lengths, and the launches then cover
            # the active shots only
            progress("fp32 batch: full-length run")
            sb.zero_fields()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sb.step(int(lens.max()))
            e1.record(stream)
            torch.cuda.synchronize()
            sec_full = e0.elapsed_time(e1) / 1e3
        del sb
        forms["fp32_batched_32_shots"] = {
            "value": round(nb * dof * 5 * bsteps / secb / 1e9, 3),
            "ms_per_step": round(secb / bsteps * 1e3, 4),
            "steps": bsteps,
            "speedup_vs_fp64": round((nb * bsteps / secb)
                                     / (args.steps / sec), 3),
            "kernel_avg_ms": round(kb, 5),
            "hbm_frac": round(stage_bytes(K, Np, 4, nb) / (kb / 1e3) / 1e9
                              / HBM_PEAK_GBS, 4),
            "launch_shape": list(shapeb),
            "note": "32 shots, one launch per stage over all shots, graph "
                    "replay; lengths 500-2000 steps, all active in the window",
            "full_length": {
                "shot_steps": int(lens.sum()),
                "steps": int(lens.max()),
                "s_total": round(sec_full, 3),
                "ms_per_shot_step": round(sec_full / float(lens.sum()) * 1e3, 4),
                "single_shot_ms_per_step": round(sec32 / args.steps * 1e3, 4),
                "per_shot_step_vs_single": round((sec32 / args.steps)
                                                 / (sec_full / float(lens.sum())), 3),
                "note": "every shot from rest to its own length in one run; "
                        "finished shots leave the launches"}}
        progress("fp32 and batched forms done")
        forms["order6"] = order6_form(torch, stream, w, max(20, args.steps // 5), 2)
        progress("order-6 form done")
        forms["general_mesh_fp64"] = general_mesh_form(
            torch, stream, w, max(20, args.steps // 5), 2, kms)
        progress("general-mesh form done")
        forms["variants_fp64"] = variants_form(
            torch, stream, w, max(20, args.steps // 5), 2, kms)
        out["forms"] = forms
    if not args.no_adjoint:
        progress("forms done")
        out["adjoint"] = adjoint_form(torch, stream)
        progress("adjoint form done")
        out["batched_gradients"] = batched_gradients_form(torch, stream, w)
        progress("batched gradients done")
        out["fwi"] = fwi_form(torch, stream)
        progress("fwi done")
    if not args.no_cpu:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

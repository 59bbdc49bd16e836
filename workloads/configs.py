"""Named workloads (sizes, media, shots) used by the tests and the benchmark.

* ``c0_periodic_pwave``: unit cube, 6*4^3 = 384 tetrahedra, order 3, FP64,
  homogeneous rho = 1, cs = 1, cp = sqrt(3), all faces periodic, initial state
  an exact P plane wave of wavenumber 2*pi along x, 100 steps at CFL 0.5.
* ``c1_layered_n24``: [0,10]^3, 6*24^3 = 82944 tetrahedra, order 4, FP64,
  free-surface top, absorbing elsewhere, layered noisy medium, Ricker
  explosive source (peak frequency 1), 64 surface receivers, 2000 steps.
* ``c2_fp32``: the c1 mesh and medium at orders 4 and 6 in FP32.
* ``c3_adjoint``: 6*16^3 = 24576 tetrahedra, order 3, layered model as the
  true medium, a blob-perturbed starting model, 1500 steps, checkpoint every
  100 steps, finite differences on 20 elements.
* ``c4_batched``: the c1 mesh and medium, 32 shots of uneven length, FP32.
"""

import numpy as np

from .mesh import kuhn_cube, element_centroids, lattice_node_coords
from .medium import layered_medium, homogeneous_medium, blob_start_medium
from .shots import default_source, default_receivers, batched_shots, ricker_f0
from .planewave import plane_wave_state

CONFIGS = {
    "c0_periodic_pwave": dict(n=4, L=1.0, N=3, precision=64, periodic=True,
                              medium="homogeneous", steps=100, cfl=0.5,
                              initial="pwave_x"),
    "c1_layered_n24": dict(n=24, L=10.0, N=4, precision=64, periodic=False,
                           medium="layered", steps=2000, cfl=0.5,
                           source=True, receivers=True),
    "c2_fp32": dict(n=24, L=10.0, N=(4, 6), precision=32, periodic=False,
                    medium="layered", steps=2000, cfl=0.5, source=True,
                    receivers=True),
    "c3_adjoint": dict(n=16, L=10.0, N=3, precision=(64, 32), periodic=False,
                       medium="layered", start_medium="blob", steps=1500,
                       cfl=0.5, ckpt_every=100, fd_elements=20, fd_seed=52,
                       source=True, receivers=True),
    "c4_batched": dict(n=24, L=10.0, N=4, precision=32, periodic=False,
                       medium="layered", nshots=32, min_steps=500,
                       max_steps=2000, cfl=0.5, gradient_shots=8,
                       source=True, receivers=True),
}


def get_config(name):
    return dict(CONFIGS[name])


def build_workload(name, n=None, N=None, medium=None):
    """Materialise a named workload; ``n``/``N``/``medium`` override the
    mesh resolution, order and medium (used for reduced-size test cases)."""
    cfg = get_config(name)
    n = cfg["n"] if n is None else n
    Nval = cfg["N"] if N is None else N
    if isinstance(Nval, tuple):
        Nval = Nval[0]
    mesh = kuhn_cube(n, cfg["L"], periodic=cfg["periodic"])
    K = mesh["etov"].shape[0]
    cen = element_centroids(mesh)
    kind = cfg["medium"] if medium is None else medium
    if kind == "homogeneous":
        rho, lam, mu = homogeneous_medium(K)
    elif kind == "layered":
        rho, lam, mu, _ = layered_medium(cen)
    elif kind == "blob":
        rho, lam, mu, _ = blob_start_medium(cen)
    else:
        raise ValueError(kind)
    w = dict(name=name, cfg=cfg, mesh=mesh, N=Nval, K=K,
             rho=rho, lam=lam, mu=mu, steps=cfg.get("steps"),
             cfl=cfg["cfl"], f0=ricker_f0, t0=1.0 / ricker_f0, amp=1.0)
    if cfg.get("source"):
        w["source"] = default_source()
    if cfg.get("receivers"):
        w["receivers"] = default_receivers()
    if cfg.get("initial") == "pwave_x":
        x = lattice_node_coords(mesh, Nval)
        q = plane_wave_state(x, 0.0, "P", (1, 0, 0), 2 * np.pi,
                             rho[0], lam[0], mu[0])
        w["q0"] = np.ascontiguousarray(q.transpose(0, 2, 1))   # [K, 9, Np]
    if name == "c4_batched":
        pos, lengths = batched_shots(cfg["nshots"], cfg["min_steps"],
                                     cfg["max_steps"])
        w["shot_positions"] = pos
        w["shot_lengths"] = lengths
    return w

"""Python binding of the dgw C ABI (argument marshalling only).

Every computation -- setup, stepping, receivers, energy, adjoint -- runs in
libdgw.so; this module converts arrays, checks status codes and wires the
PyTorch allocator and current stream into the library.
"""

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _lib

try:
    import torch
except ImportError:  # the binding itself does not need torch
    torch = None


class DGWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_lib.STATUS.get(code, code), msg))
        self.code = code
        self.status = _lib.STATUS.get(code, str(code))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _host64(a):
    if torch is not None and isinstance(a, torch.Tensor):
        a = a.detach().to("cpu", torch.float64).numpy()
    return _f64(a)


def ref_nodes(order):
    """Reference node coordinates [Np, 3] of the library's node contract."""
    lib = _lib.load()
    Np = (order + 1) * (order + 2) * (order + 3) // 6
    out = np.empty((Np, 3))
    rc = lib.dgw_ref_nodes(order, _dptr(out))
    if rc:
        raise DGWError(rc, "dgw_ref_nodes")
    return out


def ref_operators(order):
    """(Dr, Ds, Dt, M, LIFT) as computed by the library's host setup."""
    lib = _lib.load()
    Np = (order + 1) * (order + 2) * (order + 3) // 6
    Nfp = (order + 1) * (order + 2) // 2
    Dr, Ds, Dt, M = (np.empty((Np, Np)) for _ in range(4))
    LIFT = np.empty((Np, 4 * Nfp))
    rc = lib.dgw_ref_operators(order, _dptr(Dr), _dptr(Ds), _dptr(Dt),
                               _dptr(M), _dptr(LIFT))
    if rc:
        raise DGWError(rc, "dgw_ref_operators")
    return Dr, Ds, Dt, M, LIFT


ORDER_METHODS = {"morton": 0, "rcm": 1}


def order_elements(vxyz, etov, method="morton", vertex_periodic_id=None):
    """Element numbering for gather locality (``dgw_order_elements``):
    returns ``perm`` (int64 [K]) with element i of the reordered mesh being
    input element perm[i]."""
    lib = _lib.load()
    vxyz = _f64(vxyz)
    etov = np.ascontiguousarray(np.asarray(etov, dtype=np.int32))
    pid = None
    if vertex_periodic_id is not None:
        pid = np.ascontiguousarray(np.asarray(vertex_periodic_id, np.int32))
    if method not in ORDER_METHODS:
        raise ValueError("method must be one of %s" % sorted(ORDER_METHODS))
    perm = np.empty(etov.shape[0], dtype=np.int64)
    rc = lib.dgw_order_elements(
        vxyz.shape[0], _dptr(vxyz), etov.shape[0],
        etov.ctypes.data_as(C.POINTER(C.c_int32)),
        pid.ctypes.data_as(C.POINTER(C.c_int32)) if pid is not None else None,
        ORDER_METHODS[method], perm.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc:
        raise DGWError(rc, "dgw_order_elements")
    return perm


def permute_mesh(mesh, perm):
    """The mesh dict with its elements renumbered by ``perm`` (etov and
    face_bc rows; vertices unchanged)."""
    out = dict(mesh)
    out["etov"] = np.asarray(mesh["etov"])[perm]
    if mesh.get("face_bc") is not None:
        out["face_bc"] = np.asarray(mesh["face_bc"])[perm]
    return out


# contexts still open at interpreter exit are destroyed by an exit hook,
# while torch (whose allocator holds their device memory) is still alive
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_solvers():
    for s in list(_LIVE):
        try:
            s.close()
        except Exception:
            pass


class Solver:
    """One dgw context: a mesh, a medium and ``nshots`` shots."""

    def __init__(self, order, precision=64, nshots=1, stream=None,
                 torch_allocator=None):
        self.lib = _lib.load()
        self.order = order
        self.precision = precision
        self.nshots = nshots
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self._ctx = C.c_void_p()
        rc = self.lib.dgw_create(order, precision, nshots,
                                 C.c_void_p(stream) if stream else None,
                                 C.byref(self._ctx))
        if rc:
            raise DGWError(rc, "dgw_create(order=%s, precision=%s, nshots=%s)"
                           % (order, precision, nshots))
        _LIVE.add(self)
        if torch_allocator is None:
            torch_allocator = torch is not None and torch.cuda.is_available()
        self._callbacks = None
        if torch_allocator:
            self._use_torch_allocator()
        self.Np = (order + 1) * (order + 2) * (order + 3) // 6
        self.pml_n = 0
        self.Nfp = (order + 1) * (order + 2) // 2
        self.K = 0
        self.nrec = [0] * nshots

    # -- plumbing -------------------------------------------------------
    def _check(self, rc, what):
        if rc:
            msg = self.lib.dgw_last_error(self._ctx)
            raise DGWError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def _use_torch_allocator(self):
        dev = torch.cuda.current_device()

        cuda_alloc = torch.cuda.caching_allocator_alloc
        cuda_free = torch.cuda.caching_allocator_delete
        stream_of = torch.cuda.current_stream

        def alloc(nbytes, user):
            return cuda_alloc(int(nbytes), dev, stream_of(dev))

        def free(ptr, user):
            cuda_free(ptr)

        self._callbacks = (_lib.ALLOC_FN(alloc), _lib.FREE_FN(free))
        self._check(self.lib.dgw_set_allocator(self._ctx, self._callbacks[0],
                                               self._callbacks[1], None),
                    "dgw_set_allocator")

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.dgw_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ------------------------------------------------------------
    def set_mesh(self, vxyz, etov, vertex_periodic_id=None, face_bc=None):
        vxyz = _f64(vxyz)
        etov = np.ascontiguousarray(np.asarray(etov, dtype=np.int32))
        pid = None
        if vertex_periodic_id is not None:
            pid = np.ascontiguousarray(np.asarray(vertex_periodic_id, np.int32))
        bc = None
        if face_bc is not None:
            bc = np.ascontiguousarray(np.asarray(face_bc, dtype=np.int8))
        self._check(self.lib.dgw_set_mesh(
            self._ctx, vxyz.shape[0], _dptr(vxyz), etov.shape[0],
            etov.ctypes.data_as(C.POINTER(C.c_int32)),
            pid.ctypes.data_as(C.POINTER(C.c_int32)) if pid is not None else None,
            bc.ctypes.data_as(C.POINTER(C.c_int8)) if bc is not None else None),
            "dgw_set_mesh")
        self.K = etov.shape[0]

    def set_mesh_dict(self, mesh):
        self.set_mesh(mesh["vxyz"], mesh["etov"], mesh.get("vertex_periodic_id"),
                      mesh.get("face_bc"))

    def _per_element(self, a, width, name):
        """FP64 host copy of a per-element array; the library reads exactly
        K * width values, so any other size is refused here (before the
        mesh is set the library reads none and reports the call order)."""
        a = _host64(a)
        if self.K > 0 and a.size != self.K * width:
            raise ValueError("%s must hold %d values per element (%d elements), got %d"
                             % (name, width, self.K, a.size))
        return a

    def set_material(self, rho, lam, mu):
        r, l, m = (self._per_element(a, 1, n)
                   for a, n in ((rho, "rho"), (lam, "lambda"), (mu, "mu")))
        self._check(self.lib.dgw_set_material(self._ctx, _dptr(r), _dptr(l),
                                              _dptr(m)), "dgw_set_material")

    def suggest_dt(self, cfl):
        out = C.c_double()
        self._check(self.lib.dgw_suggest_dt(self._ctx, cfl, C.byref(out)),
                    "dgw_suggest_dt")
        return out.value

    def set_dt(self, dt):
        self._check(self.lib.dgw_set_dt(self._ctx, float(dt)), "dgw_set_dt")
        self.dt = float(dt)

    def set_source(self, shot, xyz, f0, t0, amp=1.0, nsteps=0, moment=None):
        x = _f64(xyz)
        m = _f64(moment) if moment is not None else None
        self._check(self.lib.dgw_set_source(
            self._ctx, shot, _dptr(x), _dptr(m) if m is not None else None,
            float(f0), float(t0), float(amp), int(nsteps)), "dgw_set_source")

    def set_receivers(self, shot, xyz, max_samples):
        x = _f64(xyz).reshape(-1, 3)
        self._check(self.lib.dgw_set_receivers(self._ctx, shot, x.shape[0],
                                               _dptr(x), int(max_samples)),
                    "dgw_set_receivers")
        self.nrec[shot] = x.shape[0]

    def set_fields(self, shot, q):
        q = _host64(q)
        if q.size != self.K * 9 * self.Np:
            raise ValueError("fields must have K*9*Np entries")
        self._check(self.lib.dgw_set_fields(self._ctx, shot, _dptr(q)),
                    "dgw_set_fields")

    def zero_fields(self):
        z = np.zeros((self.K, 9, self.Np))
        for s in range(self.nshots):
            self.set_fields(s, z)

    def set_shot_step(self, shot, step):
        """Resume shot `shot` at step `step` (after set_fields loaded the
        state saved there)."""
        self._check(self.lib.dgw_set_shot_step(self._ctx, int(shot), int(step)),
                    "dgw_set_shot_step")

    def get_fields(self, shot):
        out = np.empty((self.K, 9, self.Np))
        self._check(self.lib.dgw_get_fields(self._ctx, shot, _dptr(out)),
                    "dgw_get_fields")
        return out

    # -- stepping ---------------------------------------------------------
    def step(self, nsteps):
        self._check(self.lib.dgw_step(self._ctx, int(nsteps)), "dgw_step")

    def shot_steps(self, shot):
        n = C.c_int64()
        self._check(self.lib.dgw_shot_steps(self._ctx, shot, C.byref(n)),
                    "dgw_shot_steps")
        return n.value

    def read_traces(self, shot):
        n = C.c_int64()
        self._check(self.lib.dgw_read_traces(self._ctx, shot, None, 0,
                                             C.byref(n)), "dgw_read_traces")
        nr = self.nrec[shot]
        out = np.zeros((nr, 3, max(n.value, 1)))
        if nr and n.value:
            self._check(self.lib.dgw_read_traces(self._ctx, shot, _dptr(out),
                                                 out.shape[2], C.byref(n)),
                        "dgw_read_traces")
        return out[:, :, :n.value]

    def energy(self, shot=0):
        e = C.c_double()
        self._check(self.lib.dgw_energy(self._ctx, shot, C.byref(e)),
                    "dgw_energy")
        return e.value

    def energy_noalloc(self, shot=0):
        """dgw_energy through the library's static scratch (no device
        allocation)."""
        e = C.c_double()
        self._check(self.lib.dgw_energy_noalloc(self._ctx, shot, C.byref(e)),
                    "dgw_energy_noalloc")
        return e.value

    def check_finite(self):
        self._check(self.lib.dgw_check_finite(self._ctx), "dgw_check_finite")

    def set_watchdog(self, every, max_growth=0.0):
        """Check the fields every `every` steps of dgw_step (0: off): NaN or
        infinity raises DGW_ENONFINITE, and with max_growth > 0 an energy
        rise by more than that factor between checks raises DGW_EGROWTH."""
        self._check(self.lib.dgw_set_watchdog(self._ctx, int(every), float(max_growth)),
                    "dgw_set_watchdog")

    # -- differentiation --------------------------------------------------
    def forward_checkpointed(self, nsteps, ckpt_every, d_obs):
        d = _host64(d_obs)
        mis = np.empty(self.nshots)
        self._check(self.lib.dgw_forward_checkpointed(
            self._ctx, int(nsteps), int(ckpt_every), _dptr(d), _dptr(mis)),
            "dgw_forward_checkpointed")
        return mis

    def generation(self):
        """The context's state generation (see dgw_state_generation)."""
        g = C.c_uint64()
        self._check(self.lib.dgw_state_generation(self._ctx, C.byref(g)),
                    "dgw_state_generation")
        return g.value

    def adjoint(self):
        g = [np.empty((self.nshots, self.K)) for _ in range(3)]
        self._check(self.lib.dgw_adjoint(self._ctx, _dptr(g[0]), _dptr(g[1]),
                                         _dptr(g[2])), "dgw_adjoint")
        return g

    # -- launch shape and timing ---------------------------------------------
    def autotune(self, cache_path=None):
        """Time the launch shapes; returns (kernel, elements per work-group,
        persistent work-groups per CU) of the fastest."""
        k, be, w = C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.dgw_autotune(
            self._ctx, cache_path.encode() if cache_path else None,
            C.byref(k), C.byref(be), C.byref(w)), "dgw_autotune")
        return k.value, be.value, w.value

    def set_launch(self, kernel=0, elems=0, wgs_per_cu=0):
        self._check(self.lib.dgw_set_launch(self._ctx, int(kernel), int(elems),
                                            int(wgs_per_cu)), "dgw_set_launch")

    def set_damping(self, sigma=None):
        """Per-element damping rate of the absorbing sponge layer (None
        removes it)."""
        if sigma is None:
            self._check(self.lib.dgw_set_damping(self._ctx, None), "dgw_set_damping")
            return
        sg = self._per_element(sigma, 1, "sigma")
        self._check(self.lib.dgw_set_damping(self._ctx, _dptr(sg)), "dgw_set_damping")

    def set_pml(self, elements=None, profile=None):
        """Convolutional perfectly matched layer on the listed elements
        (strictly increasing ids) with the per-node profile [n, 6, Np]
        (d_x, d_y, d_z, alpha_x, alpha_y, alpha_z); None removes it."""
        if elements is None:
            self._check(self.lib.dgw_set_pml(self._ctx, 0, None, None), "dgw_set_pml")
            self.pml_n = 0
            return
        el = np.ascontiguousarray(elements, dtype=np.int32)
        pr = np.ascontiguousarray(profile, dtype=np.float64)
        if el.ndim != 1 or pr.shape != (el.shape[0], 6, self.Np):
            raise ValueError("elements must be [n] and profile [n, 6, Np]")
        self._check(self.lib.dgw_set_pml(
            self._ctx, el.shape[0], el.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(pr)),
            "dgw_set_pml")
        self.pml_n = el.shape[0]

    def pml_memory(self, shot=0):
        """The layer's memory variables of a shot, [n, 18, Np]."""
        out = np.empty((self.pml_n, 18, self.Np))
        self._check(self.lib.dgw_get_pml_memory(self._ctx, int(shot), _dptr(out)),
                    "dgw_get_pml_memory")
        return out

    def set_pml_memory(self, shot, m):
        """Restore a shot's memory variables, [n, 18, Np] (after set_fields)."""
        a = np.ascontiguousarray(m, dtype=np.float64)
        if a.shape != (self.pml_n, 18, self.Np):
            raise ValueError("memory variables must be [n, 18, Np]")
        self._check(self.lib.dgw_set_pml_memory(self._ctx, int(shot), _dptr(a)),
                    "dgw_set_pml_memory")

    def pml_kernel_ms(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.dgw_pml_kernel_ms(self._ctx, C.byref(ms), C.byref(n)),
                    "dgw_pml_kernel_ms")
        return ms.value, n.value

    def set_stiffness(self, C=None):
        """Anisotropic elements: Voigt stiffness per element, [K, 6, 6]
        (symmetric) or its upper triangles [K, 21] (None: isotropic
        again)."""
        if C is None:
            self._check(self.lib.dgw_set_stiffness(self._ctx, None), "dgw_set_stiffness")
            return
        C = np.asarray(C, dtype=np.float64)
        if C.ndim == 3:
            if C.shape[1:] != (6, 6):
                raise ValueError("stiffness must be [K, 6, 6] or [K, 21]")
            iu = np.triu_indices(6)
            C = C[:, iu[0], iu[1]]
        if C.ndim != 2 or C.shape[1] != 21:
            raise ValueError("stiffness must be [K, 6, 6] or [K, 21]")
        up = self._per_element(C, 21, "stiffness")
        self._check(self.lib.dgw_set_stiffness(self._ctx, _dptr(up)), "dgw_set_stiffness")

    def set_adjoint_memory(self, nbytes=-1):
        """Device bytes the reverse sweep may keep stage states in (-1:
        a quarter of the free memory, 0: recompute them)."""
        self._check(self.lib.dgw_set_adjoint_memory(self._ctx, int(nbytes)),
                    "dgw_set_adjoint_memory")

    def set_flux(self, tau=1.0):
        """Upwind weight of the face flux (1 upwind, 0 central)."""
        self._check(self.lib.dgw_set_flux(self._ctx, float(tau)), "dgw_set_flux")

    def enable_timing(self, on=True):
        self._check(self.lib.dgw_enable_timing(self._ctx, 1 if on else 0),
                    "dgw_enable_timing")

    def adjoint_stage_ms(self):
        """(average ms of one reverse stage, stages timed) of the last
        adjoint() run with timing enabled."""
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.dgw_adjoint_stage_ms(self._ctx, C.byref(ms), C.byref(n)),
                    "dgw_adjoint_stage_ms")
        return ms.value, n.value

    def stage_kernel_ms(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.dgw_stage_kernel_ms(self._ctx, C.byref(ms),
                                                 C.byref(n)),
                    "dgw_stage_kernel_ms")
        return ms.value, n.value


if torch is not None:
    class ElasticMisfit(torch.autograd.Function):
        """misfit[s] = 1/2 dt sum (trace_s - d_obs[s])^2 as a function of the
        per-element rho, lambda, mu; backward runs the library's discrete
        adjoint (with checkpointed forward recomputation).

        apply(rho, lam, mu, solver, d_obs, nsteps, ckpt_every) -> [nshots]
        Every shot starts from zero fields."""

        @staticmethod
        def forward(ctx, rho, lam, mu, solver, d_obs, nsteps, ckpt_every):
            solver.set_material(rho, lam, mu)
            solver.zero_fields()
            mis = solver.forward_checkpointed(nsteps, ckpt_every, d_obs)
            ctx.solver = solver
            ctx.generation = solver.generation()
            ctx.device = rho.device
            return torch.as_tensor(mis, dtype=torch.float64, device=rho.device)

        @staticmethod
        def backward(ctx, grad_out):
            if ctx.solver.generation() != ctx.generation:
                raise RuntimeError(
                    "ElasticMisfit.backward: the solver ran or changed after this "
                    "forward (another apply, a setter or a step); its checkpoints "
                    "belong to a different forward")
            g = ctx.solver.adjoint()
            w = grad_out.detach().to("cpu", torch.float64).numpy()
            outs = [torch.as_tensor((w[:, None] * gi).sum(axis=0),
                                    device=ctx.device) for gi in g]
            return outs[0], outs[1], outs[2], None, None, None, None
else:
    ElasticMisfit = None

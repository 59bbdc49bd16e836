"""Nodal DG right-hand side, LSERK4 time stepping, source, receivers, energy.

Oracle (test infrastructure), plain PyTorch CPU in FP64 (complex128 for
complex-step differentiation).  The paper (arXiv 2205.11052) does not describe
this method; each function states the formula it implements.

Unknowns per element k, node n: q[k, c, n] with field order
c = (vx, vy, vz, sxx, syy, szz, syz, sxz, sxy); material rho, lambda, mu is
constant per element.

Semi-discrete strong form (nodal DG; Hesthaven and Warburton 2008):

* volume:  d/dx = rx Dr + sx Ds + tx Dt (and likewise y, z), with
  (rx, ry, rz), (sx, sy, sz), (tx, ty, tz) the rows of X^-1;
  v_t = (1/rho) div(sigma);
  sigma_t = lambda div(v) I + mu (grad v + grad v^T).
* faces: n is the own element's outward normal, (v-, sigma-) the own trace,
  (v+, sigma+) the neighbour's trace at the matched node, t = sigma n on both
  sides with the same n.  Split v and t into normal parts (v_n = n.v,
  t_n = n.t) and tangential parts (v_T = v - v_n n, t_T = t - t_n n).  With
  Z = Zp = sqrt(rho (lambda + 2 mu)) for the normal parts and
  Z = Zs = sqrt(rho mu) for the tangential parts, the exact solution of the
  one-dimensional Riemann problem normal to the face (the upwind flux for
  elastic waves, Wilcox et al., J. Comput. Phys. 229, 2010) is
      t* = (Z+ t- + Z- t+ + Z- Z+ (v+ - v-)) / (Z- + Z+)
      v* = (Z- v- + Z+ v+ + t+ - t-) / (Z- + Z+).
  With dt_ = t* - t- and dv = v* - v-:
      v_t     += (1/rho-) Fscale_f LIFT_f dt_
      sigma_t += Fscale_f LIFT_f [lambda- (n.dv) I + mu- (dv n^T + n dv^T)].
* boundary ghost states (Z+ = Z-): free surface v+ = v-, sigma+ = -sigma-
  (so t* = 0); absorbing v+ = 0, sigma+ = 0.
* absorbing sponge layer (P.sponge = sigma [K] >= 0, default none): the
  right-hand side gains -sigma_k q on every field of element k, the
  damping layer of Cerjan, Kosloff, Kosloff and Reshef (Geophysics 50,
  1985); the energy then changes by -2 sum_k sigma_k E_k.
* fluid elements (mu = 0, acoustic): Zs = 0, so the tangential
  states above are well defined whenever one side is solid (the solid's
  tangential traction acts on a slip interface); where both sides are fluid
  (Zs- + Zs+ = 0) there is no tangential coupling: t*_T = t-_T, v*_T = v-_T.
* anisotropic elements (P.stiffness = C [K, 6, 6], default none):
  the stiffness in Voigt order (xx, yy, zz, yz, xz, xy) with engineering
  shear strains, symmetric positive definite, replaces lambda and mu
  (rho stays).  Volume: sigma_t = C e(v) with
  e = (dx vx, dy vy, dz vz, dy vz + dz vy, dx vz + dz vx, dx vy + dy vx).
  Faces: the strain of sym(a n^T) is N(n) a, with the 6x3 matrix
  N(n) = [[nx,0,0],[0,ny,0],[0,0,nz],[0,nz,ny],[nz,0,nx],[ny,nx,0]]; the
  traction is t = N(n)^T sigma, and along the normal coordinate x_n the
  pair (t, v) obeys rho v_t = d t / d x_n, t_t = G d v / d x_n with the
  Christoffel matrix G = N^T C N (3x3, SPD).  Its characteristic variables t -+ Z v, with the
  impedance matrix Z = (rho G)^(1/2) (the SPD square root), travel away
  from the face on either side, so the exact Riemann states are
      v* = (Z- + Z+)^-1 (Z- v- + Z+ v+ + t+ - t-),   t* = t- + Z- (v* - v-)
  (for isotropic C, Z = Zp n n^T + Zs (I - n n^T) and these are the states
  above).  Stress flux: Fscale LIFT C N(n) dv.  Boundary ghost states as
  above with Z+ = Z-.  Energy: the potential term is sigma^T C^-1 sigma.
* flux variant (P.flux_tau = tau in [0, 1], default 1): the states used are
  tau (t*, v*) + (1 - tau) ((t- + t+)/2, (v- + v+)/2), i.e. a convex
  combination of the upwind flux and the central flux (the alpha-flux family
  of Hesthaven and Warburton, section 2.2 and chapter 6, with alpha =
  1 - tau); the central flux conserves the semi-discrete energy on meshes
  without boundaries, the upwind part dissipates it.

Time stepping: five-stage fourth-order low-storage Runge-Kutta (Carpenter and
Kennedy, NASA TM-109112, 1994): for i = 1..5,
res = A_i res + dt (L q + s(t_n + C_i dt)); q = q + B_i res; res = 0 at the
start of each step.

Source: moment tensor M (default the explosion M = I) with Ricker time
function s(tau) = amp (1 - 2 pi^2 f0^2 (tau - t0)^2) exp(-pi^2 f0^2 (tau - t0)^2),
added to the stress components of the source element as
M_c s(tau) / J M^-1 l(r_s) (the projection of a Dirac delta at the source
point).

Receivers: after every step, trace[r, c, n] = l(r_r) . v_c(k_r), c = x, y, z.

Energy: E = 1/2 sum_k J_k [ rho v.Mv + (1/(2 mu)) (sum_diag s^T M s
         + 2 sum_offdiag s^T M s) - lambda / (2 mu (3 lambda + 2 mu)) tr^T M tr ];
for a fluid element (mu = 0) the potential term is the isotropic part,
tr^T M tr / (9 lambda) (the mu -> 0 limit of the above for isotropic
stress; a fluid's deviatoric stress does not evolve).

Misfit: J = 1/2 dt sum_n sum_r sum_c (trace - d)^2.
"""

import math

import numpy as np
import torch

from . import refelem, setup

# Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients.
LSERK_A = [0.0,
           -567301805773.0 / 1357537059087.0,
           -2404267990393.0 / 2016746695238.0,
           -3550918686646.0 / 2091501179385.0,
           -1275806237668.0 / 842570457699.0]
LSERK_B = [1432997174477.0 / 9575080441755.0,
           5161836677717.0 / 13612068292357.0,
           1720146321549.0 / 2090206949498.0,
           3134564353537.0 / 4481467310338.0,
           2277821191437.0 / 14882151754819.0]
LSERK_C = [0.0,
           1432997174477.0 / 9575080441755.0,
           2526269341429.0 / 6820363962896.0,
           2006345519317.0 / 3224310063776.0,
           2802321613138.0 / 2924317926251.0]

VX, VY, VZ, SXX, SYY, SZZ, SYZ, SXZ, SXY = range(9)


def ricker(tau, f0, t0, amp=1.0):
    a = (math.pi * f0 * (tau - t0)) ** 2
    return amp * (1.0 - 2.0 * a) * math.exp(-a)


class Problem:
    """Mesh-dependent data of the discretisation (independent of material)."""

    def __init__(self, mesh, N):
        self.N = N
        self.ops = refelem.operators(N)
        self.Np, self.Nfp = self.ops["Np"], self.ops["Nfp"]
        self.mesh = mesh
        self.EToE, self.EToF, self.bc, gid = setup.connectivity(mesh)
        self.nbr_node = setup.face_node_map(N, self.EToE, self.EToF, self.bc,
                                            gid)
        self.geo = setup.geometry(mesh)
        self.K = self.EToE.shape[0]
        t = lambda a: torch.as_tensor(np.asarray(a))
        self.Dr, self.Ds, self.Dt = t(self.ops["Dr"]), t(self.ops["Ds"]), t(self.ops["Dt"])
        self.LIFT = t(self.ops["LIFT"])
        self.M = t(self.ops["M"])
        self.Minv = t(self.ops["Minv"])
        self.Fmask = t(self.ops["Fmask"]).reshape(-1)             # [4 Nfp]
        self.Xinv = t(self.geo["Xinv"])
        self.J = t(self.geo["J"])
        self.normals = t(self.geo["normals"])                     # [K,4,3]
        self.Fscale = t(self.geo["Fscale"])                       # [K,4]
        Nfp = self.Nfp
        self.nb_elem = t(np.repeat(self.EToE[:, :, None], Nfp, axis=2))
        self.nb_node = t(self.nbr_node)
        self.free = t(self.bc == 1)[:, :, None]                   # [K,4,1]
        self.absorb = t(self.bc == 2)[:, :, None]
        self.EToE_t = t(self.EToE)
        self.source = None
        self.receivers = None
        # weight of the exact Riemann (upwind) flux; 1 - flux_tau goes to the
        # central flux
        self.flux_tau = 1.0
        # per-element damping rate of the absorbing sponge layer (None: none)
        self.sponge = None
        # per-element Voigt stiffness [K, 6, 6] of anisotropic elements
        # (None: isotropic lambda, mu)
        self.stiffness = None

    # --- sources and receivers -------------------------------------------
    def set_source(self, xyz, f0, t0, amp=1.0, moment=(1, 1, 1, 0, 0, 0)):
        """Point source M s(t) delta(x - xyz); moment in the order
        (xx, yy, zz, yz, xz, xy), default the explosion M = I."""
        k, rst = setup.locate(self.mesh, self.geo, np.asarray(xyz, float))
        ell = refelem.lagrange_at(self.N, rst)[0]
        vec = self.ops["Minv"] @ ell / self.geo["J"][k]
        self.source = dict(k=k, rst=rst, vec=torch.as_tensor(vec), f0=f0,
                           t0=t0, amp=amp, moment=tuple(float(m) for m in moment))

    def set_receivers(self, xyz):
        xyz = np.atleast_2d(np.asarray(xyz, float))
        ks, ws = [], []
        for x in xyz:
            k, rst = setup.locate(self.mesh, self.geo, x)
            ks.append(k)
            ws.append(refelem.lagrange_at(self.N, rst)[0])
        self.receivers = dict(k=torch.as_tensor(ks),
                              w=torch.as_tensor(np.array(ws)))

    def suggest_dt(self, rho, lam, mu, cfl):
        return setup.suggest_dt(self.geo, rho, lam, mu, self.N, cfl)


def voigt_nmat(n):
    """N(n) for normals n [..., 3]: the 6x3 matrix mapping a vector a to the
    Voigt strain (engineering shears) of sym(a n^T); its transpose maps a
    Voigt stress to the traction sigma n.  Returns [..., 6, 3]."""
    nx, ny, nz = n[..., 0], n[..., 1], n[..., 2]
    z = torch.zeros_like(nx)
    rows = [[nx, z, z], [z, ny, z], [z, z, nz], [z, nz, ny], [nz, z, nx],
            [ny, nx, z]]
    return torch.stack([torch.stack(r, dim=-1) for r in rows], dim=-2)


def impedance(rho, C, Nm):
    """Z = (rho N^T C N)^(1/2), the SPD square root by eigendecomposition;
    rho [...], C [..., 6, 6], Nm [..., 6, 3] -> [..., 3, 3]."""
    G = Nm.transpose(-1, -2) @ C @ Nm * rho[..., None, None]
    w, V = torch.linalg.eigh(G)
    return V @ torch.diag_embed(torch.sqrt(w)) @ V.transpose(-1, -2)


def face_states(P, q, rho, lam, mu):
    """Changes of the flux states against the own trace on every face node:
    dT = t* - t- and dV = v* - v- [K, 3, 4, Nfp] (upwind, blended or
    anisotropic as set on P), and the outward normals n [K, 3, 4, 1]."""
    dt_ = q.dtype
    K, Nfp = P.K, P.Nfp
    C = P.stiffness
    qm = q[:, :, P.Fmask].reshape(K, 9, 4, Nfp)
    qp = q[P.nb_elem, :, P.nb_node].permute(0, 3, 1, 2)            # [K,9,4,Nfp]
    zero = torch.zeros_like(qm)
    vm, sm = qm[:, 0:3], qm[:, 3:9]
    vp, sp = qp[:, 0:3], qp[:, 3:9]
    free = P.free[:, None]                                         # [K,1,4,1]
    absorb = P.absorb[:, None]
    vp = torch.where(free, vm, torch.where(absorb, zero[:, 0:3], vp))
    sp = torch.where(free, -sm, torch.where(absorb, zero[:, 3:9], sp))

    n = P.normals.to(dt_).permute(0, 2, 1)[:, :, :, None]          # [K,3,4,1]

    def traction(s):
        # t_a = sum_b sigma_ab n_b (Voigt order xx yy zz yz xz xy)
        sxx, syy, szz, syz, sxz, sxy = (s[:, i] for i in range(6))
        nx, ny, nz = n[:, 0], n[:, 1], n[:, 2]
        return torch.stack([sxx * nx + sxy * ny + sxz * nz,
                            sxy * nx + syy * ny + syz * nz,
                            sxz * nx + syz * ny + szz * nz], dim=1)

    tm, tp = traction(sm), traction(sp)
    Zp = torch.sqrt(rho * (lam + 2.0 * mu))
    Zs = torch.sqrt(rho * mu)
    bnd = (P.free | P.absorb)[:, :, 0]                             # [K,4]
    nb = P.EToE_t
    Zp_m = Zp[:, None].expand(K, 4)
    Zs_m = Zs[:, None].expand(K, 4)
    Zp_p = torch.where(bnd, Zp_m, Zp[nb])
    Zs_p = torch.where(bnd, Zs_m, Zs[nb])
    Zp_m, Zs_m, Zp_p, Zs_p = (z[:, None, :, None] for z in (Zp_m, Zs_m, Zp_p, Zs_p))

    def split(v):
        vn = (v * n).sum(dim=1, keepdim=True)
        return vn, v - vn * n

    vmn, vmT = split(vm)
    vpn, vpT = split(vp)
    tmn, tmT = split(tm)
    tpn, tpT = split(tp)
    tsn = (Zp_p * tmn + Zp_m * tpn + Zp_m * Zp_p * (vpn - vmn)) / (Zp_m + Zp_p)
    # fluid on both sides (mu = 0, Zs- + Zs+ = 0): no tangential coupling,
    # the tangential states stay the own ones
    zs_sum = Zs_m + Zs_p
    solid = (zs_sum.real if zs_sum.is_complex() else zs_sum) > 0
    zs_den = torch.where(solid, zs_sum, torch.ones_like(zs_sum))
    tsT = torch.where(solid, (Zs_p * tmT + Zs_m * tpT + Zs_m * Zs_p * (vpT - vmT)) / zs_den,
                      tmT)
    vsn = (Zp_m * vmn + Zp_p * vpn + tpn - tmn) / (Zp_m + Zp_p)
    vsT = torch.where(solid, (Zs_m * vmT + Zs_p * vpT + tpT - tmT) / zs_den, vmT)
    tstar, vstar = tsn * n + tsT, vsn * n + vsT
    if C is not None:
        # impedance matrices of both sides on each face, with the own
        # outward normal (G(n) = G(-n)); the ghost side of a boundary face
        # has the own one
        Nm = voigt_nmat(P.normals)                                 # [K,4,6,3]
        Zm = impedance(rho[:, None].expand(K, 4), C[:, None].expand(K, 4, 6, 6), Nm)
        Zn = impedance(rho[nb], C[nb], Nm)
        Zpl = torch.where(bnd[:, :, None, None], Zm, Zn)
        Zm, Zpl = Zm.to(dt_), Zpl.to(dt_)
        mv = lambda Z, x: torch.einsum("kfij,kjfn->kifn", Z, x)   # Z x per face
        W = torch.linalg.inv(Zm + Zpl)
        vstar = mv(W, mv(Zm, vm) + mv(Zpl, vp) + tp - tm)
        tstar = tm + mv(Zm, vstar - vm)
    # flux states: tau times the exact Riemann states plus (1 - tau) times
    # the central (averaged) states; tau = 1 is the upwind flux, tau = 0
    # the central one (boundary ghost states as above in both)
    tau = P.flux_tau
    tS = tau * tstar + (1.0 - tau) * 0.5 * (tm + tp)
    vS = tau * vstar + (1.0 - tau) * 0.5 * (vm + vp)
    dT = tS - tm                                                   # [K,3,4,Nfp]
    dV = vS - vm
    return dT, dV, n


def rhs(P, q, rho, lam, mu):
    """L q for q [K, 9, Np] (no source); rho, lam, mu are [K] tensors
    (lam and mu unused where P.stiffness is set)."""
    dt_ = q.dtype
    Dr, Ds, Dt = P.Dr.to(dt_), P.Ds.to(dt_), P.Dt.to(dt_)
    Xinv = P.Xinv.to(dt_)
    # reference derivatives of every field, then physical ones:
    # d/dx_b q_c = sum_r Xinv[r, b] (D_r q_c)
    ref = torch.stack([q @ Dr.T, q @ Ds.T, q @ Dt.T], dim=2)       # [K,9,3,Np]
    grad = torch.einsum("krb,kcrn->kcbn", Xinv, ref)              # [K,9,3,Np]
    dx = lambda c, b: grad[:, c, b]
    r = rho[:, None]
    l = lam[:, None]
    m = mu[:, None]
    divv = dx(VX, 0) + dx(VY, 1) + dx(VZ, 2)
    out = torch.stack([
        (dx(SXX, 0) + dx(SXY, 1) + dx(SXZ, 2)) / r,
        (dx(SXY, 0) + dx(SYY, 1) + dx(SYZ, 2)) / r,
        (dx(SXZ, 0) + dx(SYZ, 1) + dx(SZZ, 2)) / r,
        l * divv + 2.0 * m * dx(VX, 0),
        l * divv + 2.0 * m * dx(VY, 1),
        l * divv + 2.0 * m * dx(VZ, 2),
        m * (dx(VY, 2) + dx(VZ, 1)),
        m * (dx(VX, 2) + dx(VZ, 0)),
        m * (dx(VX, 1) + dx(VY, 0)),
    ], dim=1)                                                      # [K,9,Np]
    C = P.stiffness
    if C is not None:
        strain = torch.stack([dx(VX, 0), dx(VY, 1), dx(VZ, 2), dx(VY, 2) + dx(VZ, 1),
                              dx(VX, 2) + dx(VZ, 0), dx(VX, 1) + dx(VY, 0)], dim=1)
        out = torch.cat([out[:, 0:3],
                         torch.einsum("kij,kjn->kin", C.to(dt_), strain)], dim=1)

    dT, dV, n = face_states(P, q, rho, lam, mu)
    K, Nfp = P.K, P.Nfp
    ndv = (n * dV).sum(dim=1)                                      # [K,4,Nfp]
    lm = lam[:, None, None]
    mm = mu[:, None, None]
    flux = torch.stack([
        dT[:, 0] / rho[:, None, None], dT[:, 1] / rho[:, None, None],
        dT[:, 2] / rho[:, None, None],
        lm * ndv + 2.0 * mm * dV[:, 0] * n[:, 0],
        lm * ndv + 2.0 * mm * dV[:, 1] * n[:, 1],
        lm * ndv + 2.0 * mm * dV[:, 2] * n[:, 2],
        mm * (dV[:, 1] * n[:, 2] + dV[:, 2] * n[:, 1]),
        mm * (dV[:, 0] * n[:, 2] + dV[:, 2] * n[:, 0]),
        mm * (dV[:, 0] * n[:, 1] + dV[:, 1] * n[:, 0]),
    ], dim=1)                                                      # [K,9,4,Nfp]
    if C is not None:
        # stress flux C N(n) dv
        eN = torch.einsum("kfij,kjfn->kifn", voigt_nmat(P.normals).to(dt_), dV)
        flux = torch.cat([flux[:, 0:3], torch.einsum("kij,kjfn->kifn", C.to(dt_), eN)],
                         dim=1)
    flux = flux * P.Fscale.to(dt_)[:, None, :, None]
    out = out + flux.reshape(K, 9, 4 * Nfp) @ P.LIFT.to(dt_).T
    if P.sponge is not None:
        out = out - P.sponge.to(dt_)[:, None, None] * q
    return out


def source_term(P, tau, dtype):
    """Source contribution to the right-hand side at time tau: [K, 9, Np]."""
    out = torch.zeros(P.K, 9, P.Np, dtype=dtype)
    if P.source is not None:
        s = P.source
        val = ricker(tau, s["f0"], s["t0"], s["amp"])
        for c, mc in zip((SXX, SYY, SZZ, SYZ, SXZ, SXY), s["moment"]):
            out[s["k"], c] = val * mc * s["vec"].to(dtype)
    return out


def lserk_step(P, q, t, dt, rho, lam, mu):
    """One LSERK4 step from time t; returns the new state."""
    res = torch.zeros_like(q)
    for i in range(5):
        tau = t + LSERK_C[i] * dt
        res = LSERK_A[i] * res + dt * (rhs(P, q, rho, lam, mu)
                                       + source_term(P, tau, q.dtype))
        q = q + LSERK_B[i] * res
    return q


def sample_receivers(P, q):
    """[nrec, 3] receiver velocities of state q."""
    R = P.receivers
    v = q[R["k"], 0:3, :]                                          # [nrec,3,Np]
    return torch.einsum("rcn,rn->rc", v, R["w"].to(q.dtype))


def run(P, q0, rho, lam, mu, dt, nsteps, t0=0.0, record=False):
    """Advance nsteps; returns (q, traces [nrec, 3, nsteps] or None)."""
    q = q0
    traces = []
    for s in range(nsteps):
        q = lserk_step(P, q, t0 + s * dt, dt, rho, lam, mu)
        if record:
            traces.append(sample_receivers(P, q))
    tr = torch.stack(traces, dim=2) if record and traces else None
    return q, tr


def energy(P, q, rho, lam, mu):
    """Discrete elastic energy of state q (see module docstring)."""
    M = P.M.to(q.dtype)
    quad = lambda a, b: torch.einsum("kn,nm,km->k", a, M, b)
    kin = sum(quad(q[:, c], q[:, c]) for c in (VX, VY, VZ))
    diag = sum(quad(q[:, c], q[:, c]) for c in (SXX, SYY, SZZ))
    off = sum(quad(q[:, c], q[:, c]) for c in (SYZ, SXZ, SXY))
    tr = q[:, SXX] + q[:, SYY] + q[:, SZZ]
    trq = quad(tr, tr)
    fluid = (mu.real if mu.is_complex() else mu) == 0
    mus = torch.where(fluid, torch.ones_like(mu), mu)
    elastic = (diag + 2.0 * off) / (2.0 * mus) \
        - lam / (2.0 * mus * (3.0 * lam + 2.0 * mus)) * trq
    pot = torch.where(fluid, trq / (9.0 * lam), elastic)
    if P.stiffness is not None:
        S = torch.linalg.inv(P.stiffness).to(q.dtype)             # compliance
        sM = torch.einsum("kin,nm->kim", q[:, 3:9], M)
        pot = torch.einsum("kij,kim,kjm->k", S, sM, q[:, 3:9])
    return 0.5 * torch.sum(P.J.to(q.dtype) * (rho * kin + pot))


def misfit(traces, d_obs, dt):
    return 0.5 * dt * torch.sum((traces - d_obs) ** 2)


def as_tensor(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype)

/*
 * dgw -- nodal discontinuous Galerkin solver for the isotropic (optionally
 * anisotropic, dgw_set_stiffness) velocity-stress elastic wave equation on
 * affine tetrahedra, for AMD Instinct MI355X (gfx950).
 *
 * Method.  The paper this library accompanies (arXiv 2205.11052) does not
 * describe the discretisation, so every entry point states what it computes:
 *
 *   unknowns   q[k][c][n]: element k, field c in the order
 *              (vx, vy, vz, sxx, syy, szz, syz, sxz, sxy), node n;
 *   nodes      the equispaced lattice of order N on the reference tetrahedron
 *              (-1,-1,-1),(1,-1,-1),(-1,1,-1),(-1,-1,1); node (i,j,k),
 *              i+j+k <= N, at (r,s,t) = -1 + 2 (i,j,k)/N, ordered k outermost,
 *              then j, then i (dgw_ref_nodes returns them);
 *   faces      local face f is the face opposite local vertex f;
 *   volume     strong form, rho v_t = div sigma,
 *              sigma_t = lambda div(v) I + mu (grad v + grad v^T), with
 *              element-constant rho, lambda, mu (nodal DG, Hesthaven and
 *              Warburton, "Nodal Discontinuous Galerkin Methods", 2008);
 *   faces      exact Riemann (upwind) flux of the elastic system normal to the
 *              face with P impedance sqrt(rho (lambda + 2 mu)) on the normal
 *              parts and S impedance sqrt(rho mu) on the tangential parts
 *              (Wilcox, Stadler, Burstedde, Ghattas, J. Comput. Phys. 229,
 *              2010), optionally blended with the central flux
 *              (dgw_set_flux), lifted to the element by the exact face mass
 *              matrices;
 *   boundaries free surface (zero traction) and first-order absorbing
 *              (no incoming characteristic); periodic faces are ordinary
 *              neighbours;
 *   time       five-stage fourth-order low-storage Runge-Kutta (Carpenter and
 *              Kennedy, NASA TM-109112, 1994); the source time function is
 *              evaluated at t_n + C_i dt in stage i;
 *   source     moment-tensor point source M s(t) delta(x - x_s) added to the
 *              stress equation, s the Ricker wavelet
 *              amp (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2);
 *   receivers  velocity interpolated at each receiver after every step;
 *   misfit     J = 1/2 dt sum_steps sum_receivers sum_xyz (trace - d)^2;
 *   gradient   exact discrete adjoint of the time-stepping scheme with
 *              respect to per-element rho, lambda, mu.
 *
 * Conventions for every entry point:
 *   - Return value is a dgw_status; no C++ exception crosses the ABI.  On a
 *     failure dgw_last_error() describes it.
 *   - Host pointers are borrowed for the duration of the call only (the
 *     library copies what it keeps).  Arrays are C order, FP64 unless stated.
 *   - The context owns all device memory (allocated through the allocator
 *     hook if one is set, else hipMalloc) and releases it in dgw_destroy.
 *   - All device work is ordered on the context's stream; functions that
 *     return data to the host synchronise that stream.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef DGW_H
#define DGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgw_ctx dgw_ctx;

typedef enum dgw_status {
  DGW_OK = 0,
  DGW_EINVAL = -1,     /* invalid argument (null pointer, bad size/value)   */
  DGW_ENOMEM = -2,     /* device or host allocation failed                 */
  DGW_EMESH = -3,      /* invalid mesh: non-positive volume, non-manifold
                          face, unmatched face without boundary tag        */
  DGW_EHIP = -4,       /* a HIP runtime call failed (or no GPU present)    */
  DGW_ESTATE = -5,     /* call made in the wrong order                     */
  DGW_ERANGE = -6,     /* index or capacity out of range, point outside    */
  DGW_ENONFINITE = -7, /* non-finite value detected in the fields          */
  DGW_EGROWTH = -8     /* a shot's energy grew past the watchdog's bound   */
} dgw_status;

/* Create a context for polynomial order 1..6, precision 64 (FP64 fields and
 * arithmetic) or 32 (FP32 fields and arithmetic, geometric factors kept in
 * FP64 storage and converted in registers, reductions in FP64), and nshots
 * independent shots sharing one mesh and medium.  hip_stream is a
 * hipStream_t to order work on, or NULL for a stream owned by the library.
 * No device memory is touched until dgw_set_mesh. */
int dgw_create(int order, int precision, int nshots, void *hip_stream,
               dgw_ctx **out);
void dgw_destroy(dgw_ctx *ctx);
const char *dgw_last_error(const dgw_ctx *ctx);

/* Route device allocations through alloc(bytes, user) / free_(ptr, user)
 * (for example a PyTorch caching allocator).  Must precede dgw_set_mesh. */
int dgw_set_allocator(dgw_ctx *ctx, void *(*alloc)(size_t, void *),
                      void (*free_)(void *, void *), void *user);

/* Mesh upload.  vxyz [nvert][3]; etov [K][4] (0-based vertex ids, any
 * orientation is accepted: negatively oriented elements are rejected with
 * DGW_EMESH); vertex_periodic_id [nvert] or NULL: vertices with equal ids are
 * identified when faces are matched (periodic meshes); face_bc [K][4] gives,
 * for faces without a neighbour, 1 = free surface or 2 = absorbing (other
 * values on such a face are DGW_EMESH; the value is ignored where a neighbour
 * exists).  Faces are matched by the sorted triple of their (identified)
 * vertex ids; a triple shared by more than two faces is DGW_EMESH. */
int dgw_set_mesh(dgw_ctx *ctx, int64_t nvert, const double *vxyz, int64_t K,
                 const int32_t *etov, const int32_t *vertex_periodic_id,
                 const int8_t *face_bc);

/* Per-element density and Lame parameters [K]; requires rho > 0, mu >= 0,
 * lambda + 2 mu / 3 > 0 and finite values (DGW_EINVAL otherwise).  mu = 0
 * makes the element a fluid (acoustic; its stress is meant to be isotropic,
 * -p I): S impedance zero, coupled to solid neighbours through the same
 * Riemann states (the solid's tangential traction acts on a slip
 * interface), and with no tangential coupling where both sides are fluid.
 * dgw_energy counts a fluid element's isotropic stress only,
 * tr^T M tr / (9 lambda).  The gradient (dgw_forward_checkpointed,
 * dgw_adjoint) is not defined with fluid elements: DGW_ESTATE. */
int dgw_set_material(dgw_ctx *ctx, const double *rho, const double *lam,
                     const double *mu);

/* dt = cfl * 2 * min_k (r_k / cp_k) / (N+1)^2 with r_k = 3 V_k / sum_f A_f
 * the inradius and cp_k = sqrt((lambda + 2 mu) / rho). */
int dgw_suggest_dt(const dgw_ctx *ctx, double cfl, double *dt_out);
int dgw_set_dt(dgw_ctx *ctx, double dt);

/* Point source of shot `shot`: position xyz[3], moment tensor moment[6] in
 * the order (xx, yy, zz, yz, xz, xy) (NULL = explosion, the identity), Ricker
 * parameters f0, t0, amp; nsteps = the shot's length in steps (<= 0: no
 * limit).  The delta is projected as (1/J) M^-1 l(r_s) onto the element that
 * contains xyz (lowest element id among those whose barycentrics are all
 * >= -1e-12; DGW_ERANGE when outside the mesh). */
int dgw_set_source(dgw_ctx *ctx, int shot, const double *xyz,
                   const double *moment, double f0, double t0, double amp,
                   int64_t nsteps);

/* Receivers of shot `shot`: xyz [nrec][3] located like the source; the trace
 * buffer holds max_samples steps ([nrec][3][max_samples] velocities); a step
 * that would exceed it makes dgw_step return DGW_ERANGE without stepping.
 * Setting receivers clears the shot's traces. */
int dgw_set_receivers(dgw_ctx *ctx, int shot, int nrec, const double *xyz,
                      int64_t max_samples);

/* Replace (set) or read (get) the fields of one shot, host layout
 * q[K][9][Np] FP64 (converted for FP32 contexts).  dgw_set_fields also resets
 * the shot's step counter and time to zero and clears its traces. */
int dgw_set_fields(dgw_ctx *ctx, int shot, const double *q);
int dgw_get_fields(dgw_ctx *ctx, int shot, double *q);

/* Resume a shot at its own time: set its step counter to `step` (time
 * step * dt for the source and the trace index), after dgw_set_fields has
 * loaded the state saved at that step.  The shot's traces before `step` stay
 * as dgw_set_fields left them (zero); the next dgw_step records from `step`
 * on.  Memory variables of a perfectly matched layer restart at zero with
 * dgw_set_fields; dgw_set_pml_memory restores them.  DGW_ERANGE for a shot out of range, a
 * negative step, or a step beyond the shot's length. */
int dgw_set_shot_step(dgw_ctx *ctx, int shot, int64_t step);

/* Advance every shot that has steps left by up to nsteps steps (a shot stops
 * at its length).  Each step is five fused RHS + LSERK stage launches and one
 * receiver-sampling launch; batches of steps are replayed from a captured
 * HIP graph. */
int dgw_step(dgw_ctx *ctx, int64_t nsteps);

/* Copy the recorded traces of one shot into out [nrec][3][cap] (the first n
 * samples of each row are valid); *n = samples recorded so far. */
int dgw_read_traces(dgw_ctx *ctx, int shot, double *out, int64_t cap,
                    int64_t *n);

/* Steps taken so far by a shot. */
int dgw_shot_steps(dgw_ctx *ctx, int shot, int64_t *steps);

/* Discrete energy of one shot,
 * E = 1/2 sum_k J_k [rho v^T M v + sigma^T (S (x) M) sigma] with S the
 * isotropic compliance (fluid elements: tr^T M tr / (9 lambda) in place of
 * the stress term), accumulated in FP64 on the device. */
int dgw_energy(dgw_ctx *ctx, int shot, double *E);

/* dgw_energy without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid it).  Same quantity and arguments as dgw_energy; its partial
 * sums live in a static device array of the library (one per GPU, 65537
 * doubles, held until the process ends), so it supports meshes of at most
 * 16,777,216 elements (DGW_ERANGE beyond).  It allocates nothing and frees
 * nothing; it enqueues two kernels and an 8-byte copy on the context's
 * stream and synchronizes it.  Calls that overlap on one GPU (from several
 * threads or contexts) share the array and race: serialize them. */
int dgw_energy_noalloc(dgw_ctx *ctx, int shot, double *E);

/* DGW_ENONFINITE if any field value of any shot is NaN or infinite. */
int dgw_check_finite(dgw_ctx *ctx);

/* Step watchdog: with every > 0, dgw_step checks the fields after every
 * `every` steps it runs (counted across calls): a NaN or infinite value in
 * any shot stops the call with DGW_ENONFINITE, and with max_growth > 0 a
 * shot whose discrete energy (dgw_energy) exceeds max_growth times its
 * energy at the previous check stops it with DGW_EGROWTH; the message names
 * the shot and its step.  The steps before the check have been taken (the
 * fields stay readable).  A shot's energy baseline restarts when its fields
 * are set; a baseline of zero (a shot at rest) is never exceeded.  The
 * steps themselves are unchanged (results are identical with the watchdog
 * on or off); each check synchronises the stream and costs one reduction
 * per shot.  every = 0 turns it off.  DGW_EINVAL for every < 0, or
 * max_growth negative, not finite, or in (0, 1). */
int dgw_set_watchdog(dgw_ctx *ctx, int64_t every, double max_growth);

/* Reference element of order N (host only, no context needed):
 * rst [Np][3] node coordinates; Dr, Ds, Dt [Np][Np] (d l_n / dr at node i in
 * row i, column n); M [Np][Np] the reference mass matrix (volume 4/3);
 * LIFT [Np][4 Nfp] = M^-1 [E_0 .. E_3] with E_f the face mass matrix divided
 * by the reference face area.  Any output pointer may be NULL. */
int dgw_ref_nodes(int order, double *rst);
int dgw_ref_operators(int order, double *Dr, double *Ds, double *Dt,
                      double *M, double *LIFT);

/* Element ordering for gather locality (host only, no context needed).  The
 * stage kernel works on blocks of consecutive elements and gives each XCD a
 * contiguous range of blocks, so face neighbours close in the numbering are
 * read from the same L2; this returns a numbering that keeps them close.
 * perm [K] receives a permutation of 0..K-1: element i of the reordered mesh
 * is input element perm[i].  The caller applies it to etov, face_bc, the
 * per-element material and the fields before dgw_set_mesh (vertices are
 * unchanged).
 *   DGW_ORDER_MORTON: Morton (Z-order) curve of the element centroids,
 *     21 bits per axis over the centroids' bounding box, bits interleaved
 *     x, y, z from the least significant end, ties by input index;
 *   DGW_ORDER_RCM: reverse Cuthill-McKee (Cuthill and McKee 1969, reversed
 *     as by George 1971) on the face-adjacency graph, faces matched by their
 *     sorted vertex triples with vertex_periodic_id as in dgw_set_mesh (may
 *     be NULL); each connected component starts from an element of minimum
 *     degree (ties by index), neighbours are queued by increasing degree
 *     then index, and the breadth-first sequence is reversed.
 * Deterministic.  DGW_EINVAL for null pointers, K or nvert <= 0, a vertex id
 * outside [0, nvert) or an unknown method; DGW_EMESH (RCM) for a degenerate
 * face or a vertex triple shared by more than two faces. */
#define DGW_ORDER_MORTON 0
#define DGW_ORDER_RCM 1
int dgw_order_elements(int64_t nvert, const double *vxyz, int64_t K,
                       const int32_t *etov, const int32_t *vertex_periodic_id,
                       int method, int64_t *perm);

/* Differentiation (upwind flux only: DGW_ESTATE unless the flux weight of
 * dgw_set_flux is 1).  dgw_forward_checkpointed runs every shot from its current
 * state for nsteps steps, storing the state every ckpt_every steps in device
 * memory, and returns the misfit of each shot against d_obs
 * [nshots][nrec][3][nsteps] (misfit [nshots], accumulated in FP64).
 * dgw_adjoint then computes, by the exact discrete adjoint with forward
 * recomputation between checkpoints, the gradients of each shot's misfit with
 * respect to rho, lambda, mu: g_* [nshots][K] FP64. */
int dgw_forward_checkpointed(dgw_ctx *ctx, int64_t nsteps, int64_t ckpt_every,
                             const double *d_obs, double *misfit);
int dgw_adjoint(dgw_ctx *ctx, double *g_rho, double *g_lam, double *g_mu);

/* State generation: a counter the context bumps on every call that changes
 * what a run computes (dgw_set_material, dgw_set_dt, dgw_set_source,
 * dgw_set_receivers, dgw_set_fields, dgw_set_damping, dgw_set_flux,
 * dgw_set_stiffness, dgw_set_pml, and dgw_step when it advances a shot).
 * dgw_forward_checkpointed records the value it ends at, and dgw_adjoint
 * returns DGW_ESTATE when the counter has moved since, because the reverse
 * sweep reads the traces, material, time step and tables of the live
 * context.  Callers that keep several forwards apart compare the value
 * themselves.  *gen receives the current value. */
int dgw_state_generation(const dgw_ctx *ctx, uint64_t *gen);

/* Device memory the reverse sweep of dgw_adjoint may spend on keeping the
 * inner stage states of a checkpoint segment (ckpt_every x 4 states of all
 * shots): within the budget, the states the segment's recomputation
 * produces are kept and each reverse step reads them; otherwise each
 * reverse step recomputes its four inner stages from the step start.  The
 * results are identical either way.  bytes = -1 (the default) takes a
 * quarter of the free device memory at the call; 0 never keeps them.
 * DGW_EINVAL for bytes < -1. */
int dgw_set_adjoint_memory(dgw_ctx *ctx, int64_t bytes);

/* Time the available launch shapes of the stage kernel on this context's
 * workload (real stage launches into scratch buffers; the solver state is not
 * changed) and keep the fastest; if cache_path is not NULL the choice is read
 * from / written to that JSON file (keyed by order, precision, element count
 * and shot count).  The chosen shape is returned through the two pointers
 * (either may be NULL); see dgw_set_launch. */
int dgw_autotune(dgw_ctx *ctx, const char *cache_path, int *kernel,
                 int *elems_per_block, int *wgs_per_cu);

/* Face flux.  The flux states are tau (t*, v*) + (1 - tau) ((t- + t+)/2,
 * (v- + v+)/2): tau = 1 (the default) is the exact Riemann (upwind) flux,
 * tau = 0 the central flux, values between a convex combination (the
 * alpha-flux family of Hesthaven and Warburton 2008, section 2.2, with
 * alpha = 1 - tau; boundary ghost states as for the upwind flux).  The
 * central flux conserves the semi-discrete energy on meshes without
 * boundaries.  DGW_EINVAL outside [0, 1].  dgw_forward_checkpointed and
 * dgw_adjoint return DGW_ESTATE unless tau = 1. */
int dgw_set_flux(dgw_ctx *ctx, double tau);

/* Absorbing sponge layer: per-element damping rate sigma [K] (finite,
 * >= 0; NULL removes it).  The right-hand side of element k gains
 * -sigma_k q on all nine fields (the damping layer of Cerjan, Kosloff,
 * Kosloff and Reshef, Geophysics 50, 1985), so the energy falls by
 * 2 sum_k sigma_k E_k per unit time on top of the flux's own dissipation;
 * dgw_adjoint includes it exactly.  Requires the mesh (DGW_ESTATE);
 * DGW_EINVAL for negative or non-finite rates. */
int dgw_set_damping(dgw_ctx *ctx, const double *sigma);

/* Convolutional perfectly matched layer (the recursive-convolution PML of
 * Roden and Gedney, 2000, in the unsplit first-order form of Komatitsch and
 * Martin, Geophysics 72, 2007, stretching factor 1).  In the layer every
 * derivative d/dx_b gains a memory variable m, m_t = -(d_b + alpha_b) m -
 * d_b du/dx_b: per node, phi_cb for D_cb = d sigma_cb / dx_b and psi_cb for
 * G_cb = d v_c / dx_b (c, b = x, y, z), and the right-hand side gains
 * (1/rho) sum_b phi_cb on v_c and lambda tr(Psi) I + mu (Psi + Psi^T) on
 * sigma.  D and G are the scheme's own derivatives split by axis (volume part
 * and the lifted flux-state change times n_b, the traction change dT extended
 * to the symmetric stress change dT n^T + n dT^T - (n.dT) n n^T), so that
 * with d = 0 the step is the plain scheme's.  Memory variables advance with
 * the same LSERK4 stages.
 *   n          layer elements (0 removes the layer; elements and profile
 *              may then be NULL)
 *   elements   [n] element ids, strictly increasing
 *   profile    [n][6][Np] per node: d_x, d_y, d_z, alpha_x, alpha_y, alpha_z
 *              (finite, >= 0; copied)
 * Memory variables start at zero here and whenever dgw_set_fields sets a
 * shot.  Isotropic elements only: DGW_ESTATE with a stiffness set (and
 * dgw_set_stiffness refuses while a layer is set); dgw_forward_checkpointed
 * and dgw_adjoint return DGW_ESTATE while a layer is set.  DGW_ERANGE for an
 * element id out of range, DGW_EINVAL for unsorted ids or a negative or
 * non-finite profile value.  Device memory: 2 x nshots x n x 18 x Np reals
 * plus the profile. */
int dgw_set_pml(dgw_ctx *ctx, int64_t n, const int32_t *elements, const double *profile);

/* The layer's memory variables of one shot, out [n][18][Np] FP64 (phi_cb at
 * 3 c + b, psi_cb at 9 + 3 c + b).  DGW_ESTATE without a layer. */
int dgw_get_pml_memory(dgw_ctx *ctx, int shot, double *out);

/* Restore a shot's memory variables (the layout of dgw_get_pml_memory, FP64,
 * copied; rounded to FP32 in the FP32 form): with dgw_set_fields and
 * dgw_set_shot_step, a run with a layer resumes exactly where it was saved.
 * Call it after dgw_set_fields, which restarts them at zero.  DGW_ESTATE
 * without a layer, DGW_EINVAL for non-finite values. */
int dgw_set_pml_memory(dgw_ctx *ctx, int shot, const double *in);

/* Average duration of the layer kernel launches of the last timed dgw_step
 * (dgw_enable_timing), and how many were timed. */
int dgw_pml_kernel_ms(dgw_ctx *ctx, double *ms, int64_t *launches);

/* Anisotropic elements: per-element Voigt stiffness C [K][21], the upper
 * triangle row by row (C11 C12 .. C16 C22 .. C66) in the order xx, yy, zz,
 * yz, xz, xy with engineering shear strains; each C symmetric positive
 * definite (DGW_EINVAL otherwise, or for non-finite values; the previous
 * state is kept).  It replaces lambda and mu of dgw_set_material (rho
 * stays): stress rate C e(v); at faces the exact Riemann states from the
 * impedance matrices Z = (rho N(n)^T C N(n))^(1/2) of both sides,
 * v* = (Z- + Z+)^-1 (Z- v- + Z+ v+ + t+ - t-), t* = t- + Z- (v* - v-)
 * (N(n) maps a vector to the Voigt strain of its symmetric product with n;
 * for isotropic C these are the isotropic states), blended with the central
 * flux as set by dgw_set_flux; stress flux C N(n) dv.  Energy: the potential
 * term uses the compliance C^-1.  dgw_suggest_dt uses the largest
 * Christoffel speed over 258 sampled directions.  Both stage kernels
 * have an anisotropic form; dgw_forward_checkpointed and dgw_adjoint are
 * DGW_ESTATE.  A later dgw_set_material recomputes the impedances from the
 * new rho.  NULL returns to isotropic elements.  Requires the mesh and the
 * material (DGW_ESTATE).  Host data are copied. */
int dgw_set_stiffness(dgw_ctx *ctx, const double *C);

/* Launch shape of the stage kernel.  kernel 0: one thread per (element,
 * node) with the block's fields and lifted fluxes staged in LDS; then
 * elems_per_block is the elements per work-group (0 = default; DGW_EINVAL for
 * values the kernel does not implement) and wgs_per_cu the work-groups per
 * compute unit of a persistent grid (0 = one work-group per block of
 * elements, the default; 1..64 = a persistent grid of that many work-groups
 * per CU, rounded up to a multiple of 8, looping over the blocks of all
 * shots).  Kernel variants other than 0 that this build does not provide
 * for the context's order and precision give DGW_EINVAL. */
int dgw_set_launch(dgw_ctx *ctx, int kernel, int elems_per_block, int wgs_per_cu);

/* Average duration in milliseconds of the stage-kernel launches made by the
 * last dgw_step call, measured with HIP events on the context's stream
 * (0 if none was timed); enable with dgw_enable_timing(ctx, 1). */
int dgw_enable_timing(dgw_ctx *ctx, int on);
int dgw_stage_kernel_ms(dgw_ctx *ctx, double *ms, int64_t *launches);

/* Average duration in milliseconds of one reverse (adjoint) stage -- its two
 * kernel launches -- over the first (at most 200) reverse stages of the last
 * dgw_adjoint call made with timing enabled, from HIP events on the
 * context's stream; *stages receives how many were timed (0: none). */
int dgw_adjoint_stage_ms(dgw_ctx *ctx, double *ms, int64_t *stages);

/* Sizes: Np = (N+1)(N+2)(N+3)/6 and Nfp = (N+1)(N+2)/2 of the context. */
int dgw_sizes(const dgw_ctx *ctx, int *Np, int *Nfp, int64_t *K);

#ifdef __cplusplus
}
#endif
#endif /* DGW_H */

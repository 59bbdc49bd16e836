// Internal declarations shared by the host setup, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#define DGW_MAX_ORDER 6
#define DGW_META 48   // doubles of per-element data (see MetaLayout)
#define DGW_ANI 120   // doubles of per-element anisotropic data (see AniLayout)

namespace dgw {

// Per-element data, FP64, DGW_META doubles per element:
//   [0..8]   X^-1 row-major (rx ry rz sx sy sz tx ty tz)
//   [9..12]  Fscale_f = A_f / J
//   [13..24] outward unit normals n_f (x, y, z)
//   [25] 1/rho  [26] lambda  [27] mu  [28] Zp  [29] Zs
//   [30..33] Zp of the neighbour across face f (own Zp on boundary faces)
//   [34..37] Zs of the neighbour
//   [38..41] 1 / (Zp + Zp_nb)   [42..45] 1 / (Zs + Zs_nb)
//   [46] J   [47] unused
enum MetaLayout {
  M_XINV = 0, M_FSCALE = 9, M_NORMAL = 13, M_RHOINV = 25, M_LAM = 26,
  M_MU = 27, M_ZP = 28, M_ZS = 29, M_ZPNB = 30, M_ZSNB = 34, M_IZPS = 38,
  M_IZSS = 42, M_J = 46
};

// Per-element data of anisotropic elements, FP64, DGW_ANI doubles per
// element (only when a stiffness is set):
//   [0..20]   Voigt stiffness C (order xx yy zz yz xz xy, engineering
//             shears), upper triangle row by row: C11 C12 .. C16 C22 .. C66
//   [21 + 18 f ...] face f: Z- = (rho N^T C N)^(1/2) (own impedance matrix),
//             W = (Z- + Z+)^-1, Z+ (the neighbour's, with the own normal;
//             Z- on boundary faces); each symmetric 3x3 stored as
//             (xx, yy, zz, yz, xz, xy)
//   [93..113] Voigt compliance C^-1, upper triangle
//   [114..119] unused
enum AniLayout { A_C = 0, A_FACE = 21, A_FSTRIDE = 18, A_ZM = 0, A_W = 6, A_ZP = 12,
                 A_S = 93 };

// Packed face connectivity (int32 per element face): interior faces hold
// (neighbour << 5) | (neighbour face << 3) | orientation (0..5); boundary
// faces hold -1 (free surface) or -2 (absorbing).
constexpr int CONN_FREE = -1;
constexpr int CONN_ABSORB = -2;

struct RefElem {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<int> bary;   // [Np][4]
  std::vector<int> fmask;  // [4][Nfp]
  std::vector<double> rst, Dr, Ds, Dt, M, Minv, LIFT;
};

bool build_refelem(int N, RefElem &R);
void eval_basis(const RefElem &R, const double rst[3], double *out);

struct MeshData {
  int64_t K = 0;
  std::vector<double> vxyz;      // [nvert][3]
  std::vector<int32_t> etov;     // [K][4]
  std::vector<double> geo;       // [K][DGW_META] geometry part filled
  std::vector<int32_t> conn;     // [K][4]
  std::vector<int32_t> nbtab;    // [4][4][6][Nfp] neighbour volume node
  std::vector<int32_t> nbface;   // [4][4][6][Nfp] neighbour face-local node
  std::vector<uint8_t> nbnode;   // [K][4][Nfp] neighbour volume node (interior faces)
  std::vector<uint8_t> nbfnode;  // [K][4][Nfp] neighbour face node f2 Nfp + m2
  std::vector<double> volume;    // [K]
  std::vector<double> area;      // [K][4]
};

// Returns an empty string on success, else the reason.
std::string build_mesh(const RefElem &R, int64_t nvert, const double *vxyz,
                       int64_t K, const int32_t *etov, const int32_t *pid,
                       const int8_t *face_bc, MeshData &out);
// Element containing x (lowest id), reference coordinates; -1 if outside.
int64_t locate_point(const MeshData &m, const double x[3], double rst[3]);

// ---- device side -------------------------------------------------------

template <typename real>
struct StageArgs {
  const real *q_in;
  real *q_out;
  real *res;
  const double *meta;
  const int32_t *conn;
  const uint8_t *nbnode;        // [K][4 Nfp] neighbour volume node per face node
  const real *DrT, *DsT, *DtT;  // [j][i] (transposed)
  const real *LIFTT;            // [4Nfp][Np] (transposed)
  // operator fragments in MFMA lane order (stage kernel variant 1):
  // Avol[a][ks][mt][64] = D_a[16 mt + l % 16][4 ks + l / 16],
  // Alift[ks][mt][64] = LIFT[16 mt + l % 16][4 ks + l / 16], zero-padded
  const real *Avol, *Alift;
  // per-face lift fragments of the minimal-form kernel (kernel 2):
  // Alf[f][ks][mt][64] = c_f LIFT[16 mt + l % 16][f Nfp + 4 ks + l / 16] for
  // 4 ks + l / 16 < Nfp, else 0; c_0 = 2, c_1 = c_2 = c_3 = -2
  const real *Alf;
  const int32_t *fmask;         // [4 Nfp]
  int64_t K;
  int64_t shot_stride;          // K * 9 * Np
  // shot of each launched slot [slots], or null: slot s is shot s.  The
  // launch covers `nshots` slots (the launchers' argument), so a batch whose
  // finished shots are left out launches only the active shots' blocks.
  const int32_t *shot_map;
  const int64_t *shot_step;     // [S]
  const int64_t *shot_len;      // [S]
  const int32_t *src_elem;      // [S] (-1: none)
  const double *src_vec;        // [S][Np]
  const double *src_par;        // [S][10]: moment[6], f0, t0, amp, unused
  real ftau;                    // weight of the upwind flux (1 - ftau: central)
  const double *sponge;         // [K] damping rate, or null
  const double *aniso;          // [K][DGW_ANI] anisotropic data, or null
  double rk_a, rk_b, rk_c, dt;
};

// Perfectly matched layer launch (pml.hip), after the stage kernel of the
// same stage: the layer's nP elements `elem` (strictly increasing), their
// per-node profile prof[p][6][Np] = (d_x, d_y, d_z, alpha_x, alpha_y,
// alpha_z), memory variables mem[S][nP][18][Np] (phi_cb at 3 c + b, psi_cb
// at 9 + 3 c + b) and their stage residual mres (same layout).
template <typename real>
struct PmlArgs {
  const real *q_in;
  real *q_out;
  real *res;
  real *mem, *mres;
  const int32_t *elem;
  const double *prof;
  const double *meta;
  const int32_t *conn;
  const uint8_t *nbnode;
  const real *DrT, *DsT, *DtT, *LIFTT;
  const int32_t *fmask;
  int64_t nP;
  int64_t shot_stride;          // K * 9 * Np
  int64_t mem_stride;           // nP * 18 * Np
  const int32_t *shot_map;      // as in StageArgs
  const int64_t *shot_step;
  const int64_t *shot_len;
  real ftau;
  double rk_a, rk_b, dt;
};

hipError_t launch_pml(int N, int precision, int nshots, const void *args, hipStream_t st);

// A contiguous span of `cnt` values at element offset `off` of a
// 16-byte-aligned array, split for 16-byte vector access: `hd` scalars up
// to the first aligned address, `nv` vectors of VW values, `tl` scalars.
template <typename real>
struct Span16 {
  static constexpr int VW = 16 / (int)sizeof(real);
  typedef real vec __attribute__((ext_vector_type(VW)));
  int hd, nv, tl;
  __device__ Span16(int64_t off, int cnt) {
    const int mis = (int)(off % VW);
    hd = (VW - mis) % VW;
    if (hd > cnt) hd = cnt;
    nv = (cnt - hd) / VW;
    tl = cnt - hd - nv * VW;
  }
};

struct RecArgs {
  const void *q;                // current state (real)
  int64_t shot_stride;
  int Np;
  const int32_t *nrec;          // [S]
  int rmax;
  const int32_t *rec_elem;      // [S][rmax]
  const double *rec_w;          // [S][rmax][Np]
  double *trace;                // [S][rmax][3][cap]
  int64_t cap;
  int64_t *shot_step;
  const int64_t *shot_len;
};

// Reverse (adjoint) stage.  w = lam_r + b lam_q is the adjoint of the stage's
// residual; lam_q += dt L^T w, lam_r = a w, grad += dt (d(L q)/dm)^T w.
template <typename real>
struct AdjArgs {
  const real *q;                // stage input state
  real *lam_q, *lam_r;          // adjoint of q and of res
  real *zbuf;                   // [S][K][7][4 Nfp] combinations of Fscale LIFT^T w
  // with lift_next set, the main kernel also forms the next reverse stage's
  // lifted adjoint from its updated lam_r + next_b lam_q into zbuf_next
  real *zbuf_next;
  double next_b;
  int lift_next;
  double *grad;                 // [S][K][3] (rho, lambda, mu)
  const double *meta;
  const int32_t *conn;
  const uint8_t *nbnode;        // [K][4 Nfp] neighbour volume node per face node
  const uint8_t *nbfnode;       // [K][4 Nfp] neighbour face node f2 Nfp + m2
  const real *DrT, *DsT, *DtT;  // [j][i] = D(i, j)
  const real *Dr, *Ds, *Dt;     // [j][i] = D(j, i)
  const real *LIFT;             // [Np][4 Nfp]
  const int32_t *fmask;         // [4 Nfp]
  const int32_t *facepos;       // [4][Np]: face-local index or -1
  const double *sponge;         // [K] damping rate, or null
  int64_t K;
  int64_t shot_stride;
  const int32_t *shot_map;      // shot of each launched slot, or null (as in StageArgs)
  const int64_t *shot_step;
  const int64_t *shot_len;
  double rk_a, rk_b, dt;
};

// Launchers (adjoint_kernels.hip); nshots is the number of launched slots.
// lift: launch the lift kernel first (else zbuf already holds the stage's
// lifted adjoint, formed by the previous stage's main kernel)
hipError_t launch_adjoint_stage(int N, int precision, int nshots,
                                const void *args, bool lift, hipStream_t st);
// lam_q[k_r][c][j] += dt w_r[j] (trace[r][c][step] - d_obs[r][c][step])
hipError_t launch_inject(int precision, int nshots, int Np, void *lam_q,
                         int64_t shot_stride, const int32_t *nrec, int rmax,
                         const int32_t *rec_elem, const double *rec_w,
                         const double *trace, int64_t cap, const double *d_obs,
                         int64_t nobs, const int64_t *shot_step,
                         const int64_t *shot_len, double dt, hipStream_t st);
hipError_t launch_set_steps(int64_t *steps, int nshots, int64_t value,
                            hipStream_t st);

// Launchers (kernels.hip); return the launch error.
// kernel 0 (one thread per element node on the vector ALUs), 1 (the
// volume and lift contractions as one GEMM on the matrix cores), both with
// 256 threads per work-group, with args.aniso set each running its
// anisotropic form, or 2 (the minimal-form matrix-core kernel of
// stage_split.hip; isotropic only): be = elements per work-group,
// wpc = persistent work-groups per compute unit (0: one work-group per block
// of elements).  ncu = compute units.
hipError_t launch_stage(int kernel, int N, int precision, int be, int wpc,
                        int ncu, int nshots, const void *args, hipStream_t st);
bool stage_kernel_supported(int kernel, int N, int precision);
// Kernel 2 (stage_split.hip): the minimal-form matrix-core kernel, 16
// elements per work-group, isotropic elements only, orders 1-4 in FP64 and
// 1-6 in FP32.
bool stage_split_supported(int N, int precision);
int stage_split_block();
hipError_t launch_stage_split(int N, int precision, int nshots, const void *args,
                              hipStream_t st);
hipError_t launch_receivers(int precision, int nshots, const RecArgs &a,
                            hipStream_t st);
// aniso: [K][DGW_ANI] or null (isotropic elements)
hipError_t launch_energy(int precision, const void *q, int64_t K, int Np,
                         const double *meta, const double *aniso, const double *M,
                         double *partial, int nblocks, hipStream_t st);
hipError_t launch_finite(int precision, const void *q, int64_t n, int *flag,
                         hipStream_t st);
// Supported elements-per-block values for an order / precision.
std::vector<int> stage_block_choices(int kernel, int N, int precision);
int default_block(int kernel, int N, int precision);

}  // namespace dgw

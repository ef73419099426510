// Kernel argument structs and launchers (host side) of the TFETI library.
#pragma once

#include "tfeti_internal.h"

namespace tfeti {

struct MatC {
  double lam, mu, sy, H;
};

struct AssembleArgs {
  const SubDev* subs;
  const int32_t* elems;       // elements of one parity class
  int64_t n_colour;
  const int32_t* elem_sub;
  const double* dN;           // [8 gp][8 node][3 axis]
  double w;                   // Gauss weight times det J
  MatC M;
  const double* du;           // torn displacement increment
  const double* sigma;        // committed stress (n_gp * 6)
  const double* kappa;        // committed hardening (n_gp)
  double* dsigma;
  double* dkappa;
  uint8_t* plastic;
  unsigned long long* plastic_count;
  double* fint;               // torn internal force (accumulated)
  double* band;               // row-band tangent (accumulated)
  const uint8_t* need;        // subdomains whose tangent is assembled (mode 2)
};

void launch_return_map(const tfeti_material& mat, int64_t npts, const double* sig, const double* kap,
                       const double* de, double* ds, double* dk, double* Dt, uint8_t* pl, hipStream_t st);
// mode 1: return map, increments, internal force; mode 2: tangent of need[]
void launch_assemble(const AssembleArgs& args, int mode, hipStream_t st);
void launch_pad_identity(const SubDev* subs, int64_t nsub, const int32_t* list, double* band, hipStream_t st);
// list: subdomain indices (count of them), or NULL for subdomains 0 .. count-1
void launch_regularize(const SubDev* subs, int64_t count, const int32_t* list, const double* QQt, double* band,
                       hipStream_t st);
void launch_sub_plastic(const SubDev* subs, int64_t nsub, const uint8_t* plastic, int32_t* flags, hipStream_t st);
// src NULL: zero fill
void launch_copy_band(const SubDev* subs, int64_t count, const int32_t* list, const double* src, double* dst,
                      hipStream_t st);

// ---- solve panels ----------------------------------------------------------
// Panel geometry of one subdomain for tile TS (rows of a block row).
// Forward panel of block row I: off-diagonal columns [I TS - wF, I TS), wF =
// min(I TS, bo), then the inverted diagonal tile; chunk (cc, r) of V
// consecutive columns of row r is stored at (cc TS + r) V.  Backward panel
// of block column I: the inverted diagonal tile rows first, then rows
// [(I+1) TS, (I+1) TS + wB), wB = min(n - (I+1) TS, bo); chunk (rc, c) of V
// consecutive rows of column c is stored at (rc TS + c) V.  The offsets are
// the sums of the panel sizes TS (w + TS) of the block rows before I.
__host__ __device__ inline int64_t panel_fwd_offset(int64_t I, int64_t TS, int64_t bo) {
  const int64_t kF = (bo + TS - 1) / TS;  // block rows with I TS < bo
  const int64_t m1 = I < kF ? I : kF;
  return TS * (TS * m1 * (m1 - 1) / 2 + (I - m1) * bo + I * TS);
}
__host__ __device__ inline int64_t panel_bwd_offset(int64_t I, int64_t TS, int64_t bo, int64_t n) {
  int64_t K = n >= bo ? (n - bo) / TS : 0;  // block columns whose width is bo
  K = K < I ? K : I;
  return TS * (I * TS + K * bo + (I - K) * n - TS * (I * (I + 1) - K * (K + 1)) / 2);
}
// Column j of X = L^{-1} for the lower-triangular tile d (ts x ts, row
// stride ld): X[i][j] (i > j) goes to d[j][i], the tile's strict upper
// triangle, and X[j][j] = 1 / L[j][j] to xd[j].  One thread per column.
__device__ inline void tile_inverse_column(double* d, int ld, int ts, int j, double* xd) {
  const double xjj = 1.0 / d[j * ld + j];
  xd[j] = xjj;
  for (int i = j + 1; i < ts; ++i) {
    double v = d[i * ld + j] * xjj;
    for (int k = j + 1; k < i; ++k) v = fma(d[i * ld + k], d[j * ld + k], v);
    d[j * ld + i] = -v / d[i * ld + i];
  }
}

// ---- sparse rows -----------------------------------------------------------
// sum over e in [e0, e1) of coef[e] * fetch(idx[e]), in order of e (e1 > e0):
// the first K entries' loads are issued together with clamped indices (every
// load unconditional, one chain of dependent loads instead of one per entry),
// the rest one by one.  fetch(i) returns the vector value at index i.
template <int K, typename E, typename I, typename F>
__device__ __forceinline__ double seg_dot(E e0, E e1, const I* __restrict__ idx, const double* __restrict__ coef,
                                          F fetch) {
  I ii[K];
  double cc[K], xx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const E e = e0 + k < e1 ? e0 + k : e1 - 1;
    ii[k] = idx[e];
    cc[k] = coef[e];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) xx[k] = fetch(ii[k]);
  double s = cc[0] * xx[0];
#pragma unroll
  for (int k = 1; k < K; ++k)
    if (e0 + k < e1) s = fma(cc[k], xx[k], s);
  for (E e = e0 + K; e < e1; ++e) s = fma(coef[e], fetch(idx[e]), s);
  return s;
}

// ---- factorization -------------------------------------------------------
// In-place band Cholesky of every subdomain's row-band matrix (type T).
// bmax: largest half bandwidth; nb: block columns (0 = largest that fits LDS).
template <typename T>
int launch_band_cholesky(const SubDev* subs, int64_t nsub, const int32_t* list, T* band, int32_t* fail, int bmax,
                         int nb, hipStream_t st);
int band_cholesky_nb(int bmax, size_t elem);
// Pack the factors into forward (F) and backward (B) panels with inverted
// diagonal tiles (layout above).
// (factor in TW, panels in T; both FP64 in this library); Fq, Bq
// (optional): FP32 copies of the panels written in the same pass
template <typename TW, typename T>
void launch_pack_panels(const SubDev* subs, int64_t count, const int32_t* list, const TW* band, T* Fp, T* Bp, int TS,
                        hipStream_t st, float* Fq = nullptr, float* Bq = nullptr);
// Dense inverse of the coarse matrix from its banded Cholesky factor.
// Lt: scratch for the transposed factor (l * Wc entries), or NULL.
void launch_coarse_inverse(const double* L, int32_t l, int32_t b, int32_t Wc, double* Ginv, hipStream_t st,
                           double* Lt);

// ---- subdomain solves -----------------------------------------------------
template <typename T>
struct KsolveArgs {
  const SubDev* subs;
  const int32_t* order;       // schedule: workgroup -> subdomain
  int64_t nsub;
  const T* Fp;
  const T* Bp;
  const double* in_full;      // torn input or nullptr
  const double* lam;          // multipliers for B^T lam or nullptr
  double lam_sign;            // x += lam_sign * B^T lam
  double* out_iface;          // z at touched DOFs or nullptr
  double* out_full;           // torn output or nullptr
  const double* alpha;        // adds R alpha to out_full if not nullptr
  const double* R_full;
  const int32_t* if_fidx;
  const int32_t* if_ldof;
  const int32_t* if_rp;
  const int32_t* if_row;
  const double* if_coef;
  const int32_t* done;        // skip when *done != 0 (nullptr: never)
  const double* lam2;         // a second right-hand side in_full + lam_sign B^T lam2, or nullptr
  double* out_iface2;         // its z at the touched DOFs (with lam2)
  int32_t vec_stride;         // LDS entries per right-hand side; set by the launcher
  PcgFold fold;               // fold.S: lam is p, taken as fma(beta, p, fold.y)
  // explicit local operators applied instead of the solve to the subdomains
  // with xuse[p] != 0 (nullptr: none): their storage (type T), offsets and
  // sorted touched DOFs; x_mp: the largest 16 ceil(m_p / 16)
  const uint8_t* xuse;
  const void* xF;
  const int64_t* xfoff;
  const int32_t* xsit;
  int32_t x_mp;
};
template <typename T>
void launch_ksolve(const KsolveArgs<T>& a, int TS, int threads, int npad_max, hipStream_t st);

// ---- dual-space kernels (FP64) ---------------------------------------------
struct DualMaps {
  int64_t m, n_iface, nsub, l;
  const SubDev* subs;
  const int64_t* b_rowptr;
  const int32_t* b_iface;
  const double* b_val;
  const int32_t* if_rp;
  const int32_t* if_row;
  const double* if_coef;
  const uint32_t* if_pk;       // packed centred node coordinates per B^T entry
  const int32_t* b_sub;        // subdomain per B entry
  const uint32_t* b_pk;        // packed centred node coordinates per B entry
  const double* rscale;        // 4 per subdomain: inverse norms of the raw rigid modes
  double hh[3];                // half element edge lengths
  const double* R_full;
  const int32_t* if_ldof;      // local natural DOF of each touched DOF
  // K_bb in wavefront groups of 64 touched DOFs (lane slot = 64 group + lane)
  const int32_t* kbb_row;      // touched DOF of each lane slot, -1 past the end
  const uint32_t* kbb_mask;    // its touched nodes among the 27 around its node
  const int32_t* kbb_node;     // its node (local natural index)
  const int64_t* kbb_goff;     // value offset of each group
  const int32_t* kbb_gnb;      // neighbour blocks of each group (values 3 x 64 per block)
  const int32_t* kbb_gsub;     // subdomain of each group
  const int32_t* kbb_g0;       // first group of each subdomain (nsub + 1)
  int64_t kbb_groups;
  const double* Ginv;          // dense (G G^T)^{-1}, l x l (setup only)
  const double* Gpk;           // its lower 64 x 64 tiles, packed (coarse solves)
  double* Gpart;               // per-tile partial products, ceil(l/64) x roundup(l, 64)
  int32_t max_ndof;           // largest subdomain DOF count (LDS of the preconditioner)
};

// out[r] = sum_e b_val[e] * iface[b_iface[e]]; if dotv: partial sums of out.dotv
void launch_gather(const DualMaps& M, const double* iface, double* out, const double* dotv, double* partials,
                   const int32_t* done, hipStream_t st, const PcgFold& fold = PcgFold{});
// c[6p+j] = sum_t R_iface[t][j] (B^T w)_t   (G w)
void launch_g_apply(const DualMaps& M, const double* w, double* c, const int32_t* done, hipStream_t st,
                    const PcgFold& fold = PcgFold{});
// c[6p+j] = sum_ld R_full[ld][j] f[ld]       (R^T f)
void launch_rt_apply(const DualMaps& M, const double* f, double* c, hipStream_t st);
// u = z + R alpha per subdomain (torn vectors; alpha 6 per subdomain)
void launch_add_rigid(const DualMaps& M, const double* z, const double* alpha, double* u, hipStream_t st);
// a = scale * Ginv c
void launch_coarse_gemv(const DualMaps& M, const double* c, double* a, double scale, const int32_t* done,
                        hipStream_t st);
// tiles of the packed lower triangle of an l x l symmetric matrix (64 x 64)
int64_t coarse_tiles(int64_t l);
// Ginv in the coarse numbering; cidx (l entries) maps subdomain-order unknowns
// to coarse positions
void launch_coarse_pack(int64_t l, const double* Ginv, const int32_t* cidx, double* packed, hipStream_t st);

// ---- explicit local dual operators (touched block of K_reg^{-1}) -----------
// Touched DOFs of a subdomain in ascending factor index: sorted position i
// of subdomain p is global touched index sit[iface_off + i], factor index
// sfidx[iface_off + i]; pos[dof_off + r] is the sorted position of factor
// row r, or -1.  Ft_p: lower-triangle 16 x 16 tiles (row-major), tile (I, J)
// at foff[p] + 256 (J mt - J (J - 1) / 2 + I - J), mt = ceil(m_p / 16);
// diagonal tiles whole, padding rows and columns zero.
struct ExplicitForm {
  const SubDev* subs;
  const double* band;         // FP64 band factors
  double* dinv;               // diagonal-block inverses (512 entries per 16-row block),
                              // followed by the scratch (at zs_off)
  const int64_t* doff;        // their offset per subdomain
  const int32_t* sfidx;
  const int32_t* pos;
  const int64_t* foff;
  const int32_t* items;       // (subdomain, group of kExplicitWaves column blocks) pairs
  int64_t zs_off;             // scratch: zstride entries per wavefront of a launch
  int64_t zstride;
  int32_t kb;                 // staged tiles per row, explicit_form_kb(bmax)
  int32_t max_ndof;           // largest subdomain DOF count (LDS of the position table)
  void* F;                    // Ft storage (double or float)
};
// column blocks (wavefronts) per forming workgroup
constexpr int kExplicitWaves = 8;
// tiles per staged row of the forming kernel for half bandwidth bmax (0: too wide)
int explicit_form_kb(int bmax);
struct ExplicitApply {
  const SubDev* subs;
  const int32_t* order;       // workgroup -> subdomain, or nullptr
  int64_t nsub;
  const void* F;
  const int64_t* foff;
  const int32_t* sit;
  const double* lam;
  double lam_sign;
  double* out_iface;          // z at the touched DOFs (global touched numbering)
  const int32_t* if_rp;
  const int32_t* if_row;
  const double* if_coef;
  const int32_t* done;
  PcgFold fold;               // as in KsolveArgs
};
// copy the operators of the listed subdomains from src to dst
void launch_copy_explicit(const SubDev* subs, int64_t count, const int32_t* list, const int64_t* foff,
                          const void* src, void* dst, size_t elem, hipStream_t st);
// tiles of the lower triangle of an m x m operator
int64_t explicit_tiles(int64_t m);
void launch_diag_inverse(const SubDev* subs, int64_t count, const int32_t* list, const double* band,
                         const int64_t* doff, double* dinv, hipStream_t st);
// groups [item0, item0 + n) of a.items; n <= the scratch's group capacity
template <typename T>
void launch_explicit_form(const ExplicitForm& a, int64_t item0, int64_t n, hipStream_t st);
template <typename T>
void launch_explicit_apply(const ExplicitApply& a, int max_iface, hipStream_t st);
// out = (x ? x : 0) - sign * G^T a; optional partial sums of out.out, or of
// out.dotv when dotv is given
void launch_gt_apply(const DualMaps& M, const double* x, const double* a, double sign, double* out,
                     double* partials, const int32_t* done, hipStream_t st, const double* dotv = nullptr,
                     const PcgFold& fold = PcgFold{});
// iface_out = K_bb (B^T w) per subdomain
// K_bb values from the assembled (unregularized) band (subdomains flagged
// in need, all if NULL); copy of the listed subdomains' values
template <typename T>
void launch_gather_kbb(const DualMaps& M, const double* band, const uint8_t* need, T* out, hipStream_t st);
template <typename T>
void launch_copy_kbb(const DualMaps& M, int64_t count, const int32_t* list, const T* src, T* dst, hipStream_t st);
template <typename TV>
void launch_lumped(const DualMaps& M, const double* w, const TV* kbb_val, double* iface_out,
                   const int32_t* done, hipStream_t st);

// ---- Dirichlet preconditioner (dirichlet.hip) -------------------------------
// Sparse rows in wavefront groups of 64 (layout of NbGroupsHost in model.h).
struct NbGroups {
  const int32_t* out;          // output index of each lane slot, -1 past the end
  const int32_t* ldof;         // local natural DOF of the slot's row
  const uint32_t* mask;        // column nodes among the 27 around the row's node
  const int64_t* goff;         // value offset of each group
  const int32_t* gnb;          // neighbour blocks of each group
  const int32_t* gsub;         // subdomain of each group
  const int32_t* g0;           // first group of each subdomain (nsub + 1)
  int64_t groups;
};
// K_ii of the listed subdomains from the assembled band into the interior
// problems' row-band storage
void launch_gather_interior_band(const SubDev* subs, const SubDev* isubs, const int32_t* ilo, int64_t count,
                                 const int32_t* list, const double* band, double* iband, hipStream_t st);
template <typename T>
void launch_gather_groups(const NbGroups& G, const SubDev* subs, const double* band, const uint8_t* need, T* out,
                          hipStream_t st);
template <typename T>
void launch_copy_groups(const NbGroups& G, int64_t count, const int32_t* list, const T* src, T* dst, hipStream_t st);
// out_iface = K_tt B^T w, xint = K_it B^T w
template <typename TV>
void launch_dirichlet_a(const DualMaps& M, const NbGroups& kit, const double* w, const TV* kbb, const TV* kitv,
                        double* out, double* xint, const int32_t* done, hipStream_t st);
// out_iface -= K_ti sint
template <typename TV>
void launch_dirichlet_c(const DualMaps& M, const NbGroups& kti, const SubDev* isubs, const int32_t* ilo,
                        const double* sint, const TV* ktiv, double* out, const int32_t* done, hipStream_t st);

int reduction_blocks(int64_t n);
// message of the last failed handle-less call on this thread (or nullptr):
// tfeti_mlp_forward_noalloc and tfeti_model_host record theirs here
const char* call_error();
void set_call_error(const std::string& msg);
// scalar finalizers (single thread); see dual.hip
void launch_finalize(int kind, PcgScalars* S, const double* partials, int nparts, hipStream_t st);
enum FinalizeKind { FIN_WW = 0, FIN_YW = 1, FIN_PQ = 2, FIN_RREF = 3, FIN_SUM_TMP0 = 4 };

// y = a x + b y style helpers (guarded by done when given)
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);
void launch_copy(int64_t n, const double* x, double* y, hipStream_t st);
// nonfinite check: S->nonfinite |= any(!isfinite(x))
void launch_check_finite(int64_t n, const double* x, PcgScalars* S, hipStream_t st);

// ---- Newton-level kernels ---------------------------------------------------
// partial sums of (sum over copies of v)^2 over free global DOFs
void launch_assembled_sq(int64_t n_gdof, const int32_t* g_rp, const int64_t* g_copies, const uint8_t* g_free,
                         const double* v, double* partials, hipStream_t st);
// partial sums of v[g_first[i]]^2 and (v + w)[g_first]^2 etc. (kind selects)
void launch_untorn_sq(int64_t n_gdof, const int64_t* g_first, const double* v, double* partials, hipStream_t st);
void launch_sum_partials(const double* partials, int n, double* out, hipStream_t st);
// per-workgroup counts of the elements with a plastic Gauss point (reduction_blocks(n_elem) partials)
void launch_plastic_elements(int64_t n_elem, const uint8_t* plastic, double* partials, hipStream_t st);

// ---- learned warm start ---------------------------------------------------------
struct WarmMaps {
  int64_t n;                  // interface nodes
  const int32_t* rows;        // n * 21
  const int8_t* cls;
  const int32_t* erp;
  const int32_t* elems;
};
void launch_warm_features(const WarmMaps& W, const double* kappa, const double* lam_prev, const double dir[3],
                          double inv_slam, double kscale, float* X, float* Mk, hipStream_t st);
void launch_warm_targets(const WarmMaps& W, const double* lam_prev, const double* lam_next, double inv_slam, float* T,
                         hipStream_t st);
void launch_warm_apply(const WarmMaps& W, const double* lam_prev, const float* Y, double slam, double* out,
                       hipStream_t st);

}  // namespace tfeti

// Dual-space kernels of the PCGP (Algorithm 3), all FP64: the B gather,
// G w = R^T B^T w, G^T a = B R a, the dense coarse solve with (G G^T)^{-1},
// the lumped preconditioner B K B^T (Section 4.2; K_bb values in FP64, or in
// FP32 in the mixed-precision mode), deterministic two-stage
// reductions and the scalar updates of the iteration.  Every kernel of the
// iteration returns at once when the device "done" flag is set, so a fixed
// number of iterations can be enqueued (or replayed from a graph) and the
// ones after convergence cost only their launch.
#include "kernels.h"

namespace tfeti {

namespace {
constexpr int RB = 256;            // threads of reduction blocks
constexpr int kMaxRedBlocks = 4096;

// sum over a workgroup of RB threads: wavefront shuffles, then the
// wavefronts' sums in order (fixed order, deterministic); every thread gets
// the result
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < RB / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}
}  // namespace

int reduction_blocks(int64_t n) {
  int64_t b = (n + RB - 1) / RB;
  if (b > kMaxRedBlocks) b = kMaxRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

// ---------------------------------------------------------------- gather
// fold.S: the direction fold.p of the iteration is taken as fma(beta, p, y)
// (the update the subdomain solve applied on the fly), stored back and
// dotted with the output in place of dotv
__global__ __launch_bounds__(RB) void gather_kernel(int64_t m, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ent, const double* __restrict__ val,
                                                    const double* __restrict__ iface, double* __restrict__ out,
                                                    const double* __restrict__ dotv, double* __restrict__ partials,
                                                    PcgFold fold, const int32_t* __restrict__ done) {
  __shared__ double sh[RB];
  if (done && *done) return;
  const double beta = fold.S ? fold.S->beta : 0.0;
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < m; r += (int64_t)gridDim.x * RB) {
    // every row has an entry; most have two, nearly all at most four
    const double q = seg_dot<4>(rp[r], rp[r + 1], ent, val, [&](int32_t i) { return iface[i]; });
    out[r] = q;
    if (fold.S) {
      const double pn = fma(beta, fold.p[r], fold.y[r]);
      fold.p[r] = pn;
      acc += q * pn;
    } else if (dotv) {
      acc += q * dotv[r];
    }
  }
  if (partials) {
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

void launch_gather(const DualMaps& M, const double* iface, double* out, const double* dotv, double* partials,
                   const int32_t* done, hipStream_t st, const PcgFold& fold) {
  gather_kernel<<<dim3(reduction_blocks(M.m)), dim3(RB), 0, st>>>(M.m, M.b_rowptr, M.b_iface, M.b_val, iface, out,
                                                                    dotv, partials, fold, done);
}

// ---------------------------------------------------------------- G w
// six sums of a workgroup at once: wave shuffles, then the waves' results
// in order (fixed order, deterministic)
__device__ __forceinline__ void block_sum6(double (&acc)[6], double (*sh)[6]) {
#pragma unroll
  for (int j = 0; j < 6; ++j)
    for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_down(acc[j], off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 6; ++j) sh[w][j] = acc[j];
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int k = 0; k < RB / 64; ++k) s += sh[k][threadIdx.x];
    acc[0] = s;  // thread j < 6 holds sum j
  }
}

// One workgroup per subdomain streams the subdomain's B^T entries (U per
// thread in flight): v = coef * w[row] lands on the raw modes of the entry's
// node (translation of its component; rotations by its centred coordinates);
// the six sums are scaled to the orthonormal modes at the end.
// fold.S with S->pend: w is r of the previous iteration, taken as
// fma(-gamma, q, r)
__global__ __launch_bounds__(RB) void g_apply_kernel(DualMaps M, const double* __restrict__ w,
                                                     double* __restrict__ c, PcgFold fold,
                                                     const int32_t* __restrict__ done) {
  __shared__ double sh[RB / 64][6];
  if (done && *done) return;
  const bool pend = fold.S && fold.S->pend;
  const double mg = pend ? -fold.S->gamma : 0.0;
  const int64_t p = blockIdx.x;
  const int64_t t0 = M.subs[p].iface_off;
  const int32_t e0 = M.if_rp[t0], e1 = M.if_rp[t0 + M.subs[p].n_iface];
  const double hh[3] = {M.hh[0], M.hh[1], M.hh[2]};
  double acc[6] = {0, 0, 0, 0, 0, 0};
  constexpr int U = 8;  // entries per thread in flight: one pass covers an 8^3 subdomain's B^T
  for (int32_t eb = e0 + (int32_t)threadIdx.x; eb < e1; eb += U * RB) {
    int32_t row[U];
    uint32_t pk[U];
    double cf[U], wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t e = eb + u * RB < e1 ? eb + u * RB : eb;  // clamped: loads stay unconditional
      row[u] = M.if_row[e];
      pk[u] = M.if_pk[e];
      cf[u] = eb + u * RB < e1 ? M.if_coef[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) wv[u] = w[row[u]];
    if (pend) {
      double qv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) qv[u] = fold.q[row[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) wv[u] = fma(mg, qv[u], wv[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double v = cf[u] * wv[u];
      double x, y, z;
      const int32_t cc = rigid_unpack(pk[u], hh, x, y, z);
      acc[0] += cc == 0 ? v : 0.0;
      acc[1] += cc == 1 ? v : 0.0;
      acc[2] += cc == 2 ? v : 0.0;
      acc[3] += (cc == 0 ? -y : (cc == 1 ? x : 0.0)) * v;
      acc[4] += (cc == 1 ? -z : (cc == 2 ? y : 0.0)) * v;
      acc[5] += (cc == 0 ? z : (cc == 2 ? -x : 0.0)) * v;
    }
  }
  block_sum6(acc, sh);
  if (threadIdx.x < 6) {
    const double* sc = M.rscale + 4 * p;
    c[6 * p + threadIdx.x] = acc[0] * sc[threadIdx.x < 3 ? 0 : threadIdx.x - 2];
  }
}

void launch_g_apply(const DualMaps& M, const double* w, double* c, const int32_t* done, hipStream_t st,
                    const PcgFold& fold) {
  g_apply_kernel<<<dim3((unsigned)M.nsub), dim3(RB), 0, st>>>(M, w, c, fold, done);
}

// ---------------------------------------------------------------- R^T f
__global__ __launch_bounds__(RB) void rt_apply_kernel(DualMaps M, const double* __restrict__ f,
                                                      double* __restrict__ c) {
  __shared__ double sh[RB / 64][6];
  const int64_t p = blockIdx.x;
  const SubDev s = M.subs[p];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int ld = threadIdx.x; ld < s.ndof; ld += RB) {
    double v = f[s.dof_off + ld];
    const double* R = M.R_full + 6 * (s.dof_off + ld);
    for (int j = 0; j < 6; ++j) acc[j] += R[j] * v;
  }
  block_sum6(acc, sh);
  if (threadIdx.x < 6) c[6 * p + threadIdx.x] = acc[0];
}

void launch_rt_apply(const DualMaps& M, const double* f, double* c, hipStream_t st) {
  rt_apply_kernel<<<dim3((unsigned)M.nsub), dim3(RB), 0, st>>>(M, f, c);
}

// ---------------------------------------------------------------- u = z + R alpha
__global__ __launch_bounds__(RB) void add_rigid_kernel(DualMaps M, const double* __restrict__ z,
                                                       const double* __restrict__ alpha, double* __restrict__ u) {
  const int64_t p = blockIdx.x;
  const SubDev s = M.subs[p];
  const double* al = alpha + 6 * p;
  const double a0 = al[0], a1 = al[1], a2 = al[2], a3 = al[3], a4 = al[4], a5 = al[5];
  for (int ld = threadIdx.x; ld < s.ndof; ld += RB) {
    const int64_t d = s.dof_off + ld;
    const double* R = M.R_full + 6 * d;
    u[d] = z[d] + R[0] * a0 + R[1] * a1 + R[2] * a2 + R[3] * a3 + R[4] * a4 + R[5] * a5;
  }
}

void launch_add_rigid(const DualMaps& M, const double* z, const double* alpha, double* u, hipStream_t st) {
  add_rigid_kernel<<<dim3((unsigned)M.nsub), dim3(RB), 0, st>>>(M, z, alpha, u);
}

// ---------------------------------------------------------------- coarse solve
// a = scale * Ginv c with the symmetric (G G^T)^{-1} stored as its lower
// CT x CT tiles (I >= J, tile t = I (I+1)/2 + J, row-major, zero-padded past
// l): each tile is read once and contributes A_IJ c_J to block I and, off the
// diagonal, A_IJ^T c_I to block J.  Every output block gets exactly one
// partial per tile column index, summed in a fixed order by the second kernel.
namespace {
constexpr int CT = 64;
__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
  I = (int)sqrtf(2.0f * (float)t);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  J = t - I * (I + 1) / 2;
}
}  // namespace

// G is the inverse in the coarse numbering; cidx maps a subdomain-order
// coarse unknown to its coarse position
__global__ __launch_bounds__(256) void coarse_pack_kernel(int64_t l, const double* __restrict__ G,
                                                          const int32_t* __restrict__ cidx, double* __restrict__ P) {
  int I, J;
  tile_ij(blockIdx.x, I, J);
  double* out = P + (int64_t)blockIdx.x * CT * CT;
  for (int q = threadIdx.x; q < CT * CT; q += 256) {
    const int64_t gi = (int64_t)I * CT + q / CT, gj = (int64_t)J * CT + q % CT;
    out[q] = (gi < l && gj < l) ? G[(int64_t)cidx[gi] * l + cidx[gj]] : 0.0;
  }
}

__global__ __launch_bounds__(256) void coarse_symv_kernel(int64_t l, int64_t lp, const double* __restrict__ P,
                                                          const double* __restrict__ c, double* __restrict__ part,
                                                          const int32_t* __restrict__ done) {
  __shared__ double A[CT][CT + 1];
  __shared__ double xI[CT], xJ[CT];
  if (done && *done) return;
  int I, J;
  tile_ij(blockIdx.x, I, J);
  const double* tile = P + (int64_t)blockIdx.x * CT * CT;
  const int tid = threadIdx.x;
  double v[CT * CT / 256];
#pragma unroll
  for (int u = 0; u < CT * CT / 256; ++u) v[u] = __builtin_nontemporal_load(tile + u * 256 + tid);
  if (tid < CT) {
    const int64_t gj = (int64_t)J * CT + tid, gi = (int64_t)I * CT + tid;
    xJ[tid] = gj < l ? c[gj] : 0.0;
    xI[tid] = gi < l ? c[gi] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < CT * CT / 256; ++u) {
    const int q = u * 256 + tid;
    A[q / CT][q % CT] = v[u];
  }
  __syncthreads();
  if (tid < CT) {
    double sr = 0.0;
    for (int j = 0; j < CT; ++j) sr += A[tid][j] * xJ[j];
    part[(int64_t)J * lp + (int64_t)I * CT + tid] = sr;
  } else if (tid < 2 * CT && I != J) {
    const int j = tid - CT;
    double sc = 0.0;
    for (int i = 0; i < CT; ++i) sc += A[i][j] * xI[i];
    part[(int64_t)I * lp + (int64_t)J * CT + j] = sc;
  }
}

// 16 outputs per workgroup, 16 slices of the partials per output (up to 8
// loads in flight per thread), then the slices added in a fixed order
__global__ __launch_bounds__(256) void coarse_reduce_kernel(int64_t l, int64_t lp, int nT,
                                                            const double* __restrict__ part, double* __restrict__ a,
                                                            double scale, const int32_t* __restrict__ done) {
  __shared__ double q[16][17];
  if (done && *done) return;
  const int o = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + o;
  double s = 0.0;
  if (i < l) {
    for (int k0 = sl; k0 < nT; k0 += 8 * 16) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + 16 * u;
        v[u] = k < nT ? part[(int64_t)k * lp + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
  }
  q[sl][o] = s;
  __syncthreads();
  if (sl == 0 && i < l) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += q[k][o];
    a[i] = scale * t;
  }
}

int64_t coarse_tiles(int64_t l) {
  const int64_t nT = (l + CT - 1) / CT;
  return nT * (nT + 1) / 2;
}

void launch_coarse_pack(int64_t l, const double* Ginv, const int32_t* cidx, double* packed, hipStream_t st) {
  const int64_t nt = coarse_tiles(l);
  if (nt > 0) coarse_pack_kernel<<<dim3((unsigned)nt), dim3(256), 0, st>>>(l, Ginv, cidx, packed);
}

void launch_coarse_gemv(const DualMaps& M, const double* c, double* a, double scale, const int32_t* done,
                        hipStream_t st) {
  const int nT = (int)((M.l + CT - 1) / CT);
  const int64_t lp = (int64_t)nT * CT;
  coarse_symv_kernel<<<dim3((unsigned)coarse_tiles(M.l)), dim3(256), 0, st>>>(M.l, lp, M.Gpk, c, M.Gpart, done);
  coarse_reduce_kernel<<<dim3((unsigned)((M.l + 15) / 16)), dim3(256), 0, st>>>(M.l, lp, nT, M.Gpart, a, scale,
                                                                                done);
}

// ---------------------------------------------------------------- x - G^T a
// One multiplier row per thread: (G^T a)_r = sum_e b_val[e] R(node_e) . a_p(e),
// the mode values of the entry's node formed from its packed coordinates.
// fold.S with S->pend: x is r of the previous iteration; fma(-gamma, q, r)
// is used and stored to fold.r, and lambda takes fma(gamma, p, lambda)
__global__ __launch_bounds__(RB) void gt_apply_kernel(DualMaps M, const double* x,
                                                      const double* __restrict__ a, double sign,
                                                      double* __restrict__ out, double* __restrict__ partials,
                                                      const double* __restrict__ dotv, PcgFold fold,
                                                      const int32_t* __restrict__ done) {
  __shared__ double sh[RB];
  if (done && *done) return;
  const bool pend = fold.S && fold.S->pend;
  const double gam = pend ? fold.S->gamma : 0.0;
  const double hh[3] = {M.hh[0], M.hh[1], M.hh[2]};
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < M.m; r += (int64_t)gridDim.x * RB) {
    const int64_t e0 = M.b_rowptr[r], e1 = M.b_rowptr[r + 1];
    double xr = x ? x[r] : 0.0;
    if (pend) {
      xr = fma(-gam, fold.q[r], xr);
      fold.r[r] = xr;
      fold.lam[r] = fma(gam, fold.p[r], fold.lam[r]);
    }
    double g = 0.0;
    // entries two at a time, the second one's index clamped so that every
    // load is unconditional and in flight together
    for (int64_t e = e0; e < e1; e += 2) {
      const bool h1 = e + 1 < e1;
      const int64_t f1 = h1 ? e + 1 : e;
      const int32_t p0 = M.b_sub[e], p1 = M.b_sub[f1];
      const uint32_t k0 = M.b_pk[e], k1 = M.b_pk[f1];
      const double bv0 = M.b_val[e], bv1 = M.b_val[f1];
      double s0[4], s1[4], a0[6], a1[6];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s0[j] = M.rscale[4 * (int64_t)p0 + j];
        s1[j] = M.rscale[4 * (int64_t)p1 + j];
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        a0[j] = a[6 * (int64_t)p0 + j];
        a1[j] = a[6 * (int64_t)p1 + j];
      }
      double x0, y0, z0, x1, y1, z1, R0[6], R1[6];
      rigid_row(rigid_unpack(k0, hh, x0, y0, z0), x0, y0, z0, s0, R0);
      rigid_row(rigid_unpack(k1, hh, x1, y1, z1), x1, y1, z1, s1, R1);
      double v0 = 0.0, v1 = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        v0 += R0[j] * a0[j];
        v1 += R1[j] * a1[j];
      }
      g += bv0 * v0;
      const double g2 = g + bv1 * v1;
      g = h1 ? g2 : g;
    }
    double o = xr - sign * g;
    out[r] = o;
    acc += o * (dotv ? dotv[r] : o);
  }
  if (partials) {
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

void launch_gt_apply(const DualMaps& M, const double* x, const double* a, double sign, double* out,
                     double* partials, const int32_t* done, hipStream_t st, const double* dotv,
                     const PcgFold& fold) {
  gt_apply_kernel<<<dim3(reduction_blocks(M.m)), dim3(RB), 0, st>>>(M, x, a, sign, out, partials, dotv, fold,
                                                                      done);
}

// ---------------------------------------------------------------- lumped preconditioner
// One workgroup per subdomain.  B^T w is scattered into an LDS copy of the
// whole subdomain vector (zero off the touched DOFs).  Then each wavefront
// takes groups of 64 touched DOFs (one per lane; the group's values are
// stored slot-major, so every load is 64 consecutive values) and walks the
// lanes' neighbour masks LU nodes at a time, summing values x neighbour
// components in bit order (fixed order, deterministic); lanes with fewer
// nodes than the group read zero values against their own node.  A
// wavefront's first group (slot data and first block of values) does not
// depend on the scatter and is requested before it, so its loads are in
// flight during the scatter's chain of dependent loads.
namespace {
constexpr int LT = 1024;  // threads of the preconditioner workgroups
constexpr int LU = 4;     // neighbour nodes per step
}  // namespace

template <typename TV>
__global__ __launch_bounds__(LT) void lumped_kernel(DualMaps M, const double* __restrict__ w,
                                                    const TV* __restrict__ kv, double* __restrict__ out,
                                                    const int32_t* __restrict__ done) {
  extern __shared__ double vloc[];
  if (done && *done) return;
  const int64_t p = blockIdx.x;
  const int32_t nif = M.subs[p].n_iface, ndof = M.subs[p].ndof, N0 = M.subs[p].N[0], N1 = M.subs[p].N[1];
  const int64_t ioff = M.subs[p].iface_off;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int32_t gend = M.kbb_g0[p + 1];
  // the wavefront's current group: output row, neighbour mask, node, node
  // count, values, and the block of values of LU nodes from b0 on (past the
  // group's count the last node's values again, zeroed)
  int32_t g = M.kbb_g0[p] + wave, it = -1, a = 0, nb = 1;
  uint32_t mask = 0;
  const TV* v = kv;
  TV x[3 * LU];
  auto load_block = [&](int b0) {
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const bool in = b0 + u < nb;
      const int bb = in ? b0 + u : nb - 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const TV t = v[(int64_t)(3 * bb + c) * 64];
        x[3 * u + c] = in ? t : TV(0);
      }
    }
  };
  auto start_group = [&]() {
    const int64_t slot = 64 * (int64_t)g + lane;
    it = M.kbb_row[slot];
    mask = M.kbb_mask[slot];
    a = M.kbb_node[slot];
    nb = M.kbb_gnb[g];
    v = kv + M.kbb_goff[g] + lane;
    load_block(0);
  };
  if (g < gend) start_group();

  for (int q = threadIdx.x; q < ndof; q += LT) vloc[q] = 0.0;
  __syncthreads();
  for (int t = threadIdx.x; t < nif; t += LT) {
    // every touched DOF has an entry; nearly all have at most four
    const int64_t i = ioff + t;
    vloc[M.if_ldof[i]] = seg_dot<4>(M.if_rp[i], M.if_rp[i + 1], M.if_row, M.if_coef,
                                    [&](int32_t row) { return w[row]; });
  }
  __syncthreads();
  while (g < gend) {
    double y = 0.0;
    for (int b0 = 0; b0 < nb; b0 += LU) {
      if (b0 > 0) load_block(b0);
      int a2[LU];
#pragma unroll
      for (int u = 0; u < LU; ++u) {
        const int k = mask ? __ffs(mask) - 1 : 13;  // 13: the node itself
        mask &= mask - 1;
        a2[u] = a + (k % 3 - 1) + N0 * ((k / 3) % 3 - 1 + N1 * (k / 9 - 1));
      }
#pragma unroll
      for (int u = 0; u < LU; ++u)
#pragma unroll
        for (int c = 0; c < 3; ++c) y += (double)x[3 * u + c] * vloc[3 * a2[u] + c];
    }
    if (it >= 0) out[it] = y;
    g += LT / 64;
    if (g < gend) start_group();
  }
}

template <typename TV>
void launch_lumped(const DualMaps& M, const double* w, const TV* kbb_val, double* iface_out, const int32_t* done,
                   hipStream_t st) {
  size_t shm = (size_t)(M.max_ndof > 0 ? M.max_ndof : 1) * sizeof(double);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)lumped_kernel<TV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  lumped_kernel<TV><<<dim3((unsigned)M.nsub), dim3(LT), shm, st>>>(M, w, kbb_val, iface_out, done);
}
template void launch_lumped<double>(const DualMaps&, const double*, const double*, double*, const int32_t*,
                                    hipStream_t);
template void launch_lumped<float>(const DualMaps&, const double*, const float*, double*, const int32_t*,
                                   hipStream_t);

// ---------------------------------------------------------------- reductions
// one workgroup of FB threads: the partials (up to 4096) in at most four
// loads per thread, wavefront shuffles, then the wavefronts' sums in order
constexpr int FB = 1024;
__device__ __forceinline__ double final_sum(const double* __restrict__ partials, int n) {
  __shared__ double sh[FB / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += FB) acc += partials[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  double s = sh[0];
#pragma unroll
  for (int w = 1; w < FB / 64; ++w) s += sh[w];
  return s;
}

__global__ __launch_bounds__(FB) void finalize_kernel(int kind, PcgScalars* S, const double* __restrict__ partials,
                                                      int nparts) {
  if (kind != FIN_RREF && kind != FIN_SUM_TMP0 && S->done) return;
  const double sum = final_sum(partials, nparts);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case FIN_WW: {
      S->ww = sum;
      double nw = sqrt(sum);
      S->rr = nw;
      if (!(nw == nw)) {
        S->nonfinite = 1;
        S->done = 3;
      } else if (nw <= S->eps * S->r_ref || S->r_ref == 0.0) {
        S->done = 1;
      } else if (S->iters >= S->maxit) {
        S->done = 2;
      }
      S->pend = 0;  // the projection before this applied them
      break;
    }
    case FIN_YW:
      S->yw = sum;
      S->beta = (S->iters == 0) ? 0.0 : sum / S->yw_prev;
      break;
    case FIN_PQ:
      S->pq = sum;
      S->gamma = S->yw / sum;
      S->yw_prev = S->yw;
      S->iters += 1;
      S->pend = 1;
      break;
    case FIN_RREF:
      S->r_ref = sqrt(sum);
      break;
    case FIN_SUM_TMP0:
      S->tmp0 = sum;
      break;
  }
}

void launch_finalize(int kind, PcgScalars* S, const double* partials, int nparts, hipStream_t st) {
  finalize_kernel<<<dim3(1), dim3(FB), 0, st>>>(kind, S, partials, nparts);
}

__global__ __launch_bounds__(FB) void sum_partials_kernel(const double* __restrict__ partials, int n,
                                                         double* __restrict__ out) {
  const double s = final_sum(partials, n);
  if (threadIdx.x == 0) *out = s;
}

void launch_sum_partials(const double* partials, int n, double* out, hipStream_t st) {
  sum_partials_kernel<<<dim3(1), dim3(FB), 0, st>>>(partials, n, out);
}

// ---------------------------------------------------------------- vector updates
__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // b == 0 does not read y (it may hold anything, NaN included)
  if (i < n) y[i] = a * (x ? x[i] : 0.0) + (b != 0.0 ? b * y[i] : 0.0);
}
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  if (n > 0) axpby_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(n, a, x, b, y);
}

__global__ void copy_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
void launch_copy(int64_t n, const double* x, double* y, hipStream_t st) {
  if (n > 0) copy_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(n, x, y);
}

__global__ void check_finite_kernel(int64_t n, const double* __restrict__ x, PcgScalars* S) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) S->nonfinite = 1;
}
void launch_check_finite(int64_t n, const double* x, PcgScalars* S, hipStream_t st) {
  if (n > 0) check_finite_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(n, x, S);
}

// ---------------------------------------------------------------- Newton-level norms
__global__ __launch_bounds__(RB) void assembled_sq_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                          const int64_t* __restrict__ cp,
                                                          const uint8_t* __restrict__ free_,
                                                          const double* __restrict__ v, double* __restrict__ partials) {
  __shared__ double sh[RB];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    if (!free_[i]) continue;
    double s = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += v[cp[e]];
    acc += s * s;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

void launch_assembled_sq(int64_t n_gdof, const int32_t* g_rp, const int64_t* g_copies, const uint8_t* g_free,
                         const double* v, double* partials, hipStream_t st) {
  assembled_sq_kernel<<<dim3(reduction_blocks(n_gdof)), dim3(RB), 0, st>>>(n_gdof, g_rp, g_copies, g_free, v,
                                                                            partials);
}

__global__ __launch_bounds__(RB) void untorn_sq_kernel(int64_t n, const int64_t* __restrict__ first,
                                                       const double* __restrict__ v, double* __restrict__ partials) {
  __shared__ double sh[RB];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    double x = v[first[i]];
    acc += x * x;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

void launch_untorn_sq(int64_t n_gdof, const int64_t* g_first, const double* v, double* partials, hipStream_t st) {
  untorn_sq_kernel<<<dim3(reduction_blocks(n_gdof)), dim3(RB), 0, st>>>(n_gdof, g_first, v, partials);
}

// Elements with a plastic Gauss point (the 8 flags of element e are bytes
// 8e .. 8e + 7), per workgroup, as doubles for launch_sum_partials.
__global__ __launch_bounds__(RB) void plastic_elements_kernel(int64_t n_elem, const uint8_t* __restrict__ pl,
                                                              double* __restrict__ partials) {
  __shared__ double sh[RB];
  double c = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n_elem; e += (int64_t)gridDim.x * RB) {
    const uint2 v = *reinterpret_cast<const uint2*>(pl + 8 * e);
    c += (v.x | v.y) != 0u ? 1.0 : 0.0;
  }
  double s = block_sum(c, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

void launch_plastic_elements(int64_t n_elem, const uint8_t* plastic, double* partials, hipStream_t st) {
  plastic_elements_kernel<<<dim3(reduction_blocks(n_elem)), dim3(RB), 0, st>>>(n_elem, plastic, partials);
}

}  // namespace tfeti

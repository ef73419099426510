// Dirichlet preconditioner Bbar Sbar Bbar^T of Section 4.2, applied without
// forming the Schur complements: with b the DOFs of the nodes that carry a
// row of B and i the others (the interior, a box of the node lattice),
//
//   Sbar x_b = K_bb x_b - K_bi K_ii^{-1} K_ib x_b,
//
// and since Bbar^T w vanishes off the touched DOFs t, the touched part of
// the result is K_tt x_t - K_ti K_ii^{-1} K_it x_t.  Per application:
//   A  one workgroup per subdomain scatters x = B^T w into LDS, writes
//      K_tt x at the touched DOFs (the lumped preconditioner's product) and
//      K_it x into the interior vector;
//   S  the interior solves s = K_ii^{-1} (K_it x) with banded Cholesky
//      factors of K_ii (the subdomain solve kernel on the interior boxes);
//   C  one workgroup per subdomain scatters s into LDS and subtracts K_ti s
//      at the touched DOFs;
// then the B gather.  The explicit Schur complement of an 8^3-element
// subdomain (1158 boundary DOFs) would be read as 5.4 MB (packed symmetric)
// per application; the factor of its 7^3-node interior and the coupling
// rows read about 3 MB, and forming them costs a band Cholesky of K_ii
// instead of a dense product of rank 1029.
#include "kernels.h"

namespace tfeti {

namespace {

// subdomain factor index of interior factor index fi (interior box with its
// own factor ordering, shifted by lo on the subdomain lattice)
__device__ __forceinline__ int32_t interior_to_sub(const SubDev& si, const SubDev& s, const int32_t* lo, int32_t fi) {
  const int32_t q = fi / 3, c = fi - 3 * q;
  const int32_t N0 = si.perm[0] == 0 ? si.N[0] : (si.perm[0] == 1 ? si.N[1] : si.N[2]);
  const int32_t N1 = si.perm[1] == 0 ? si.N[0] : (si.perm[1] == 1 ? si.N[1] : si.N[2]);
  const int32_t i0 = q % N0, t = q / N0, i1 = t % N1, i2 = t / N1;
  // coordinates along the local axes x, y, z
  const int32_t cx = si.perm[0] == 0 ? i0 : (si.perm[1] == 0 ? i1 : i2);
  const int32_t cy = si.perm[0] == 1 ? i0 : (si.perm[1] == 1 ? i1 : i2);
  const int32_t cz = si.perm[0] == 2 ? i0 : (si.perm[1] == 2 ? i1 : i2);
  return 3 * ((cx + lo[0]) * s.fs[0] + (cy + lo[1]) * s.fs[1] + (cz + lo[2]) * s.fs[2]) + c;
}

// entry (f, f2) of the assembled band (row max, column min; zero outside)
__device__ __forceinline__ double band_entry(const double* A, const SubDev& s, int32_t f, int32_t f2) {
  const int32_t r = f > f2 ? f : f2, c = f > f2 ? f2 : f;
  return r - c <= s.b ? A[(int64_t)r * s.Wb + (c - r + s.b)] : 0.0;
}

}  // namespace

// K_ii of the listed subdomains in the interior problems' row-band storage,
// read from the assembled (unregularized) band; identity on padding rows.
__global__ __launch_bounds__(256) void gather_interior_band_kernel(const SubDev* __restrict__ subs,
                                                                   const SubDev* __restrict__ isubs,
                                                                   const int32_t* __restrict__ ilo, int64_t count,
                                                                   const int32_t* __restrict__ list,
                                                                   const double* __restrict__ band,
                                                                   double* __restrict__ iband) {
  if ((int64_t)blockIdx.y >= count) return;
  const int64_t p = list[blockIdx.y];
  const SubDev s = subs[p], si = isubs[p];
  const int32_t lo[3] = {ilo[3 * p], ilo[3 * p + 1], ilo[3 * p + 2]};
  const double* A = band + s.band_off;
  double* D = iband + si.band_off;
  const int64_t len = (int64_t)si.npad * si.Wb;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = (int32_t)(q / si.Wb), k = (int32_t)(q - (int64_t)r * si.Wb), c = r - si.b + k;
    double v = 0.0;
    if (r >= si.ndof)
      v = k == si.b ? 1.0 : 0.0;
    else if (c >= 0 && k <= si.b)
      v = band_entry(A, s, interior_to_sub(si, s, lo, r), interior_to_sub(si, s, lo, c));
    D[q] = v;
  }
}

void launch_gather_interior_band(const SubDev* subs, const SubDev* isubs, const int32_t* ilo, int64_t count,
                                 const int32_t* list, const double* band, double* iband, hipStream_t st) {
  if (count > 0)
    gather_interior_band_kernel<<<dim3(32, (unsigned)count), dim3(256), 0, st>>>(subs, isubs, ilo, count, list, band,
                                                                                 iband);
}

// Values of a group set from the assembled band (subdomains flagged in
// need): each lane slot walks its mask in bit order and writes the three
// entries coupling its row DOF to each masked node; zeros past its count.
template <typename T>
__global__ __launch_bounds__(256) void gather_groups_kernel(NbGroups G, const SubDev* __restrict__ subs,
                                                            const double* __restrict__ band,
                                                            const uint8_t* __restrict__ need, T* __restrict__ out) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = slot / 64;
  if (g >= G.groups) return;
  if (need && !need[G.gsub[g]]) return;
  const int lane = (int)(slot % 64);
  const int nb = G.gnb[g];
  T* o = out + G.goff[g] + lane;
  uint32_t mask = G.mask[slot];
  int b = 0;
  if (G.out[slot] >= 0) {
    const SubDev s = subs[G.gsub[g]];
    const int32_t ld = G.ldof[slot], a = ld / 3;
    const int32_t f = factor_index(s, ld);
    const double* A = band + s.band_off;
    for (; mask; ++b) {
      const int k = __ffs(mask) - 1;
      mask &= mask - 1;
      const int32_t a2 = a + (k % 3 - 1) + s.N[0] * ((k / 3) % 3 - 1 + s.N[1] * (k / 9 - 1));
#pragma unroll
      for (int c = 0; c < 3; ++c) o[(int64_t)(3 * b + c) * 64] = (T)band_entry(A, s, f, factor_index(s, 3 * a2 + c));
    }
  }
  for (; b < nb; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) o[(int64_t)(3 * b + c) * 64] = T(0);
}

template <typename T>
void launch_gather_groups(const NbGroups& G, const SubDev* subs, const double* band, const uint8_t* need, T* out,
                          hipStream_t st) {
  const int64_t slots = 64 * G.groups;
  if (slots > 0)
    gather_groups_kernel<T><<<dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st>>>(G, subs, band, need, out);
}
template void launch_gather_groups<double>(const NbGroups&, const SubDev*, const double*, const uint8_t*, double*,
                                           hipStream_t);
template void launch_gather_groups<float>(const NbGroups&, const SubDev*, const double*, const uint8_t*, float*,
                                          hipStream_t);

// Values of the listed subdomains' groups copied from src.
template <typename T>
__global__ __launch_bounds__(256) void copy_groups_kernel(NbGroups G, int64_t count, const int32_t* __restrict__ list,
                                                          const T* __restrict__ src, T* __restrict__ dst) {
  if ((int64_t)blockIdx.y >= count) return;
  const int32_t p = list[blockIdx.y];
  const int64_t v0 = G.goff[G.g0[p]], v1 = G.goff[G.g0[p + 1]];
  for (int64_t i = v0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v1; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename T>
void launch_copy_groups(const NbGroups& G, int64_t count, const int32_t* list, const T* src, T* dst, hipStream_t st) {
  if (count > 0) copy_groups_kernel<T><<<dim3(16, (unsigned)count), dim3(256), 0, st>>>(G, count, list, src, dst);
}
template void launch_copy_groups<double>(const NbGroups&, int64_t, const int32_t*, const double*, double*,
                                         hipStream_t);
template void launch_copy_groups<float>(const NbGroups&, int64_t, const int32_t*, const float*, float*, hipStream_t);

namespace {

constexpr int DT = 512;  // threads of the application workgroups

// One pass over the groups [g, gend) of a subdomain, a wavefront per group:
// lane l of the group sums its row's values times the LDS vector entries of
// its masked nodes (three components each) in bit order, and emit(out, y)
// stores the sum.
template <typename TV, typename Emit>
__device__ __forceinline__ void walk_groups(const NbGroups& G, int32_t g, int32_t gend, const TV* __restrict__ kv,
                                            const double* vloc, int N0, int N1, Emit emit) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (g += wave; g < gend; g += DT / 64) {
    const int64_t slot = 64 * (int64_t)g + lane;
    const int32_t out = G.out[slot];
    uint32_t mask = G.mask[slot];
    const int32_t a = G.ldof[slot] / 3;
    const int nb = G.gnb[g];
    const TV* v = kv + G.goff[g] + lane;
    double y = 0.0;
    for (int b = 0; b < nb; ++b) {
      const int k = mask ? __ffs(mask) - 1 : 13;  // 13: the row's own node (its values are zero)
      mask &= mask - 1;
      const int32_t a2 = a + (k % 3 - 1) + N0 * ((k / 3) % 3 - 1 + N1 * (k / 9 - 1));
#pragma unroll
      for (int c = 0; c < 3; ++c) y += (double)v[(int64_t)(3 * b + c) * 64] * vloc[3 * a2 + c];
    }
    if (out >= 0) emit(out, y);
  }
}

}  // namespace

// A: x = B^T w in LDS; out_iface = K_tt x (touched DOFs), xint = K_it x.
template <typename TV>
__global__ __launch_bounds__(DT) void dirichlet_a_kernel(DualMaps M, NbGroups kit, const double* __restrict__ w,
                                                         const TV* __restrict__ kbb, const TV* __restrict__ kitv,
                                                         double* __restrict__ out, double* __restrict__ xint,
                                                         const int32_t* __restrict__ done) {
  extern __shared__ double vloc[];
  if (done && *done) return;
  const int64_t p = blockIdx.x;
  const SubDev s = M.subs[p];
  for (int q = threadIdx.x; q < s.ndof; q += DT) vloc[q] = 0.0;
  __syncthreads();
  for (int t = threadIdx.x; t < s.n_iface; t += DT) {
    const int64_t i = s.iface_off + t;
    vloc[M.if_ldof[i]] = seg_dot<4>(M.if_rp[i], M.if_rp[i + 1], M.if_row, M.if_coef,
                                    [&](int32_t row) { return w[row]; });
  }
  __syncthreads();
  // K_tt: the lumped preconditioner's groups (the row's node in kbb_node)
  {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int32_t g = M.kbb_g0[p] + wave; g < M.kbb_g0[p + 1]; g += DT / 64) {
      const int64_t slot = 64 * (int64_t)g + lane;
      const int32_t it = M.kbb_row[slot];
      uint32_t mask = M.kbb_mask[slot];
      const int32_t a = M.kbb_node[slot];
      const int nb = M.kbb_gnb[g];
      const TV* v = kbb + M.kbb_goff[g] + lane;
      double y = 0.0;
      for (int b = 0; b < nb; ++b) {
        const int k = mask ? __ffs(mask) - 1 : 13;
        mask &= mask - 1;
        const int32_t a2 = a + (k % 3 - 1) + s.N[0] * ((k / 3) % 3 - 1 + s.N[1] * (k / 9 - 1));
#pragma unroll
        for (int c = 0; c < 3; ++c) y += (double)v[(int64_t)(3 * b + c) * 64] * vloc[3 * a2 + c];
      }
      if (it >= 0) out[it] = y;
    }
  }
  walk_groups<TV>(kit, kit.g0[p], kit.g0[p + 1], kitv, vloc, s.N[0], s.N[1],
                  [&](int32_t o, double y) { xint[o] = y; });
}

// C: s (interior vector) in LDS at its subdomain DOFs; out_iface -= K_ti s.
template <typename TV>
__global__ __launch_bounds__(DT) void dirichlet_c_kernel(DualMaps M, NbGroups kti, const SubDev* __restrict__ isubs,
                                                         const int32_t* __restrict__ ilo,
                                                         const double* __restrict__ sint, const TV* __restrict__ ktiv,
                                                         double* __restrict__ out, const int32_t* __restrict__ done) {
  extern __shared__ double vloc[];
  if (done && *done) return;
  const int64_t p = blockIdx.x;
  const SubDev s = M.subs[p], si = isubs[p];
  if (si.ndof == 0 || kti.g0[p] == kti.g0[p + 1]) return;
  const int32_t lo0 = ilo[3 * p], lo1 = ilo[3 * p + 1], lo2 = ilo[3 * p + 2];
  for (int q = threadIdx.x; q < s.ndof; q += DT) vloc[q] = 0.0;
  __syncthreads();
  for (int li = threadIdx.x; li < si.ndof; li += DT) {
    const int32_t ai = li / 3, c = li - 3 * ai;
    const int32_t ii = ai % si.N[0], t = ai / si.N[0], jj = t % si.N[1], kk = t / si.N[1];
    const int32_t a = (ii + lo0) + s.N[0] * ((jj + lo1) + s.N[1] * (kk + lo2));
    vloc[3 * a + c] = sint[si.dof_off + li];
  }
  __syncthreads();
  walk_groups<TV>(kti, kti.g0[p], kti.g0[p + 1], ktiv, vloc, s.N[0], s.N[1],
                  [&](int32_t o, double y) { out[o] -= y; });
}

template <typename TV>
void launch_dirichlet_a(const DualMaps& M, const NbGroups& kit, const double* w, const TV* kbb, const TV* kitv,
                        double* out, double* xint, const int32_t* done, hipStream_t st) {
  const size_t shm = (size_t)(M.max_ndof > 0 ? M.max_ndof : 1) * sizeof(double);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)dirichlet_a_kernel<TV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  dirichlet_a_kernel<TV><<<dim3((unsigned)M.nsub), dim3(DT), shm, st>>>(M, kit, w, kbb, kitv, out, xint, done);
}

template <typename TV>
void launch_dirichlet_c(const DualMaps& M, const NbGroups& kti, const SubDev* isubs, const int32_t* ilo,
                        const double* sint, const TV* ktiv, double* out, const int32_t* done, hipStream_t st) {
  const size_t shm = (size_t)(M.max_ndof > 0 ? M.max_ndof : 1) * sizeof(double);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)dirichlet_c_kernel<TV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  dirichlet_c_kernel<TV><<<dim3((unsigned)M.nsub), dim3(DT), shm, st>>>(M, kti, isubs, ilo, sint, ktiv, out, done);
}

template void launch_dirichlet_a<double>(const DualMaps&, const NbGroups&, const double*, const double*,
                                         const double*, double*, double*, const int32_t*, hipStream_t);
template void launch_dirichlet_a<float>(const DualMaps&, const NbGroups&, const double*, const float*, const float*,
                                        double*, double*, const int32_t*, hipStream_t);
template void launch_dirichlet_c<double>(const DualMaps&, const NbGroups&, const SubDev*, const int32_t*,
                                         const double*, const double*, double*, const int32_t*, hipStream_t);
template void launch_dirichlet_c<float>(const DualMaps&, const NbGroups&, const SubDev*, const int32_t*,
                                        const double*, const float*, double*, const int32_t*, hipStream_t);

}  // namespace tfeti

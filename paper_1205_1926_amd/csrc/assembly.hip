// Return mapping (Section 2.4; Voigt form of Section 3.1) and the subdomain
// assembly of Algorithm 5 on gfx950.
//
// Assembly runs in 8 launches, one per element parity class (i&1, j&1, k&1):
// elements of one class share no node, so each launch adds its element
// contributions into the row-band tangent and the torn internal force
// without atomics, and the summation order of every entry is fixed
// (class 0..7), which makes the result bitwise reproducible.
#include "kernels.h"

namespace tfeti {

__device__ __forceinline__ void return_map_point(const MatC& M, const double* sig, double kap,
                                                 const double* de, double* ds, double* dk,
                                                 double* D /* 36 or nullptr */, bool* plastic) {
  const double lam = M.lam, mu = M.mu;
  double tr = de[0] + de[1] + de[2];
  double Cde[6] = {lam * tr + 2.0 * mu * de[0], lam * tr + 2.0 * mu * de[1], lam * tr + 2.0 * mu * de[2],
                   mu * de[3], mu * de[4], mu * de[5]};
  double tau[6];
  for (int i = 0; i < 6; ++i) tau[i] = sig[i] + Cde[i];
  double pm = (tau[0] + tau[1] + tau[2]) / 3.0;
  double s[6] = {tau[0] - pm, tau[1] - pm, tau[2] - pm, tau[3], tau[4], tau[5]};
  double q = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
  double phi = sqrt(1.5) * q - (M.sy + M.H * kap);
  // a committed plastic point lies on the yield surface up to rounding; the
  // tie is elastic within a relative margin of 1e-12 of the yield radius, so
  // the tangent at a zero increment is the elastic one
  if (!(phi > 1e-12 * (M.sy + M.H * kap))) {
    for (int i = 0; i < 6; ++i) ds[i] = Cde[i];
    *dk = 0.0;
    *plastic = false;
    if (D) {
      for (int i = 0; i < 36; ++i) D[i] = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D[6 * i + j] = lam + (i == j ? 2.0 * mu : 0.0);
      D[21] = D[28] = D[35] = mu;
    }
    return;
  }
  const double three_mu_H = 3.0 * mu + M.H;
  const double beta = 3.0 * mu / three_mu_H;
  double n[6];
  for (int i = 0; i < 6; ++i) n[i] = s[i] / q;
  const double corr = beta * sqrt(2.0 / 3.0) * phi;
  for (int i = 0; i < 6; ++i) ds[i] = Cde[i] - corr * n[i];
  *dk = phi / three_mu_H;
  *plastic = true;
  if (D) {
    const double a = 2.0 * mu * beta;
    const double coef = a * sqrt(2.0 / 3.0) * (M.sy + M.H * kap) / q;
    // E_eps: 1/3 [2 -1 -1; -1 2 -1; -1 -1 2] on normals, 1/2 on shears
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double ee;
        if (i < 3 && j < 3)
          ee = (i == j ? 2.0 : -1.0) / 3.0;
        else
          ee = (i == j) ? 0.5 : 0.0;
        double c = 0.0;
        if (i < 3 && j < 3)
          c = lam + (i == j ? 2.0 * mu : 0.0);
        else if (i == j)
          c = mu;
        D[6 * i + j] = c - a * ee - coef * (n[i] * n[j] - ee);
      }
  }
}

__global__ void return_map_kernel(MatC M, int64_t npts, const double* __restrict__ sig,
                                  const double* __restrict__ kap, const double* __restrict__ de,
                                  double* __restrict__ ds, double* __restrict__ dk,
                                  double* __restrict__ Dt, uint8_t* __restrict__ pl) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  double s[6], e[6], o[6], D[36], k;
  for (int i = 0; i < 6; ++i) {
    s[i] = sig[6 * p + i];
    e[i] = de[6 * p + i];
  }
  bool plastic;
  return_map_point(M, s, kap[p], e, o, &k, Dt ? D : nullptr, &plastic);
  for (int i = 0; i < 6; ++i) ds[6 * p + i] = o[i];
  dk[p] = k;
  if (Dt)
    for (int i = 0; i < 36; ++i) Dt[36 * p + i] = D[i];
  if (pl) pl[p] = plastic ? 1 : 0;
}

void launch_return_map(const tfeti_material& mat, int64_t npts, const double* sig, const double* kap,
                       const double* de, double* ds, double* dk, double* Dt, uint8_t* pl,
                       hipStream_t st) {
  MatC M;
  M.lam = mat.E * mat.nu / ((1.0 + mat.nu) * (1.0 - 2.0 * mat.nu));
  M.mu = mat.E / (2.0 * (1.0 + mat.nu));
  M.sy = mat.sigma_y;
  M.H = mat.H;
  int64_t blocks = (npts + 127) / 128;
  if (npts > 0) return_map_kernel<<<dim3((unsigned)blocks), dim3(128), 0, st>>>(M, npts, sig, kap, de, ds, dk, Dt, pl);
}

// ---------------------------------------------------------------------------
// Assembly
// ---------------------------------------------------------------------------
constexpr int kElemPerBlock = 16;

// strain rows and derivative axes of the three nonzeros of column 3a+c of B_g
__constant__ int8_t c_rows[3][3] = {{0, 3, 5}, {1, 3, 4}, {2, 4, 5}};
__constant__ int8_t c_axis[3][3] = {{0, 1, 2}, {1, 0, 2}, {2, 1, 0}};
__constant__ int8_t c_noff[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                    {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

// MODE 1: return map, state increments and internal force of every
// element; MODE 2: the tangent of the elements of the subdomains flagged in
// A.need (the return map is evaluated again for its D).
template <int MODE>
__global__ __launch_bounds__(256) void assemble_kernel(AssembleArgs A) {
  __shared__ double s_dN[8][8][3];                       // [gp][node][axis]
  __shared__ double s_D[MODE == 2 ? kElemPerBlock : 1][8][36];
  __shared__ double s_ds[kElemPerBlock][8][6];           // w * dsigma
  __shared__ double s_du[kElemPerBlock][24];
  __shared__ int32_t s_dof[kElemPerBlock][24];           // torn DOF
  __shared__ int32_t s_fid[kElemPerBlock][24];           // factor index
  __shared__ int64_t s_band[kElemPerBlock];              // band offset of the subdomain
  __shared__ int32_t s_Wb[kElemPerBlock], s_b[kElemPerBlock];
  __shared__ int32_t s_cnt;

  const int tid = threadIdx.x;
  const int64_t first = (int64_t)blockIdx.x * kElemPerBlock;
  if (tid == 0) s_cnt = 0;
  for (int q = tid; q < 8 * 8 * 3; q += blockDim.x) {
    int g = q / 24, a = (q / 3) % 8, d = q % 3;
    s_dN[g][a][d] = A.dN[q];
  }
  // element metadata and displacement gather: one thread per (element, node)
  if (tid < kElemPerBlock * 8) {
    int el = tid / 8, a = tid % 8;
    int64_t ci = first + el;
    if (ci < A.n_colour && (MODE != 2 || A.need[A.elem_sub[A.elems[ci]]])) {
      int32_t e = A.elems[ci];
      const SubDev& s = A.subs[A.elem_sub[e]];
      int32_t le = (int32_t)(e - s.elem_off);
      int32_t i = le % s.n[0], j = (le / s.n[0]) % s.n[1], k = le / (s.n[0] * s.n[1]);
      int32_t an = (i + c_noff[a][0]) + s.N[0] * ((j + c_noff[a][1]) + s.N[1] * (k + c_noff[a][2]));
      for (int c = 0; c < 3; ++c) {
        int32_t ld = 3 * an + c;
        s_dof[el][3 * a + c] = (int32_t)(s.dof_off + ld);
        s_fid[el][3 * a + c] = factor_index(s, ld);
        s_du[el][3 * a + c] = A.du[s.dof_off + ld];
      }
      if (a == 0) {
        s_band[el] = s.band_off;
        s_Wb[el] = s.Wb;
        s_b[el] = s.b;
      }
    }
  }
  __syncthreads();
  // an element of this block takes part (MODE 2: its subdomain is flagged)
  auto active = [&](int el) {
    const int64_t ci = first + el;
    return ci < A.n_colour && (MODE != 2 || A.need[A.elem_sub[A.elems[ci]]]);
  };
  // return map: one thread per (element, Gauss point)
  if (tid < kElemPerBlock * 8) {
    int el = tid / 8, g = tid % 8;
    int64_t ci = first + el;
    if (active(el)) {
      int32_t e = A.elems[ci];
      int64_t gp = 8 * (int64_t)e + g;
      double de[6] = {0, 0, 0, 0, 0, 0};
      for (int a = 0; a < 8; ++a)
        for (int c = 0; c < 3; ++c) {
          double u = s_du[el][3 * a + c];
          for (int t = 0; t < 3; ++t) de[c_rows[c][t]] += s_dN[g][a][c_axis[c][t]] * u;
        }
      double sg[6], ds[6], dk;
      for (int i = 0; i < 6; ++i) sg[i] = A.sigma[6 * gp + i];
      bool plastic;
      return_map_point(A.M, sg, A.kappa[gp], de, ds, &dk, MODE == 2 ? &s_D[el][g][0] : nullptr, &plastic);
      if (MODE == 1) {
        for (int i = 0; i < 6; ++i) {
          A.dsigma[6 * gp + i] = ds[i];
          s_ds[el][g][i] = A.w * ds[i];
        }
        A.dkappa[gp] = dk;
        A.plastic[gp] = plastic ? 1 : 0;
        if (plastic) atomicAdd(&s_cnt, 1);
      }
    }
  }
  __syncthreads();
  if (MODE == 1) {
    if (tid == 0 && s_cnt) atomicAdd(A.plastic_count, (unsigned long long)s_cnt);
  }
  // internal force: one thread per (element, element DOF)
  for (int q = tid; q < (MODE == 1 ? kElemPerBlock * 24 : 0); q += blockDim.x) {
    int el = q / 24, al = q % 24;
    if (first + el >= A.n_colour) continue;
    int a = al / 3, c = al % 3;
    double f = 0.0;
    for (int g = 0; g < 8; ++g)
      for (int t = 0; t < 3; ++t) f += s_dN[g][a][c_axis[c][t]] * s_ds[el][g][c_rows[c][t]];
    A.fint[s_dof[el][al]] += f;
  }
  // tangent: the 300 lower entries of each element matrix
  for (int q = tid; q < (MODE == 2 ? kElemPerBlock * 300 : 0); q += blockDim.x) {
    int el = q / 300, r = q % 300;
    if (!active(el)) continue;
    // r -> (al, be) with al >= be, row-major lower triangle
    int al = (int)((sqrt(8.0 * r + 1.0) - 1.0) * 0.5);
    while ((al + 1) * (al + 2) / 2 <= r) ++al;
    while (al * (al + 1) / 2 > r) --al;
    int be = r - al * (al + 1) / 2;
    int a = al / 3, c = al % 3, bn = be / 3, d = be % 3;
    double kv = 0.0;
    for (int g = 0; g < 8; ++g) {
      const double* D = &s_D[MODE == 2 ? el : 0][g][0];
      for (int u = 0; u < 3; ++u) {
        double lu = s_dN[g][a][c_axis[c][u]];
        int ru = c_rows[c][u];
        double acc = 0.0;
        for (int v = 0; v < 3; ++v) acc += D[6 * ru + c_rows[d][v]] * s_dN[g][bn][c_axis[d][v]];
        kv += lu * acc;
      }
    }
    kv *= A.w;
    int32_t fa = s_fid[el][al], fb = s_fid[el][be];
    int32_t row = fa > fb ? fa : fb, col = fa > fb ? fb : fa;
    int64_t off = s_band[el] + (int64_t)row * s_Wb[el] + (col - row + s_b[el]);
    A.band[off] += kv;
  }
}

void launch_assemble(const AssembleArgs& args, int mode, hipStream_t st) {
  if (args.n_colour <= 0) return;
  int64_t blocks = (args.n_colour + kElemPerBlock - 1) / kElemPerBlock;
  if (mode == 1)
    assemble_kernel<1><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(args);
  else
    assemble_kernel<2><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(args);
}

// identity rows for the padding of the listed subdomain factors (all if
// list is NULL)
__global__ void pad_identity_kernel(const SubDev* __restrict__ subs, int64_t nsub, const int32_t* __restrict__ list,
                                    double* __restrict__ band) {
  if ((int64_t)blockIdx.x >= nsub) return;
  const int64_t p = list ? list[blockIdx.x] : blockIdx.x;
  const SubDev s = subs[p];
  for (int32_t r = s.ndof + threadIdx.x; r < s.npad; r += blockDim.x)
    band[s.band_off + (int64_t)r * s.Wb + s.b] = 1.0;
}

void launch_pad_identity(const SubDev* subs, int64_t nsub, const int32_t* list, double* band, hipStream_t st) {
  if (nsub > 0) pad_identity_kernel<<<dim3((unsigned)nsub), dim3(64), 0, st>>>(subs, nsub, list, band);
}

// K_bb values for the lumped preconditioner (before regularization)
// K_bb values of the lumped preconditioner, read from the assembled band:
// one thread per lane slot of a group walks its neighbour mask in bit order
// and writes the three entries (components 0, 1, 2) coupling its touched
// DOF to each masked node, zeros past its own count; the band position of
// entry (f, f2) is row max(f, f2), column min(f, f2).
template <typename T>
__global__ __launch_bounds__(256) void gather_kbb_kernel(DualMaps M, const double* __restrict__ band,
                                                         const uint8_t* __restrict__ need, T* __restrict__ out) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = slot / 64;
  if (g >= M.kbb_groups) return;
  if (need && !need[M.kbb_gsub[g]]) return;
  const int lane = (int)(slot % 64);
  const int nb = M.kbb_gnb[g];
  T* o = out + M.kbb_goff[g] + lane;
  const int32_t it = M.kbb_row[slot];
  uint32_t mask = M.kbb_mask[slot];
  int b = 0;
  if (it >= 0) {
    const SubDev s = M.subs[M.kbb_gsub[g]];
    const int32_t ld = M.if_ldof[it], a = ld / 3;
    const int32_t f = factor_index(s, ld);
    const double* A = band + s.band_off;
    for (; mask; ++b) {
      const int k = __ffs(mask) - 1;
      mask &= mask - 1;
      const int32_t a2 = a + (k % 3 - 1) + s.N[0] * ((k / 3) % 3 - 1 + s.N[1] * (k / 9 - 1));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int32_t f2 = factor_index(s, 3 * a2 + c);
        const int32_t r = f > f2 ? f : f2, cc = f > f2 ? f2 : f;
        o[(int64_t)(3 * b + c) * 64] = (T)A[(int64_t)r * s.Wb + (cc - r + s.b)];
      }
    }
  }
  for (; b < nb; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) o[(int64_t)(3 * b + c) * 64] = T(0);
}

template <typename T>
void launch_gather_kbb(const DualMaps& M, const double* band, const uint8_t* need, T* out, hipStream_t st) {
  const int64_t slots = 64 * M.kbb_groups;
  if (slots > 0)
    gather_kbb_kernel<T><<<dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st>>>(M, band, need, out);
}
template void launch_gather_kbb<double>(const DualMaps&, const double*, const uint8_t*, double*, hipStream_t);
template void launch_gather_kbb<float>(const DualMaps&, const double*, const uint8_t*, float*, hipStream_t);

// K_bb values of the listed subdomains copied from src (whole groups)
template <typename T>
__global__ __launch_bounds__(256) void copy_kbb_kernel(DualMaps M, int64_t count, const int32_t* __restrict__ list,
                                                       const T* __restrict__ src, T* __restrict__ dst) {
  if ((int64_t)blockIdx.y >= count) return;
  const int32_t p = list[blockIdx.y];
  const int64_t v0 = M.kbb_goff[M.kbb_g0[p]], v1 = M.kbb_goff[M.kbb_g0[p + 1]];
  for (int64_t i = v0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v1; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename T>
void launch_copy_kbb(const DualMaps& M, int64_t count, const int32_t* list, const T* src, T* dst, hipStream_t st) {
  if (count > 0) copy_kbb_kernel<T><<<dim3(16, (unsigned)count), dim3(256), 0, st>>>(M, count, list, src, dst);
}
template void launch_copy_kbb<double>(const DualMaps&, int64_t, const int32_t*, const double*, double*, hipStream_t);
template void launch_copy_kbb<float>(const DualMaps&, int64_t, const int32_t*, const float*, float*, hipStream_t);

// K_reg = K + rho Q Q^T at the fixing DOFs, rho = max_j K[j, j] (Remark 1)
__global__ __launch_bounds__(256) void regularize_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                         const int32_t* __restrict__ list,
                                                         const double* __restrict__ QQt, double* __restrict__ band) {
  __shared__ double red[256];
  if ((int64_t)blockIdx.x >= count) return;
  const int64_t p = list ? list[blockIdx.x] : blockIdx.x;
  const int32_t ndof = subs[p].ndof, Wb = subs[p].Wb, b = subs[p].b;
  const int64_t boff = subs[p].band_off;
  double mx = 0.0;
  for (int32_t r = threadIdx.x; r < ndof; r += blockDim.x) {
    double v = band[boff + (int64_t)r * Wb + b];
    mx = v > mx ? v : mx;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  double rho = red[0];
  if (threadIdx.x < 81) {
    int i = threadIdx.x / 9, j = threadIdx.x % 9;
    const int32_t* fix = subs[p].fix;
    int32_t fi = fix[i], fj = fix[j];
    if (fi >= fj) band[boff + (int64_t)fi * Wb + (fj - fi + b)] += rho * QQt[81 * p + 9 * i + j];
  }
}

void launch_regularize(const SubDev* subs, int64_t count, const int32_t* list, const double* QQt, double* band,
                       hipStream_t st) {
  if (count > 0) regularize_kernel<<<dim3((unsigned)count), dim3(256), 0, st>>>(subs, count, list, QQt, band);
}

// flags[p] = 1 if a Gauss point of subdomain p is on the plastic branch
__global__ __launch_bounds__(256) void sub_plastic_kernel(const SubDev* __restrict__ subs, int64_t nsub,
                                                          const uint8_t* __restrict__ plastic,
                                                          int32_t* __restrict__ flags) {
  const int64_t p = blockIdx.x;
  if (p >= nsub) return;
  const int64_t g0 = 8 * subs[p].elem_off, ng = 8 * (int64_t)subs[p].n_elem;
  int any = 0;
  for (int64_t g = threadIdx.x; g < ng; g += blockDim.x) any |= plastic[g0 + g] != 0;
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[p] = any ? 1 : 0;
}

void launch_sub_plastic(const SubDev* subs, int64_t nsub, const uint8_t* plastic, int32_t* flags, hipStream_t st) {
  if (nsub > 0) sub_plastic_kernel<<<dim3((unsigned)nsub), dim3(256), 0, st>>>(subs, nsub, plastic, flags);
}

}  // namespace tfeti

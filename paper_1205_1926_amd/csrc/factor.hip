// Batched band Cholesky of the regularized subdomain tangents (Remark 1:
// regularized blocks factorized by a standard Cholesky method for
// nonsingular matrices), panel packing for the triangular solves, and the
// dense inverse of the coarse matrix G G^T.
//
// Storage: row-band, row r holds columns r-b..r (entry (r, k) is column
// r-b+k, k = b the diagonal); rows are the subdomain DOFs in the factor
// ordering, padded with identity rows to a multiple of 64.
#include "kernels.h"

namespace tfeti {

namespace {

template <typename T>
__device__ __forceinline__ T bcast_lane(T v, int l);

template <>
__device__ __forceinline__ float bcast_lane<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ double bcast_lane<double>(double v, int l) {
  long long x = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffLL), l);
  int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int NB = 32;     // factorization block (diagonal tile) size
constexpr int TT = 64;     // trailing-update tile edge

}  // namespace

// One workgroup (256 threads) per band matrix; right-looking blocked
// algorithm: Cholesky of the NB x NB diagonal tile by one wave in registers,
// triangular solve of the rows below it that lie in the band, then the
// symmetric rank-NB update of the trailing band window in 64 x 64 tiles.
template <typename T>
__global__ __launch_bounds__(256) void band_cholesky_kernel(const SubDev* __restrict__ subs, int64_t nsub,
                                                            T* __restrict__ W, int32_t* __restrict__ fail) {
  __shared__ T sL[NB][NB + 1];
  __shared__ T sR[TT][NB + 1];
  __shared__ T sC[TT][NB + 1];
  __shared__ int s_fail;
  const int64_t p = blockIdx.x;
  if (p >= nsub) return;
  const SubDev s = subs[p];
  T* A = W + s.band_off;
  const int b = s.b, Wb = s.Wb, n = s.npad;
  const int tid = threadIdx.x;
  if (tid == 0) s_fail = 0;
  __syncthreads();
  auto at = [&](int r, int c) -> T& { return A[(int64_t)r * Wb + (c - r + b)]; };

  for (int J = 0; J < n; J += NB) {
    const int jb = (n - J) < NB ? (n - J) : NB;
    // ---- 1. diagonal tile by wave 0, lane = row ----
    if (tid < 64) {
      const int i = tid;
      T a[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) a[j] = (i < jb && j <= i && (i - j) <= b) ? at(J + i, J + j) : T(0);
      bool bad = false;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k < jb) {
          T dkk = bcast_lane(a[k], k);
          if (!(dkk > T(0))) {
            bad = true;
            dkk = T(1);
          }
          T lkk = sqrt(dkk);
          if (i == k) a[k] = lkk;
          if (i > k) a[k] = a[k] / lkk;
#pragma unroll
          for (int j = k + 1; j < NB; ++j) {
            T ljk = bcast_lane(a[k], j);
            if (i >= j && j < jb) a[j] -= a[k] * ljk;
          }
        }
      }
      if (bad && i == 0) s_fail = 1;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (i < jb && j <= i && (i - j) <= b) at(J + i, J + j) = a[j];
        if (i < NB) sL[i][j] = a[j];
      }
    }
    __syncthreads();
    const int rbeg = J + jb;
    int rend = J + jb + b;        // rows r with r - b <= J + jb - 1
    if (rend > n) rend = n;
    // ---- 2. rows below: x := x L_JJ^{-T} ----
    for (int r = rbeg + tid; r < rend; r += blockDim.x) {
      T x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = (j < jb && r - (J + j) <= b) ? at(r, J + j) : T(0);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < jb) {
          T v = x[j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= x[k] * sL[j][k];
          x[j] = v / sL[j][j];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < jb && r - (J + j) <= b) at(r, J + j) = x[j];
    }
    __syncthreads();
    // ---- 3. trailing update of the band window ----
    for (int RT = rbeg; RT < rend; RT += TT) {
      for (int CT = rbeg; CT <= RT; CT += TT) {
        if (RT - (CT + TT - 1) > b) continue;
        for (int q = tid; q < TT * NB; q += blockDim.x) {
          int i = q / NB, k = q % NB;
          int r = RT + i, c = CT + i;
          sR[i][k] = (k < jb && r < rend && r - (J + k) <= b) ? at(r, J + k) : T(0);
          sC[i][k] = (k < jb && c < rend && c - (J + k) <= b) ? at(c, J + k) : T(0);
        }
        __syncthreads();
        const int ty = tid / 16, tx = tid % 16;
        T acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
        for (int k = 0; k < NB; ++k) {
          T ra[4], cb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) ra[u] = sR[ty * 4 + u][k];
#pragma unroll
          for (int v = 0; v < 4; ++v) cb[v] = sC[tx + 16 * v][k];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += ra[u] * cb[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            int r = RT + ty * 4 + u, c = CT + tx + 16 * v;
            if (r < rend && c <= r && r - c <= b) at(r, c) -= acc[u][v];
          }
        __syncthreads();
      }
    }
  }
  if (tid == 0 && s_fail) atomicOr(fail, 1);
}

template <typename T>
void launch_band_cholesky(const SubDev* subs, int64_t nsub, T* band, int32_t* fail, hipStream_t st) {
  band_cholesky_kernel<T><<<dim3((unsigned)nsub), dim3(256), 0, st>>>(subs, nsub, band, fail);
}
template void launch_band_cholesky<double>(const SubDev*, int64_t, double*, int32_t*, hipStream_t);
template void launch_band_cholesky<float>(const SubDev*, int64_t, float*, int32_t*, hipStream_t);

template <typename T>
__global__ void convert_band_kernel(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = (T)src[i];
}

template <typename T>
void launch_convert_band(const double* src, T* dst, int64_t n, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (n > 0) convert_band_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(src, dst, n);
}
template void launch_convert_band<double>(const double*, double*, int64_t, hipStream_t);
template void launch_convert_band<float>(const double*, float*, int64_t, hipStream_t);

// Panels.  Tile rows TS, vector width V = 16 bytes / sizeof(T).
// Forward panel of block row I: off-diagonal columns [I TS - w_I, I TS) then
// the inverted diagonal tile; chunk (cc, r) of V consecutive columns of row
// r is stored at ((cc TS) + r) V.  Backward panel of block column I: the
// inverted diagonal tile rows first, then rows [(I+1) TS, (I+1) TS + w'_I);
// chunk (rc, c) of V consecutive rows of column c is stored at (rc TS + c) V.
template <typename T, int TS>
__global__ __launch_bounds__(256) void pack_panels_kernel(const SubDev* __restrict__ subs, int64_t nsub,
                                                          const T* __restrict__ W, T* __restrict__ Fp,
                                                          T* __restrict__ Bp) {
  constexpr int V = 16 / sizeof(T);
  // sD holds the diagonal tile L in its lower triangle and, after the
  // inversion, X = L^{-1} transposed in its strict upper triangle
  // (sD[c][r] = X[r][c], r > c); sXd holds the diagonal of X.
  __shared__ double sD[TS][TS + 1];
  __shared__ double sXd[TS];
  const int64_t p = blockIdx.x;
  if (p >= nsub) return;
  const SubDev s = subs[p];
  const T* A = W + s.band_off;
  T* F = Fp + s.panel_off;
  T* Bk = Bp + s.panel_off;
  const int b = s.b, Wb = s.Wb, n = s.npad, nb = n / TS;
  const int tid = threadIdx.x;
  auto L = [&](int r, int c) -> T { return (c <= r && r - c <= b && c >= 0) ? A[(int64_t)r * Wb + (c - r + b)] : T(0); };
  int64_t offF = 0, offB = 0;
  for (int I = 0; I < nb; ++I) {
    const int wF = I * TS < s.bo ? I * TS : s.bo;
    const int rem = n - (I + 1) * TS;
    const int wB = rem < s.bo ? rem : s.bo;
    for (int q = tid; q < TS * TS; q += blockDim.x) {
      int i = q / TS, j = q % TS;
      sD[i][j] = (i >= j) ? (double)L(I * TS + i, I * TS + j) : 0.0;
    }
    __syncthreads();
    // inverse of the lower-triangular diagonal tile, one column per thread
    if (tid < TS) {
      const int j = tid;
      const double xjj = 1.0 / sD[j][j];
      sXd[j] = xjj;
      for (int i = j + 1; i < TS; ++i) {
        double v = sD[i][j] * xjj;
        for (int k = j + 1; k < i; ++k) v += sD[i][k] * sD[j][k];
        sD[j][i] = -v / sD[i][i];
      }
    }
    __syncthreads();
    // diagonal chunks of both layouts
    for (int q = tid; q < TS * TS; q += blockDim.x) {
      int r = q / TS, c = q % TS;
      double x = (r == c) ? sXd[c] : (r > c ? sD[c][r] : 0.0);
      T v = (T)x;
      F[offF + ((int64_t)((wF + c) / V) * TS + r) * V + (c % V)] = v;
      Bk[offB + ((int64_t)(r / V) * TS + c) * V + (r % V)] = v;
    }
    // off-diagonal part of the forward panel: columns I TS - wF .. I TS - 1
    for (int64_t q = tid; q < (int64_t)TS * wF; q += blockDim.x) {
      int r = (int)(q % TS), cc = (int)(q / TS);
      int col = I * TS - wF + cc;
      F[offF + ((int64_t)(cc / V) * TS + r) * V + (cc % V)] = L(I * TS + r, col);
    }
    // off-diagonal part of the backward panel: rows (I+1) TS .. + wB - 1
    for (int64_t q = tid; q < (int64_t)TS * wB; q += blockDim.x) {
      int c = (int)(q % TS), rr = (int)(q / TS);
      int row = (I + 1) * TS + rr;
      Bk[offB + ((int64_t)((TS + rr) / V) * TS + c) * V + ((TS + rr) % V)] = L(row, I * TS + c);
    }
    offF += (int64_t)TS * (wF + TS);
    offB += (int64_t)TS * (TS + wB);
    __syncthreads();
  }
}

template <typename T>
void launch_pack_panels(const SubDev* subs, int64_t nsub, const T* band, T* Fp, T* Bp, int TS, hipStream_t st) {
  if (TS == 16)
    pack_panels_kernel<T, 16><<<dim3((unsigned)nsub), dim3(256), 0, st>>>(subs, nsub, band, Fp, Bp);
  else if (TS == 32)
    pack_panels_kernel<T, 32><<<dim3((unsigned)nsub), dim3(256), 0, st>>>(subs, nsub, band, Fp, Bp);
  else
    pack_panels_kernel<T, 64><<<dim3((unsigned)nsub), dim3(256), 0, st>>>(subs, nsub, band, Fp, Bp);
}
template void launch_pack_panels<double>(const SubDev*, int64_t, const double*, double*, double*, int, hipStream_t);
template void launch_pack_panels<float>(const SubDev*, int64_t, const float*, float*, float*, int, hipStream_t);

// Dense inverse of the coarse matrix from its banded Cholesky factor L
// (row-band, l rows, half bandwidth b): thread j solves L L^T x = e_j and
// writes column j of Ginv (l x l, row-major); a wave's threads hold
// consecutive columns, so every access to Ginv is coalesced.
__global__ __launch_bounds__(64) void coarse_inverse_kernel(const double* __restrict__ L, int32_t l, int32_t b,
                                                            int32_t Wc, double* __restrict__ G) {
  const int j0 = blockIdx.x * 64;
  const int j = j0 + threadIdx.x;
  const bool act = j < l;
  auto Lat = [&](int r, int c) -> double { return L[(int64_t)r * Wc + (c - r + b)]; };
  // forward: L y = e_j (rows from the wave's first column on)
  for (int i = j0; i < l; ++i) {
    double sum = (i == j) ? 1.0 : 0.0;
    int t0 = i - b > j0 ? i - b : j0;
    for (int t = t0; t < i; ++t) sum -= Lat(i, t) * (act ? G[(int64_t)t * l + j] : 0.0);
    if (act) G[(int64_t)i * l + j] = sum / Lat(i, i);
  }
  // rows above the wave's first column are zero in y
  for (int i = 0; i < j0; ++i)
    if (act) G[(int64_t)i * l + j] = 0.0;
  // backward: L^T x = y
  for (int i = l - 1; i >= 0; --i) {
    double sum = act ? G[(int64_t)i * l + j] : 0.0;
    int t1 = i + b < l - 1 ? i + b : l - 1;
    for (int t = i + 1; t <= t1; ++t) sum -= Lat(t, i) * (act ? G[(int64_t)t * l + j] : 0.0);
    if (act) G[(int64_t)i * l + j] = sum / Lat(i, i);
  }
}

void launch_coarse_inverse(const double* L, int32_t l, int32_t b, int32_t Wc, double* Ginv, hipStream_t st) {
  int blocks = (l + 63) / 64;
  coarse_inverse_kernel<<<dim3(blocks), dim3(64), 0, st>>>(L, l, b, Wc, Ginv);
}

}  // namespace tfeti

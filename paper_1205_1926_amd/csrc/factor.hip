// Band copies, panel packing for the triangular solves, and
// the dense inverse of the coarse matrix G G^T.
//
// Storage: row-band, row r holds columns r-b..r (entry (r, k) is column
// r-b+k, k = b the diagonal); rows are the subdomain DOFs in the factor
// ordering, padded with identity rows to a multiple of 64.
#include "kernels.h"

namespace tfeti {

// Copy the row-band matrices of the listed subdomains (zero them if src is
// NULL): blockIdx.y picks the subdomain, the blockIdx.x slices stride over
// its entries.
__global__ __launch_bounds__(256) void copy_band_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                        const int32_t* __restrict__ list,
                                                        const double* __restrict__ src, double* __restrict__ dst) {
  if ((int64_t)blockIdx.y >= count) return;
  const int64_t p = list[blockIdx.y];
  const int64_t off = subs[p].band_off, len = (int64_t)subs[p].npad * subs[p].Wb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    dst[off + i] = src ? src[off + i] : 0.0;
}

void launch_copy_band(const SubDev* subs, int64_t count, const int32_t* list, const double* src, double* dst,
                      hipStream_t st) {
  if (count > 0) copy_band_kernel<<<dim3(32, (unsigned)count), dim3(256), 0, st>>>(subs, count, list, src, dst);
}

// Panels (layout in kernels.h): tile rows TS, vector width V = 16 bytes /
// sizeof(T).  Each workgroup takes block rows of one subdomain.

template <typename TW, typename T, int TS>
__global__ __launch_bounds__(256) void pack_panels_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                          const int32_t* __restrict__ list,
                                                          const TW* __restrict__ W, T* __restrict__ Fp,
                                                          T* __restrict__ Bp, float* __restrict__ Fq,
                                                          float* __restrict__ Bq) {
  constexpr int V = 16 / sizeof(T);
  // sD holds the diagonal tile L in its lower triangle and, after the
  // inversion, X = L^{-1} transposed in its strict upper triangle
  // (sD[c][r] = X[r][c], r > c); sXd holds the diagonal of X.
  __shared__ double sD[TS][TS + 1];
  __shared__ double sXd[TS];
  if ((int64_t)blockIdx.y >= count) return;
  const int64_t p = list ? list[blockIdx.y] : blockIdx.y;
  const SubDev s = subs[p];
  const TW* A = W + s.band_off;
  T* F = Fp + s.panel_off;
  T* Bk = Bp + s.panel_off;
  // optional second copy in FP32 (its own chunk width V2) from the same pass
  constexpr int V2 = 4;
  float* F2 = Fq ? Fq + s.panel_off : nullptr;
  float* B2 = Bq ? Bq + s.panel_off : nullptr;
  const int b = s.b, Wb = s.Wb, n = s.npad, nb = n / TS;
  const int tid = threadIdx.x;
  auto L = [&](int r, int c) -> T { return (c <= r && r - c <= b && c >= 0) ? (T)A[(int64_t)r * Wb + (c - r + b)] : T(0); };
  auto put = [](T* dst, const double* v) {
    if constexpr (V == 2)
      *reinterpret_cast<double2*>(dst) = double2{v[0], v[1]};
    else
      *reinterpret_cast<float4*>(dst) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  };
  auto put32 = [](float* dst, const double* v) {
    *reinterpret_cast<float4*>(dst) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  };
  // entries of a TS x TS tile per thread, loaded one tile ahead
  constexpr int TPT = (TS * TS + 255) / 256;
  // block columns J = blockIdx.x, blockIdx.x + gridDim.x, ...: the diagonal
  // tile (inverted, into block row J's forward panel and block column J's
  // backward panel), then the tiles (I, J) below it inside the backward
  // window, each read once and written as one contiguous block of block
  // column J's backward panel and one of block row I's forward panel
  for (int J = blockIdx.x; J < nb; J += gridDim.x) {
    const int64_t offF = panel_fwd_offset(J, TS, s.bo), offB = panel_bwd_offset(J, TS, s.bo, n);
    const int wF = J * TS < s.bo ? J * TS : s.bo;
    const int rem = n - (J + 1) * TS;
    const int wB = rem < s.bo ? rem : s.bo;
    // the first tile below the diagonal is requested before the diagonal
    // tile's inversion, so that its loads are in flight meanwhile
    const int nI = (wB + TS - 1) / TS;
    double nx[TPT];
    auto fetch = [&](int I, double (&v)[TPT]) {
#pragma unroll
      for (int u = 0; u < TPT; ++u) {
        const int q = tid + 256 * u;
        v[u] = q < TS * TS ? (double)L(I * TS + q / TS, J * TS + q % TS) : 0.0;
      }
    };
    __syncthreads();
    for (int q = tid; q < TS * TS; q += blockDim.x) {
      int i = q / TS, j = q % TS;
      sD[i][j] = (i >= j) ? (double)L(J * TS + i, J * TS + j) : 0.0;
    }
    if (nI > 0) fetch(J + 1, nx);
    __syncthreads();
    // inverse of the lower-triangular diagonal tile, one column per thread
    if (tid < TS) tile_inverse_column(&sD[0][0], TS + 1, TS, tid, sXd);
    __syncthreads();
    // diagonal chunks of both layouts
    for (int q = tid; q < TS * TS; q += blockDim.x) {
      int r = q / TS, c = q % TS;
      double x = (r == c) ? sXd[c] : (r > c ? sD[c][r] : 0.0);
      T v = (T)x;
      F[offF + ((int64_t)((wF + c) / V) * TS + r) * V + (c % V)] = v;
      Bk[offB + ((int64_t)(r / V) * TS + c) * V + (r % V)] = v;
      if (F2) {
        F2[offF + ((int64_t)((wF + c) / V2) * TS + r) * V2 + (c % V2)] = (float)x;
        B2[offB + ((int64_t)(r / V2) * TS + c) * V2 + (r % V2)] = (float)x;
      }
    }
    // tiles below the diagonal: block rows I = J + 1 .. while the block row
    // starts inside the backward window (wB and the forward windows are
    // multiples of 4, so every 16-byte chunk is wholly in or out)
    for (int t = 0; t < nI; ++t) {
      const int I = J + 1 + t;
      __syncthreads();  // the previous tile (or the diagonal) is written out
#pragma unroll
      for (int u = 0; u < TPT; ++u) {
        const int q = tid + 256 * u;
        if (q < TS * TS) sD[q / TS][q % TS] = nx[u];
      }
      if (t + 1 < nI) fetch(I + 1, nx);
      __syncthreads();
      // backward panel of block column J: rows rr0 + i, chunks of V rows
      const int rr0 = t * TS;
      for (int q = tid; q < TS * TS / V; q += blockDim.x) {
        const int rl = q / TS, c = q % TS;
        if (rr0 + rl * V < wB) {
          double v[V];
#pragma unroll
          for (int k = 0; k < V; ++k) v[k] = sD[rl * V + k][c];
          put(Bk + offB + ((int64_t)((TS + rr0) / V + rl) * TS + c) * V, v);
        }
      }
      if (B2)
        for (int q = tid; q < TS * TS / V2; q += blockDim.x) {
          const int rl = q / TS, c = q % TS;
          if (rr0 + rl * V2 < wB) {
            double v[V2];
#pragma unroll
            for (int k = 0; k < V2; ++k) v[k] = sD[rl * V2 + k][c];
            put32(B2 + offB + ((int64_t)((TS + rr0) / V2 + rl) * TS + c) * V2, v);
          }
        }
      // forward panel of block row I: its columns cf0 + j (those >= 0)
      const int wFI = I * TS < s.bo ? I * TS : s.bo;
      const int cf0 = wFI - (I - J) * TS;
      const int64_t offFI = panel_fwd_offset(I, TS, s.bo);
      for (int q = tid; q < TS * TS / V; q += blockDim.x) {
        const int cl = q / TS, i = q % TS;
        if (cf0 + cl * V >= 0) {
          double v[V];
#pragma unroll
          for (int k = 0; k < V; ++k) v[k] = sD[i][cl * V + k];
          put(F + offFI + ((int64_t)((cf0 + cl * V) / V) * TS + i) * V, v);
        }
      }
      if (F2)
        for (int q = tid; q < TS * TS / V2; q += blockDim.x) {
          const int cl = q / TS, i = q % TS;
          if (cf0 + cl * V2 >= 0) {
            double v[V2];
#pragma unroll
            for (int k = 0; k < V2; ++k) v[k] = sD[i][cl * V2 + k];
            put32(F2 + offFI + ((int64_t)((cf0 + cl * V2) / V2) * TS + i) * V2, v);
          }
        }
    }
  }
}

template <typename TW, typename T>
void launch_pack_panels(const SubDev* subs, int64_t count, const int32_t* list, const TW* band, T* Fp, T* Bp, int TS,
                        hipStream_t st, float* Fq, float* Bq) {
  if (count <= 0) return;
  dim3 grid(64, (unsigned)count);  // block rows x subdomains
  if (TS == 16)
    pack_panels_kernel<TW, T, 16><<<grid, dim3(256), 0, st>>>(subs, count, list, band, Fp, Bp, Fq, Bq);
  else if (TS == 32)
    pack_panels_kernel<TW, T, 32><<<grid, dim3(256), 0, st>>>(subs, count, list, band, Fp, Bp, Fq, Bq);
  else
    pack_panels_kernel<TW, T, 64><<<grid, dim3(256), 0, st>>>(subs, count, list, band, Fp, Bp, Fq, Bq);
}
template void launch_pack_panels<double, double>(const SubDev*, int64_t, const int32_t*, const double*, double*,
                                                 double*, int, hipStream_t, float*, float*);

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

// Lt[i][k] = L[i + k][i] (row-band storage of the transpose; zero past l).
__global__ __launch_bounds__(256) void band_transpose_kernel(const double* __restrict__ L, int32_t l, int32_t b,
                                                             int32_t Wc, double* __restrict__ Lt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)l * Wc) return;
  const int32_t i = (int32_t)(q / Wc), k = (int32_t)(q - (int64_t)i * Wc);
  Lt[q] = (k <= b && i + k < l) ? L[(int64_t)(i + k) * Wc + (b - k)] : 0.0;
}

// One wavefront per column j of the inverse: y = L^{-1} e_j (rows j..l-1)
// and then x = L^{-T} y, with the vector in LDS; every step's sum over the
// band is split across the 64 lanes (coalesced row reads of L and of its
// transpose) and reduced by lane shuffles in a fixed order.  Column j of
// the symmetric inverse is written as row j.
__global__ __launch_bounds__(64) void coarse_inverse_wave_kernel(const double* __restrict__ L,
                                                                 const double* __restrict__ Lt, int32_t l, int32_t b,
                                                                 int32_t Wc, double* __restrict__ G) {
  extern __shared__ double yv[];
  const int j = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < l; i += 64) yv[i] = 0.0;
  __syncthreads();
  auto wave_sum = [&](double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  };
  for (int i = j; i < l; ++i) {
    const int t0 = i - b > j ? i - b : j;
    const double* Li = L + (int64_t)i * Wc + (b - i);
    double s = 0.0;
    for (int t = t0 + lane; t < i; t += 64) s = fma(Li[t], yv[t], s);
    s = wave_sum(s);
    if (lane == 0) yv[i] = ((i == j ? 1.0 : 0.0) - s) / Li[i];
    __syncthreads();
  }
  for (int i = l - 1; i >= 0; --i) {
    const int t1 = i + b < l - 1 ? i + b : l - 1;
    const double* Ti = Lt + (int64_t)i * Wc - i;
    double s = 0.0;
    for (int t = i + 1 + lane; t <= t1; t += 64) s = fma(Ti[t], yv[t], s);
    s = wave_sum(s);
    if (lane == 0) yv[i] = (yv[i] - s) / Ti[i];
    __syncthreads();
  }
  for (int i = lane; i < l; i += 64) G[(int64_t)j * l + i] = yv[i];
}

// Lt: scratch of l * Wc entries for the transposed factor (may be NULL:
// then the one-thread-per-column kernel runs, as it does when a column does
// not fit the LDS of a workgroup).
void launch_coarse_inverse(const double* L, int32_t l, int32_t b, int32_t Wc, double* Ginv, hipStream_t st,
                           double* Lt) {
  int dev = 0, lds = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 65536;
  const size_t shm = (size_t)l * sizeof(double);
  if (Lt && l > 0 && shm <= (size_t)lds) {
    const int64_t nt = (int64_t)l * Wc;
    band_transpose_kernel<<<dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st>>>(L, l, b, Wc, Lt);
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)coarse_inverse_wave_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm);
    coarse_inverse_wave_kernel<<<dim3((unsigned)l), dim3(64), shm, st>>>(L, Lt, l, b, Wc, Ginv);
    return;
  }
  int blocks = (l + 63) / 64;
  coarse_inverse_kernel<<<dim3(blocks), dim3(64), 0, st>>>(L, l, b, Wc, Ginv);
}

}  // namespace tfeti

// Batched band Cholesky of the regularized subdomain tangents (Remark 1:
// once regularized, each block is factorized by a standard Cholesky method
// for nonsingular matrices).
//
// Storage: row-band, row r holds columns r-b..r (entry (r, k) is column
// r-b+k, k = b the diagonal); rows are the subdomain DOFs in the factor
// ordering, padded with identity rows to a multiple of 64.
//
// One workgroup (256 threads) per band matrix, right-looking by block
// columns of NB: the panel (the NB block columns of every row the band
// reaches, at most NB + b rows) is staged in LDS and factored column by
// column with each row in a thread's registers (one barrier per column);
// the panel is written back and the trailing
// band window is updated from the LDS panel in 16 x 16 blocks on the FP64
// matrix cores (FP32: 64 x 64 tiles, 4 x 4 outputs per thread), so global
// traffic is one read-modify-write of the window per block column.
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

constexpr int TT = 64;  // trailing-update tile edge

}  // namespace

template <typename T, int NB>
__global__ __launch_bounds__(256, 2) void band_cholesky_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                            const int32_t* __restrict__ list,
                                                            T* __restrict__ W, int32_t* __restrict__ fail) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* Lp = reinterpret_cast<T*>(smem);          // panel rows x (NB + 1)
  constexpr int LS = NB + 1;
  __shared__ int s_fail;
  if ((int64_t)blockIdx.x >= count) return;
  const int64_t p = list ? list[blockIdx.x] : blockIdx.x;
  const int b = subs[p].b, Wb = subs[p].Wb, n = subs[p].npad;
  T* A = W + subs[p].band_off;
  const int tid = threadIdx.x;
  if (tid == 0) s_fail = 0;

  for (int J = 0; J < n; J += NB) {
    const int jb = (n - J) < NB ? (n - J) : NB;
    int rend = J + jb + b;
    if (rend > n) rend = n;
    const int nr = rend - J;                      // panel rows (>= jb)
    // ---- stage the panel (8 loads in flight per thread) ----
    for (int q0 = tid; q0 < nr * NB; q0 += 8 * 256) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * 256;
        const int r = q / NB, j = q - (q / NB) * NB;
        v[u] = (q < nr * NB && j < jb && j <= r && r - j <= b) ? A[(int64_t)(J + r) * Wb + (j - r + b)] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * 256;
        if (q < nr * NB) Lp[(q / NB) * LS + (q - (q / NB) * NB)] = v[u];
      }
    }
    __syncthreads();
    // ---- panel factorization, column by column: thread r < blockDim.x
    //      keeps row r of the panel in registers; at column j every row
    //      below j takes L[r][j] = (x_r[j] - x_r[0:j] . L[j][0:j]) / L[j][j]
    //      with row j read from LDS (one address for all lanes), and row j+1
    //      completes its diagonal entry and publishes itself for the next
    //      column; one barrier per column ----
    {
      const int r = tid;
      const bool have = r < nr;
      T x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = have ? Lp[r * LS + j] : T(0);
      bool bad = false;
      if (r == 0 && jb > 0) {
        T d = x[0];
        if (!(d > T(0))) {
          bad = true;
          d = T(1);
        }
        x[0] = sqrt(d);
        Lp[0] = x[0];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < jb) {
          if (have && r > j) {
            T v = x[j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= x[k] * Lp[j * LS + k];
            x[j] = v / Lp[j * LS + j];
            if (r == j + 1 && j + 1 < jb) {
              T d = x[j + 1];
#pragma unroll
              for (int k = 0; k <= j; ++k) d -= x[k] * x[k];
              if (!(d > T(0))) {
                bad = true;
                d = T(1);
              }
              x[j + 1] = sqrt(d);
#pragma unroll
              for (int k = 0; k <= j + 1; ++k) Lp[r * LS + k] = x[k];
            }
          }
          __syncthreads();
        }
      }
      if (bad) s_fail = 1;
      if (have) {
#pragma unroll
        for (int j = 0; j < NB; ++j) Lp[r * LS + j] = x[j];
      }
    }
    __syncthreads();
    // ---- rows past the first blockDim.x: solved against the finished
    //      diagonal tile, independently ----
    for (int r = (int)blockDim.x + tid; r < nr; r += blockDim.x) {
      T x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = Lp[r * LS + j];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < jb) {
          T v = x[j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= x[k] * Lp[j * LS + k];
          x[j] = v / Lp[j * LS + j];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) Lp[r * LS + j] = x[j];
    }
    __syncthreads();
    // ---- write the panel back ----
    for (int q = tid; q < nr * NB; q += blockDim.x) {
      const int r = q / NB, j = q - (q / NB) * NB;
      if (j < jb && j <= r && r - j <= b) A[(int64_t)(J + r) * Wb + (j - r + b)] = Lp[r * LS + j];
    }
    // ---- trailing update from the LDS panel (columns >= J + jb only) ----
    if constexpr (sizeof(T) == 8) {
      // 16 x 16 blocks of the lower band window on the FP64 matrix cores:
      // block (RB, CB) accumulates P_R P_C^T over the panel columns, 4 at a
      // time (lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; output r
      // of lane l is D[l / 16 + 4 r][l % 16])
      const int nwin = nr - jb, nbw = (nwin + 15) / 16;
      const int wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
      const int nblk = nbw * (nbw + 1) / 2;
      typedef double d4 __attribute__((ext_vector_type(4)));
      // this wave's blocks are q = wave + 4 i; they are processed BT at a
      // time, the window values of the next batch loaded while the current
      // batch runs its (interleaved) matrix-core chains
      constexpr int BT = 4;
      const int nmine = nblk > wave ? (nblk - wave + 3) / 4 : 0;
      auto block_of = [&](int i, int& RB, int& CB) -> bool {
        const int q = wave + 4 * i;
        if (i >= nmine) return false;
        RB = (int)sqrtf(2.0f * (float)q);
        while (RB * (RB + 1) / 2 > q) --RB;
        while ((RB + 1) * (RB + 2) / 2 <= q) ++RB;
        CB = q - RB * (RB + 1) / 2;
        return RB * 16 - (CB * 16 + 15) <= b;  // inside the band
      };
      auto load_batch = [&](int i0, T (&c)[BT][4]) {
#pragma unroll
        for (int t = 0; t < BT; ++t) {
          int RB = 0, CB = 0;
          const bool ok = block_of(i0 + t, RB, CB);
          const int row0 = J + jb + RB * 16 + lk, col = J + jb + CB * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = row0 + 4 * r;
            const bool in = ok && row < rend && col <= row && row - col <= b;
            c[t][r] = in ? A[(int64_t)row * Wb + (col - row + b)] : T(0);
          }
        }
      };
      T cur[BT][4], nxt[BT][4];
      if (nmine > 0) load_batch(0, cur);
      for (int i0 = 0; i0 < nmine; i0 += BT) {
        if (i0 + BT < nmine) load_batch(i0 + BT, nxt);
        int ra[BT], rb[BT], row0[BT], col[BT];
        bool ok[BT];
#pragma unroll
        for (int t = 0; t < BT; ++t) {
          int RB = 0, CB = 0;
          ok[t] = block_of(i0 + t, RB, CB);
          ra[t] = jb + RB * 16 + li;
          rb[t] = jb + CB * 16 + li;
          row0[t] = J + jb + RB * 16 + lk;
          col[t] = J + jb + CB * 16 + li;
        }
        d4 acc[BT];
#pragma unroll
        for (int t = 0; t < BT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
        // operand rows past the panel (and blocks outside the band) read
        // row 0 instead: their products only reach outputs that are not
        // written back, so they need no zeroing, only an address in bounds
        const T* pa[BT];
        const T* pb[BT];
#pragma unroll
        for (int t = 0; t < BT; ++t) {
          pa[t] = Lp + (ok[t] && ra[t] < nr ? ra[t] : 0) * LS + lk;
          pb[t] = Lp + (ok[t] && rb[t] < nr ? rb[t] : 0) * LS + lk;
        }
        if (jb == NB) {
#pragma unroll
          for (int k0 = 0; k0 < NB; k0 += 4) {
            double av[BT], bv[BT];
#pragma unroll
            for (int t = 0; t < BT; ++t) {
              av[t] = (double)pa[t][k0];
              bv[t] = (double)pb[t][k0];
            }
#pragma unroll
            for (int t = 0; t < BT; ++t)
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc[t], 0, 0, 0);
          }
        } else {
          for (int k0 = 0; k0 < jb; k0 += 4) {
            const bool kin = k0 + lk < jb;
            double av[BT], bv[BT];
#pragma unroll
            for (int t = 0; t < BT; ++t) {
              av[t] = kin ? (double)pa[t][k0] : 0.0;
              bv[t] = kin ? (double)pb[t][k0] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < BT; ++t)
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc[t], 0, 0, 0);
          }
        }
#pragma unroll
        for (int t = 0; t < BT; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = row0[t] + 4 * r;
            if (ok[t] && row < rend && col[t] <= row && row - col[t] <= b)
              A[(int64_t)row * Wb + (col[t] - row + b)] = cur[t][r] - (T)acc[t][r];
          }
        }
#pragma unroll
        for (int t = 0; t < BT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) cur[t][r] = nxt[t][r];
      }
    } else {
      const int rbeg = J + jb;
      const int ty = tid / 16, tx = tid % 16;
      for (int RT = rbeg; RT < rend; RT += TT) {
        for (int CT = rbeg; CT <= RT; CT += TT) {
          if (RT - (CT + TT - 1) > b) continue;
          int ri[4], ci[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            int r = RT + ty * 4 + u - J;
            ri[u] = (r < nr ? r : nr - 1) * LS;
            int c = CT + tx + 16 * u - J;
            ci[u] = (c < nr ? c : nr - 1) * LS;
          }
          T acc[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
          for (int k = 0; k < jb; ++k) {
            T ra[4], cb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) ra[u] = Lp[ri[u] + k];
#pragma unroll
            for (int v = 0; v < 4; ++v) cb[v] = Lp[ci[v] + k];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[u][v] += ra[u] * cb[v];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = RT + ty * 4 + u, c = CT + tx + 16 * v;
              if (r < rend && c <= r && r - c <= b) A[(int64_t)r * Wb + (c - r + b)] -= acc[u][v];
            }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && s_fail) atomicOr(fail, 1);
}

namespace {
int g_smem_limit = 0;
}

int band_cholesky_nb(int bmax, size_t elem) {
  if (g_smem_limit == 0) {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 65536;
    g_smem_limit = v;
  }
  for (int nb : {32, 16, 8})
    if ((size_t)(nb + bmax) * (nb + 1) * elem <= (size_t)g_smem_limit) return nb;
  return 0;
}

template <typename T, int NB>
static int launch_nb(const SubDev* subs, int64_t nsub, const int32_t* list, T* band, int32_t* fail, int bmax,
                     hipStream_t st) {
  size_t shm = (size_t)(NB + bmax) * (NB + 1) * sizeof(T);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)band_cholesky_kernel<T, NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  if (nsub > 0) band_cholesky_kernel<T, NB><<<dim3((unsigned)nsub), dim3(256), shm, st>>>(subs, nsub, list, band, fail);
  return 0;
}

template <typename T>
int launch_band_cholesky(const SubDev* subs, int64_t nsub, const int32_t* list, T* band, int32_t* fail, int bmax,
                         int nb, hipStream_t st) {
  if (nb <= 0) nb = band_cholesky_nb(bmax, sizeof(T));
  switch (nb) {
    case 32:
      return launch_nb<T, 32>(subs, nsub, list, band, fail, bmax, st);
    case 16:
      return launch_nb<T, 16>(subs, nsub, list, band, fail, bmax, st);
    case 8:
      return launch_nb<T, 8>(subs, nsub, list, band, fail, bmax, st);
    default:
      return -1;
  }
}
template int launch_band_cholesky<double>(const SubDev*, int64_t, const int32_t*, double*, int32_t*, int, int,
                                          hipStream_t);
template int launch_band_cholesky<float>(const SubDev*, int64_t, const int32_t*, float*, int32_t*, int, int,
                                         hipStream_t);

}  // namespace tfeti

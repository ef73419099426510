// Batched band Cholesky of the regularized subdomain tangents (Remark 1:
// once regularized, each block is factorized by a standard Cholesky method
// for nonsingular matrices).
//
// Storage: row-band, row r holds columns r-b..r (entry (r, k) is column
// r-b+k, k = b the diagonal); rows are the subdomain DOFs in the factor
// ordering, padded with identity rows to a multiple of 64.
//
// One workgroup (256 threads) per band matrix, left-looking by block columns
// of NB.  Per block column J (the panel: the NB columns of every row the
// band reaches, at most NB + b rows):
//  U. the panel takes its updates from the finished columns in the band,
//     A_panel - L_panel,k L_tile,k^T over k in [J - b, J), on the FP64
//     matrix cores: the tile rows' L (negated) are staged in LDS, each
//     wavefront keeps the accumulators of its row blocks in registers
//     (initialized with the panel's entries) and streams its rows of L from
//     memory 16 columns at a time, the next chunk's loads in flight;
//  F. the accumulators become the LDS panel;
//  D. the diagonal tile is factored by one wavefront (one row per lane, no
//     workgroup barrier), then the rows below are solved against it;
//  W. the panel is written back.
// Finished columns are only read, so the band is written once per entry
// and no store waits on the matrix-core chain.
#include "kernels.h"

namespace tfeti {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// row stride (doubles) of the staged tile rows: whole 16-column chunks
// covering b, plus 2 so that the 16 rows of a read start in distinct banks
__host__ __device__ inline int tile_stride(int bmax) { return ((bmax + 15) / 16 * 16 + 29) / 32 * 32 + 2; }

}  // namespace

template <int NB, int G>
__global__ __launch_bounds__(256, 2) void band_cholesky_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                            const int32_t* __restrict__ list,
                                                            double* __restrict__ W, int32_t* __restrict__ fail,
                                                            int LB) {
  static_assert(NB % 16 == 0 && NB <= 64, "tile of whole 16 x 16 blocks, one row per lane of a wavefront");
  extern __shared__ __align__(16) unsigned char smem[];
  // phase U: the tile rows' negated L over the update columns (NB x LB);
  // phases F..W: the panel (rows x LS), whose diagonal tile's rows hold L in
  // slots 0..r and the transposed inverse, X[r'][r] at slot r' + 1 (r' >= r)
  double* Bt = reinterpret_cast<double*>(smem);
  double* P = reinterpret_cast<double*>(smem);
  constexpr int LS = NB + 1;
  constexpr int KS = NB / 4;   // matrix-core steps over the panel columns
  constexpr int NJ = NB / 16;  // column blocks of the panel
  __shared__ int s_fail;
  __shared__ double s_rcp[NB];  // reciprocals of the tile's diagonal
  if ((int64_t)blockIdx.x >= count) return;
  const int64_t p = list ? list[blockIdx.x] : blockIdx.x;
  const int b = subs[p].b, Wb = subs[p].Wb, n = subs[p].npad;
  double* A = W + subs[p].band_off;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
  if (tid == 0) s_fail = 0;

  for (int J = 0; J < n; J += NB) {
    const int jb = (n - J) < NB ? (n - J) : NB;
    int rend = J + jb + b;
    if (rend > n) rend = n;
    const int nr = rend - J;                      // panel rows (>= jb)
    const int nbr = (nr + 15) / 16;               // panel row blocks
    const int kbeg = J > b ? J - b : 0;           // first update column
    const int nq = (J - kbeg + 15) / 16;          // 16-column update chunks
    const bool multi = nbr > 4 * G;               // row blocks in several passes
    // ---- U. updates from the finished columns ----
    for (int q0 = tid; q0 < NB * 16 * nq; q0 += 8 * 256) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * 256;
        const int c = q / (16 * nq), kk = q - c * (16 * nq);
        const int row = J + c, k = kbeg + kk;
        const int rc = row < rend ? row : rend - 1;
        int kc = k > rc - b ? k : rc - b;
        kc = kc < rc ? kc : rc;
        v[u] = A[(int64_t)rc * Wb + (kc - rc + b)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * 256;
        const int c = q / (16 * nq), kk = q - c * (16 * nq);
        const int row = J + c, k = kbeg + kk;
        const bool in = c < jb && k < J && k >= row - b;
        if (q < NB * 16 * nq) Bt[c * LB + kk] = in ? -v[u] : 0.0;
      }
    }
    __syncthreads();
    // row blocks of this wavefront in pass `pass`: zigzag over groups of 4
    auto row_block = [&](int pass, int g) { return 4 * G * pass + 4 * g + ((g & 1) ? 3 - wave : wave); };
    d4 acc[G][NJ];
    for (int pass = 0; pass * 4 * G < nbr; ++pass) {
      // accumulators start from the panel's entries (zero outside the band)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int R = row_block(pass, g);
            const int row = J + 16 * R + lk + 4 * r, col = J + 16 * jc + li;
            const bool in = R < nbr && row < rend && col < J + jb && col <= row && row - col <= b;
            const int rc = row < rend ? row : rend - 1;
            int cc = col > rc - b ? col : rc - b;
            cc = cc < rc ? cc : rc;
            const double v = A[(int64_t)rc * Wb + (cc - rc + b)];
            acc[g][jc][r] = in ? v : 0.0;
          }
      // one chunk: the next chunk's L rows are requested (clamped addresses,
      // so unconditionally), this chunk's rows (copied from the previous
      // request) meet the staged tile rows, and the request is copied over
      // at the end, when the matrix-core chain has been issued
      auto load_chunk = [&](int q, double (&a)[G][4]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int R = row_block(pass, g);
          const int row = J + 16 * R + li;
          const int rc = row < rend ? row : rend - 1;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = kbeg + 16 * q + 4 * lk + s;
            int kc = k > rc - b ? k : rc - b;
            kc = kc < rc ? kc : rc;
            a[g][s] = A[(int64_t)rc * Wb + (kc - rc + b)];
          }
        }
      };
      double a[G][4], an[G][4];
      load_chunk(0, a);
      for (int q = 0; q < nq; ++q) {
        load_chunk(q + 1, an);
        double bq[NJ][4];
#pragma unroll
        for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
          for (int s = 0; s < 4; ++s) bq[jc][s] = Bt[(16 * jc + li) * LB + 16 * q + 4 * lk + s];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int R = row_block(pass, g);
          // rows of block R meet this chunk's columns inside the band?
          if (R < nbr && kbeg + 16 * q + 15 >= J + 16 * R - b) {
            const int row = J + 16 * R + li;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const int k = kbeg + 16 * q + 4 * lk + s;
              const double av = (row < rend && k < J && k >= row - b) ? a[g][s] : 0.0;
#pragma unroll
              for (int jc = 0; jc < NJ; ++jc) acc[g][jc] = mfma4(av, bq[jc][s], acc[g][jc]);
            }
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int s = 0; s < 4; ++s) a[g][s] = an[g][s];
      }
      if (multi) {
        // several passes: this pass's panel rows go back to memory and are
        // staged with the others below
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int R = row_block(pass, g);
              const int row = J + 16 * R + lk + 4 * r, col = J + 16 * jc + li;
              if (R < nbr && row < rend && col < J + jb && col <= row && row - col <= b)
                A[(int64_t)row * Wb + (col - row + b)] = acc[g][jc][r];
            }
      }
    }
    __syncthreads();
    // ---- F. the LDS panel (zero outside the band and past jb) ----
    if (!multi) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int R = row_block(0, g);
            const int i = 16 * R + lk + 4 * r, j = 16 * jc + li;
            if (R < nbr && i < nr) P[i * LS + j] = acc[g][jc][r];
          }
    } else {
      for (int q = tid; q < nr * NB; q += 256) {
        const int r = q / NB, j = q - (q / NB) * NB;
        const bool in = j < jb && j <= r && r - j <= b;
        const double x = A[in ? (int64_t)(J + r) * Wb + (j - r + b) : 0];
        P[r * LS + j] = in ? x : 0.0;
      }
    }
    __syncthreads();
    // ---- D. the diagonal tile by wavefront 0, one row per lane: at column j
    //      lane j completes its diagonal entry (its sum of squares is kept
    //      as the row is finished) and publishes the reciprocal, then every
    //      lane r > j forms L[r][j] = (x_r[j] - x_r[0:j] . L[j][0:j]) / L[j][j]
    //      with row j read from LDS (one address for all lanes) and stores it
    //      for the columns to come.  The lanes of one wavefront see each
    //      other's LDS stores in program order, so the tile needs no
    //      workgroup barrier; lanes jb..63 finish rows jb..63 of the panel on
    //      the way.  Dot products run as two interleaved partial sums. ----
    if (wave == 0) {
      const int r = lane;
      const bool have = r < nr;
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = have ? P[(have ? r : 0) * LS + j] : 0.0;
      double sa = 0.0, sb = 0.0;
      bool bad = false;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < jb) {
          if (r == j) {
            double d = x[j] - (sa + sb);
            if (!(d > 0.0)) {
              bad = true;
              d = 1.0;
            }
            x[j] = sqrt(d);
            P[j * LS + j] = x[j];
            s_rcp[j] = 1.0 / x[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          if (have && r > j) {
            double v0 = x[j], v1 = 0.0;
#pragma unroll
            for (int k = 0; k < j; ++k) {
              if (k & 1)
                v1 -= x[k] * P[j * LS + k];
              else
                v0 -= x[k] * P[j * LS + k];
            }
            x[j] = (v0 + v1) * s_rcp[j];
            P[r * LS + j] = x[j];
            if (j & 1)
              sb += x[j] * x[j];
            else
              sa += x[j] * x[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
      }
      if (bad) s_fail = 1;
    }
    __syncthreads();
    // ---- rows 64.. of the panel: solved against the finished diagonal
    //      tile, independently ----
    for (int r = 64 + tid; r < nr; r += 256) {
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = P[r * LS + j];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < jb) {
          double v0 = x[j], v1 = 0.0;
#pragma unroll
          for (int k = 0; k < j; ++k) {
            if (k & 1)
              v1 -= x[k] * P[j * LS + k];
            else
              v0 -= x[k] * P[j * LS + k];
          }
          x[j] = (v0 + v1) * s_rcp[j];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) P[r * LS + j] = x[j];
    }
    __syncthreads();
    // ---- W. write the panel back ----
    for (int q = tid; q < nr * NB; q += blockDim.x) {
      const int r = q / NB, j = q - (q / NB) * NB;
      if (j < jb && j <= r && r - j <= b) A[(int64_t)(J + r) * Wb + (j - r + b)] = P[r * LS + j];
    }
    __syncthreads();
  }
  if (tid == 0 && s_fail) atomicOr(fail, 1);
}

namespace {
int g_smem_limit = 0;

size_t chol_lds(int nb, int bmax) {
  const size_t tile = (size_t)nb * tile_stride(bmax), panel = (size_t)(nb + bmax) * (nb + 1);
  return (tile > panel ? tile : panel) * sizeof(double);
}
}  // namespace

int band_cholesky_nb(int bmax, size_t elem) {
  (void)elem;
  if (g_smem_limit == 0) {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 65536;
    g_smem_limit = v;
  }
  for (int nb : {32, 16})
    if (chol_lds(nb, bmax) <= (size_t)g_smem_limit) return nb;
  return 0;
}

template <int NB, int G>
static int launch_nb(const SubDev* subs, int64_t nsub, const int32_t* list, double* band, int32_t* fail, int bmax,
                     hipStream_t st) {
  const size_t shm = chol_lds(NB, bmax);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)band_cholesky_kernel<NB, G>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  if (nsub > 0)
    band_cholesky_kernel<NB, G><<<dim3((unsigned)nsub), dim3(256), shm, st>>>(subs, nsub, list, band, fail,
                                                                             tile_stride(bmax));
  return 0;
}

template <typename T>
int launch_band_cholesky(const SubDev* subs, int64_t nsub, const int32_t* list, T* band, int32_t* fail, int bmax,
                         int nb, hipStream_t st) {
  static_assert(sizeof(T) == 8, "FP64 factors");
  if (nb <= 0) nb = band_cholesky_nb(bmax, sizeof(T));
  switch (nb) {
    case 32:
      return launch_nb<32, 5>(subs, nsub, list, band, fail, bmax, st);
    case 16:
      return launch_nb<16, 5>(subs, nsub, list, band, fail, bmax, st);
    default:
      return -1;
  }
}
template int launch_band_cholesky<double>(const SubDev*, int64_t, const int32_t*, double*, int32_t*, int, int,
                                          hipStream_t);

}  // namespace tfeti

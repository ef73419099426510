// Subdomain solves with the regularized factors: the action of the
// generalized inverse K^+ (Remark 1: forward and backward substitution per
// subdomain) fused with the B^T scatter and the interface write of the dual
// operator F = B K^+ B^T (Section 4.2).
//
// One workgroup (256, 512 or 1024 threads) per subdomain, in a schedule order
// chosen by the host; the whole subdomain vector lives in LDS.  Each
// triangular solve walks the block rows (TS rows each): all waves
// stream the off-diagonal panel chunks (16-byte loads, one output row per
// lane, coalesced) and accumulate partial dot products; wave 0 reduces them
// and applies the inverted diagonal tile with lane broadcasts.
//
// The panels are rectangles, but a factor row is zero left of the first
// column of its envelope (Cholesky keeps the envelope of the node lattice:
// row 3q + c starts at node q minus one step along every axis on which q is
// not on the lower boundary), and the inverted diagonal tiles are
// triangular.  Lanes skip the loads of chunks that lie entirely in those zero
// parts (the backward pass with the interior envelope, a bound that is
// monotone in the row), so the bytes read approach the envelope (skyline);
// in the forward pass the 8 rows that share a 128-byte line skip together,
// up to the earliest of their envelopes, so that no line is requested by
// two load instructions (a line requested twice may be fetched twice).  In
// the backward pass a column also meets zero rows inside that bound (rows
// of nodes on a lower boundary start later): a table of the first envelope
// column of every chunk of rows sends such a lane's load to a line of zeros
// instead, so the instruction stays unconditional and fetches only the lines
// some lane needs.
// Panel loads are non-temporal (each factor entry is read once per apply)
// and issued four chunks at a time per lane (a sweep of 2..16 on MI355X put
// the optimum at 4 for both precisions).
#include "kernels.h"

namespace tfeti {

namespace {

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
  static constexpr int V = 2;
};
template <>
struct Vec<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
  static constexpr int V = 4;
};

template <typename T>
__device__ __forceinline__ T bcast(T v, int l);
template <>
__device__ __forceinline__ float bcast<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ double bcast<double>(double v, int l) {
  long long x = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffLL), l);
  int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// zeros standing in for the panel chunks a lane skips (64 lanes x 16 bytes)
__device__ __align__(256) double g_zero_chunks[128] = {};

template <typename VT, int V>
__device__ __forceinline__ auto vdot(const VT& a, const VT& b) -> decltype(a[0] * b[0]) {
  auto s = a[0] * b[0];
#pragma unroll
  for (int v = 1; v < V; ++v) s += a[v] * b[v];
  return s;
}

}  // namespace

template <typename T, int TS, int NT, int NR>
__global__ __launch_bounds__(NT) void ksolve_kernel(KsolveArgs<T> A) {
  using VT = typename Vec<T>::type;
  constexpr int V = Vec<T>::V;
  constexpr int RPT = NT / TS;           // threads per tile row
  constexpr int UNR = 4;                 // panel chunks loaded back to back per lane
  extern __shared__ __align__(16) unsigned char smem[];
  // NR right-hand sides, each a vector of vec_stride entries in LDS, one
  // partial sum per thread and right-hand side, then the first envelope
  // column of each chunk of V rows
  T* xs0 = reinterpret_cast<T*>(smem);
  T* part0 = xs0 + NR * A.vec_stride;
  int32_t* fcr = reinterpret_cast<int32_t*>(part0 + NR * NT);
  const int VS = A.vec_stride;

  if (A.done && *A.done) return;
  const int tid = threadIdx.x;
  const int32_t p = A.order[blockIdx.x];
  const SubDev s = A.subs[p];
  const int n = s.npad, nb = n / TS;

  // node counts along the two fastest axes of the factor ordering
  const int pa = s.perm[0], pb = s.perm[1];
  const int N0 = pa == 0 ? s.N[0] : (pa == 1 ? s.N[1] : s.N[2]);
  const int N1 = pb == 0 ? s.N[0] : (pb == 1 ? s.N[1] : s.N[2]);

  // first envelope column of row `row` (padding rows: the diagonal)
  auto first_col = [&](int row) {
    if (row >= s.ndof) return row;
    const int q = row / 3, i0 = q % N0, t = q / N0, i1 = t % N1, i2 = t / N1;
    return 3 * (q - (i0 > 0) - (i1 > 0) * N0 - (i2 > 0) * N0 * N1);
  };

  // ---- input: x_k = in_full (factor order) + lam_sign B^T lam_k ----
  for (int i = tid; i < n; i += NT)
#pragma unroll
    for (int k = 0; k < NR; ++k) xs0[k * VS + i] = T(0);
  for (int g = tid; g < n / V; g += NT) {
    int f = first_col(g * V);
#pragma unroll
    for (int v = 1; v < V; ++v) f = min(f, first_col(g * V + v));
    fcr[g] = f;
  }
  __syncthreads();
  if (A.in_full) {
    for (int ld = tid; ld < s.ndof; ld += NT) {
      const T f = (T)A.in_full[s.dof_off + ld];
      const int fi = factor_index(s, ld);
#pragma unroll
      for (int k = 0; k < NR; ++k) xs0[k * VS + fi] = f;
    }
    __syncthreads();
  }
  if (A.lam) {
    const double beta = A.fold.S ? A.fold.S->beta : 0.0;
    for (int t = tid; t < s.n_iface; t += NT) {
      const int64_t it = s.iface_off + t;
      double v = A.in_full ? A.in_full[s.dof_off + A.if_ldof[it]] : 0.0;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const double* lam = k == 0 ? A.lam : A.lam2;
        double bt = 0.0;
        for (int e = A.if_rp[it]; e < A.if_rp[it + 1]; ++e) {
          const int32_t row = A.if_row[e];
          const double lv = (k == 0 && A.fold.S) ? fma(beta, lam[row], A.fold.y[row]) : lam[row];
          bt += A.if_coef[e] * lv;
        }
        xs0[k * VS + A.if_fidx[it]] = (T)(v + A.lam_sign * bt);
      }
    }
  }
  __syncthreads();

  // ---- forward substitution L y = x (in place) ----
  {
    const T* P = A.Fp + s.panel_off;
    int64_t off = 0;
    const int r = tid % TS;
    for (int I = 0; I < nb; ++I) {
      const int w = I * TS < s.bo ? I * TS : s.bo;
      const int nco = w / V;
      const int c0 = I * TS - w;
      T acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = T(0);
      // first envelope column of the row (padding rows: the diagonal), and
      // the first chunk holding a column at or after it
      int fc = first_col(I * TS + r);
      // the 8 rows of a 128-byte line (lanes 8k .. 8k+7 of the tile row)
      // start at their earliest chunk together, so every line is requested
      // by one load instruction and fetched once
      fc = min(fc, __shfl_xor(fc, 1));
      fc = min(fc, __shfl_xor(fc, 2));
      fc = min(fc, __shfl_xor(fc, 4));
      const int cmin = fc > c0 ? (fc - c0) / V : 0;
      int cc = tid / TS;
      if (cc < cmin) cc += (cmin - cc + RPT - 1) / RPT * RPT;
      // UNR chunk loads in flight per lane, then their products
      for (; cc + (UNR - 1) * RPT < nco; cc += UNR * RPT) {
        VT L[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) L[u] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(P + off + ((int64_t)(cc + u * RPT) * TS + r) * V));
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(L[u], *reinterpret_cast<const VT*>(xs0 + k * VS + c0 + (cc + u * RPT) * V));
      }
      for (; cc < nco; cc += RPT) {
        VT L = *reinterpret_cast<const VT*>(P + off + ((int64_t)cc * TS + r) * V);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          VT y = *reinterpret_cast<const VT*>(xs0 + k * VS + c0 + cc * V);
          acc[k] += vdot<VT, V>(L, y);
        }
      }
#pragma unroll
      for (int k = 0; k < NR; ++k) part0[k * NT + tid] = acc[k];
      __syncthreads();
      if (tid < 64) {
        T a[NR], y[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          a[k] = T(0);
          y[k] = T(0);
          if (tid < TS) {
            T sum = T(0);
#pragma unroll
            for (int j = 0; j < RPT; ++j) sum += part0[k * NT + j * TS + tid];
            a[k] = xs0[k * VS + I * TS + tid] - sum;
          }
        }
#pragma unroll
        for (int cc = 0; cc < TS / V; ++cc) {
          VT L;
          if (tid < TS && cc * V <= tid)  // the inverse of a lower triangle is lower
            L = *reinterpret_cast<const VT*>(P + off + ((int64_t)(nco + cc) * TS + tid) * V);
          else
            L = VT(T(0));
#pragma unroll
          for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) y[k] += L[v] * bcast<T>(a[k], cc * V + v);
        }
        if (tid < TS)
#pragma unroll
          for (int k = 0; k < NR; ++k) xs0[k * VS + I * TS + tid] = y[k];
      }
      __syncthreads();
      off += (int64_t)TS * (w + TS);
    }
  }

  // ---- backward substitution L^T z = y (in place) ----
  {
    const T* P = A.Bp + s.panel_off;
    int64_t off = s.panel_len;
    const int c = tid % TS;
    for (int I = nb - 1; I >= 0; --I) {
      const int rem = n - (I + 1) * TS;
      const int w = rem < s.bo ? rem : s.bo;
      off -= (int64_t)TS * (TS + w);
      const int nco = w / V;
      const int rbase = (I + 1) * TS;
      T acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = T(0);
      // rows below the block that can reach column I TS + c: no row of node
      // q starts before node q - 1 - N0 - N0 N1, so rows past the last DOF of
      // node col/3 + 1 + N0 + N0 N1 are zero in this column, and so are the
      // padding rows; rend = the chunks before that row
      int rend;
      {
        const int col = I * TS + c;
        int last = 3 * (col / 3 + 1 + N0 + N0 * N1) + 2;
        if (last > s.ndof - 1) last = s.ndof - 1;
        int cnt = last + 1 - rbase;
        cnt = cnt < 0 ? 0 : (cnt > nco * V ? nco * V : cnt);
        rend = (cnt + V - 1) / V;
      }
      // chunk rr of this column, or zeros where its rows all start after it
      const int col = I * TS + c;
      const VT* zsrc = reinterpret_cast<const VT*>(g_zero_chunks) + (tid & 63);
      auto src = [&](int rr) -> const VT* {
        const VT* p = reinterpret_cast<const VT*>(P + off + ((int64_t)(TS / V + rr) * TS + c) * V);
        return fcr[rbase / V + rr] <= col ? p : zsrc;
      };
      int rr = tid / TS;
      for (; rr + (UNR - 1) * RPT < rend; rr += UNR * RPT) {
        VT L[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) L[u] = __builtin_nontemporal_load(src(rr + u * RPT));
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(L[u], *reinterpret_cast<const VT*>(xs0 + k * VS + rbase + (rr + u * RPT) * V));
      }
      for (; rr < rend; rr += RPT) {
        VT L = *src(rr);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          VT z = *reinterpret_cast<const VT*>(xs0 + k * VS + rbase + rr * V);
          acc[k] += vdot<VT, V>(L, z);
        }
      }
#pragma unroll
      for (int k = 0; k < NR; ++k) part0[k * NT + tid] = acc[k];
      __syncthreads();
      if (tid < 64) {
        T a[NR], z[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          a[k] = T(0);
          z[k] = T(0);
          if (tid < TS) {
            T sum = T(0);
#pragma unroll
            for (int j = 0; j < RPT; ++j) sum += part0[k * NT + j * TS + tid];
            a[k] = xs0[k * VS + I * TS + tid] - sum;
          }
        }
#pragma unroll
        for (int rc = 0; rc < TS / V; ++rc) {
          VT L;
          if (tid < TS && rc * V + V - 1 >= tid)  // the inverse transpose is upper
            L = *reinterpret_cast<const VT*>(P + off + ((int64_t)rc * TS + tid) * V);
          else
            L = VT(T(0));
#pragma unroll
          for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) z[k] += L[v] * bcast<T>(a[k], rc * V + v);
        }
        if (tid < TS)
#pragma unroll
          for (int k = 0; k < NR; ++k) xs0[k * VS + I * TS + tid] = z[k];
      }
      __syncthreads();
    }
  }

  // ---- outputs ----
  if (A.out_iface) {
    for (int t = tid; t < s.n_iface; t += NT) {
      const int64_t it = s.iface_off + t;
      A.out_iface[it] = (double)xs0[A.if_fidx[it]];
      if (NR > 1) A.out_iface2[it] = (double)xs0[VS + A.if_fidx[it]];
    }
  }
  if (A.out_full) {
    for (int ld = tid; ld < s.ndof; ld += NT) {
      double v = (double)xs0[factor_index(s, ld)];
      if (A.alpha) {
        const double* R = A.R_full + 6 * (s.dof_off + ld);
        const double* al = A.alpha + 6 * (int64_t)p;
        for (int j = 0; j < 6; ++j) v += R[j] * al[j];
      }
      A.out_full[s.dof_off + ld] = v;
    }
  }
}

template <typename T, int NT, int NR>
static void launch_ts(const KsolveArgs<T>& b, int TS, size_t shm, hipStream_t st) {
  dim3 grid((unsigned)b.nsub), block(NT);
  if (TS == 16) {
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)ksolve_kernel<T, 16, NT, NR>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    ksolve_kernel<T, 16, NT, NR><<<grid, block, shm, st>>>(b);
  } else if (TS == 32) {
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)ksolve_kernel<T, 32, NT, NR>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    ksolve_kernel<T, 32, NT, NR><<<grid, block, shm, st>>>(b);
  } else if constexpr (NT <= 512) {
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)ksolve_kernel<T, 64, NT, NR>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    ksolve_kernel<T, 64, NT, NR><<<grid, block, shm, st>>>(b);
  }
}

template <typename T>
void launch_ksolve(const KsolveArgs<T>& a, int TS, int threads, int npad_max, hipStream_t st) {
  // shared memory: NR vectors (npad_max entries each, rounded to 16 bytes)
  // + NR partial sums per thread + one envelope column per chunk of rows;
  // a second right-hand side when lam2 is set
  // 1024 threads only with tiles of 16 or 32 rows (the 64-row kernel needs
  // more registers than 16 waves per compute unit leave)
  const int NT = (threads == 1024 && TS <= 32) ? 1024 : (threads == 512 ? 512 : 256);
  const int NR = a.lam2 ? 2 : 1;
  const size_t vec = ((size_t)npad_max * sizeof(T) + 15) / 16 * 16;
  const size_t shm = NR * (vec + (size_t)NT * sizeof(T)) + (size_t)npad_max / (16 / sizeof(T)) * sizeof(int32_t);
  KsolveArgs<T> b = a;
  b.vec_stride = (int32_t)(vec / sizeof(T));
  if (NR == 2) {
    if (NT == 1024)
      launch_ts<T, 1024, 2>(b, TS, shm, st);
    else if (NT == 512)
      launch_ts<T, 512, 2>(b, TS, shm, st);
    else
      launch_ts<T, 256, 2>(b, TS, shm, st);
  } else if (NT == 1024) {
    launch_ts<T, 1024, 1>(b, TS, shm, st);
  } else if (NT == 512) {
    launch_ts<T, 512, 1>(b, TS, shm, st);
  } else {
    launch_ts<T, 256, 1>(b, TS, shm, st);
  }
}
template void launch_ksolve<double>(const KsolveArgs<double>&, int, int, int, hipStream_t);
template void launch_ksolve<float>(const KsolveArgs<float>&, int, int, int, hipStream_t);

}  // namespace tfeti

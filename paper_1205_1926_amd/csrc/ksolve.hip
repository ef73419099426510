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
// the optimum at 4 for both precisions on the cube benchmark; the FP64
// 64-row tiles of large subdomains take 8), a lane's last chunks of a block
// row in one batch as well except in the FP64 narrow-tile and two-right-hand-
// side kernels.
#include "explicit_apply.h"

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

template <typename T, int TS, int NT, int NR, bool X = false>
__global__ __launch_bounds__(NT, (X && TS <= 32) ? 4 : 1) void ksolve_kernel(KsolveArgs<T> A) {
  using VT = typename Vec<T>::type;
  constexpr int V = Vec<T>::V;
  constexpr int RPT = NT / TS;           // threads per tile row
  // panel chunks loaded back to back per lane: 4 (a sweep of 2..16 on the
  // cube benchmark), 8 for the FP64 64-row tiles, whose lanes stream about 25
  // chunks per block row and still run two wavefronts per SIMD with 8
  constexpr int UNR = (sizeof(T) == 8 && TS == 64) ? 8 : 4;
  extern __shared__ __align__(16) unsigned char smem[];
  // NR right-hand sides, each a vector of vec_stride entries in LDS, one
  // partial sum per thread and right-hand side, then the first envelope
  // column of each chunk of V rows
  T* xs0 = reinterpret_cast<T*>(smem);
  T* part0 = xs0 + NR * A.vec_stride;
  int32_t* fcr = reinterpret_cast<int32_t*>(part0 + NR * NT);
  const int VS = A.vec_stride;
  // the diagonal tile of the block row being solved, for tiles too large to
  // hold in wavefront 0's registers (after the envelope table, 16-byte aligned)
  T* dg = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(fcr) + ((size_t)VS * sizeof(T) / 4 + 15) / 16 * 16);

  if (A.done && *A.done) return;
  const int tid = threadIdx.x;
  const int32_t p = A.order[blockIdx.x];
  // (a separate instance: the plain solve keeps its registers and occupancy)
  if constexpr (X) if (A.xuse[p]) {
    // a kept elastic factor's explicit operator: all threads build x and
    // sum y; two wavefronts walk its tiles, four per batch, in the instances
    // held to four wavefronts per SIMD (tiles of 16 and 32 rows), and half
    // of the workgroup's wavefronts, eight per batch, in the 64-row instances,
    // which keep their registers (large subdomains, whose operators are the
    // launch's longest chains)
    ExplicitApply e{};
    e.subs = A.subs;
    e.F = A.xF;
    e.foff = A.xfoff;
    e.sit = A.xsit;
    e.lam = A.lam;
    e.lam_sign = A.lam_sign;
    e.out_iface = A.out_iface;
    e.if_rp = A.if_rp;
    e.if_row = A.if_row;
    e.if_coef = A.if_coef;
    e.fold = A.fold;
    constexpr int XW = TS >= 64 ? NT / 128 : 2, XU = TS >= 64 ? 8 : 4;
    explicit_apply_body<T, XW, NT, XU>(e, p, reinterpret_cast<double*>(smem));
    return;
  }
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
        const bool fold = k == 0 && A.fold.S;
        const double bt = seg_dot<4>(A.if_rp[it], A.if_rp[it + 1], A.if_row, A.if_coef, [&](int32_t row) {
          return fold ? fma(beta, lam[row], A.fold.y[row]) : lam[row];
        });
        xs0[k * VS + A.if_fidx[it]] = (T)(v + A.lam_sign * bt);
      }
    }
  }
  __syncthreads();

  // Both passes walk the block rows; per block row all lanes stream their
  // off-diagonal chunks (UNR loads in flight) into partial dots, then wave 0
  // reduces them and applies the inverted diagonal tile.  Two kinds of load
  // do not depend on the block row just solved and are requested before the
  // barriers that order the work: wave 0's diagonal-tile chunks (before the
  // first barrier, when the tile is small enough to hold in registers), and
  // every lane's first batch of chunks of the next block row (before the
  // second barrier, while wave 0 solves the diagonal block).
  constexpr bool DIAG_PRE = TS / V <= 8;
  // larger tiles: every lane fetches DGU vectors of the diagonal tile (a
  // contiguous TS x TS block of the panel) with the off-diagonal chunks and
  // stores them in LDS before the first barrier, so that wavefront 0's
  // diagonal step reads LDS instead of waiting on memory
  constexpr int DGV = TS * TS / V, DGU = DIAG_PRE ? 1 : (DGV + NT - 1) / NT;

  // ---- forward substitution L y = x (in place) ----
  {
    const T* P = A.Fp + s.panel_off;
    const int r = tid % TS;
    const VT* zsrc = reinterpret_cast<const VT*>(g_zero_chunks) + (tid & 63);
    // block row I: chunk count, first column, and this lane's first chunk
    // (the 8 rows of a 128-byte line, lanes 8k .. 8k+7 of the tile row,
    // start at their earliest envelope chunk together, so every line is
    // requested by one load instruction and fetched once)
    auto start = [&](int I, int& nco, int& c0) {
      const int w = I * TS < s.bo ? I * TS : s.bo;
      nco = w / V;
      c0 = I * TS - w;
      int fc = first_col(I * TS + r);
      fc = min(fc, __shfl_xor(fc, 1));
      fc = min(fc, __shfl_xor(fc, 2));
      fc = min(fc, __shfl_xor(fc, 4));
      const int cmin = fc > c0 ? (fc - c0) / V : 0;
      int cc = tid / TS;
      if (cc < cmin) cc += (cmin - cc + RPT - 1) / RPT * RPT;
      return cc;
    };
    auto chunk = [&](int64_t off, int cc) {
      return reinterpret_cast<const VT*>(P + off + ((int64_t)cc * TS + r) * V);
    };
    int64_t off = 0;
    int nco, c0;
    int cc0 = start(0, nco, c0);
    VT Lp[UNR];
    bool pre = cc0 + (UNR - 1) * RPT < nco;
    if (pre)
#pragma unroll
      for (int u = 0; u < UNR; ++u) Lp[u] = __builtin_nontemporal_load(chunk(off, cc0 + u * RPT));
    for (int I = 0; I < nb; ++I) {
      VT dgv[DGU];
      if constexpr (!DIAG_PRE) {
        // chunk q = dc TS + row, needed where dc V <= row (the inverse of a
        // lower triangle is lower); the others are never read
        const VT* dsrc = reinterpret_cast<const VT*>(P + off + (int64_t)nco * TS * V);
#pragma unroll
        for (int u = 0; u < DGU; ++u) {
          const int q = tid + u * NT;
          if (q < DGV && (q / TS) * V <= q % TS) dgv[u] = __builtin_nontemporal_load(dsrc + q);
        }
      }
      T acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = T(0);
      int cc = cc0;
      if (pre) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(Lp[u], *reinterpret_cast<const VT*>(xs0 + k * VS + c0 + (cc + u * RPT) * V));
        cc += UNR * RPT;
      }
      for (; cc + (UNR - 1) * RPT < nco; cc += UNR * RPT) {
        VT L[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) L[u] = __builtin_nontemporal_load(chunk(off, cc + u * RPT));
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(L[u], *reinterpret_cast<const VT*>(xs0 + k * VS + c0 + (cc + u * RPT) * V));
      }
      if constexpr (DIAG_PRE && (NR > 1 || sizeof(T) == 8)) {
        for (; cc < nco; cc += RPT) {
          VT L = *chunk(off, cc);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            VT y = *reinterpret_cast<const VT*>(xs0 + k * VS + c0 + cc * V);
            acc[k] += vdot<VT, V>(L, y);
          }
        }
      } else if (cc < nco) {
        // this lane's last chunks as one batch, the loads past the end
        // reading zeros with the vector index held at a valid entry (the
        // wide tiles and the single-right-hand-side FP32 kernels; the others
        // measured as fast or faster one chunk at a time, or ran out of
        // registers)
        VT L[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int c = cc + u * RPT;
          L[u] = __builtin_nontemporal_load(c < nco ? chunk(off, c) : zsrc);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int c = cc + u * RPT < nco ? cc + u * RPT : cc;
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(L[u], *reinterpret_cast<const VT*>(xs0 + k * VS + c0 + c * V));
        }
      }
      if constexpr (!DIAG_PRE) {
#pragma unroll
        for (int u = 0; u < DGU; ++u) {
          const int q = tid + u * NT;
          if (q < DGV && (q / TS) * V <= q % TS) *reinterpret_cast<VT*>(dg + (int64_t)q * V) = dgv[u];
        }
      }
      // the inverse of a lower triangle is lower: lane tid < TS needs the
      // diagonal chunks dc with dc V <= tid
      auto diag = [&](int dc) -> VT {
        if constexpr (DIAG_PRE)
          return (tid < TS && dc * V <= tid) ? *reinterpret_cast<const VT*>(P + off + ((int64_t)(nco + dc) * TS + tid) * V)
                                             : VT(T(0));
        else
          return (tid < TS && dc * V <= tid) ? *reinterpret_cast<const VT*>(dg + ((int64_t)dc * TS + tid) * V) : VT(T(0));
      };
      VT Ld[DIAG_PRE ? TS / V : 1];
      if (DIAG_PRE && tid < 64)
#pragma unroll
        for (int dc = 0; dc < (DIAG_PRE ? TS / V : 1); ++dc) Ld[dc] = diag(dc);
#pragma unroll
      for (int k = 0; k < NR; ++k) part0[k * NT + tid] = acc[k];
      __syncthreads();
      // the next block row's first batch
      const int64_t offn = off + (int64_t)TS * (nco * V + TS);
      int ncon = 0, c0n = 0, ccn = 0;
      bool pren = false;
      if (I + 1 < nb) {
        ccn = start(I + 1, ncon, c0n);
        pren = ccn + (UNR - 1) * RPT < ncon;
        if (pren)
#pragma unroll
          for (int u = 0; u < UNR; ++u) Lp[u] = __builtin_nontemporal_load(chunk(offn, ccn + u * RPT));
      }
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
        for (int dc = 0; dc < TS / V; ++dc) {
          VT L;
          if constexpr (DIAG_PRE)
            L = Ld[dc];
          else
            L = diag(dc);
#pragma unroll
          for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) y[k] += L[v] * bcast<T>(a[k], dc * V + v);
        }
        if (tid < TS)
#pragma unroll
          for (int k = 0; k < NR; ++k) xs0[k * VS + I * TS + tid] = y[k];
      }
      __syncthreads();
      off = offn;
      nco = ncon;
      c0 = c0n;
      cc0 = ccn;
      pre = pren;
    }
  }

  // ---- backward substitution L^T z = y (in place) ----
  {
    const T* P = A.Bp + s.panel_off;
    const int c = tid % TS;
    const VT* zsrc = reinterpret_cast<const VT*>(g_zero_chunks) + (tid & 63);
    // block row I: panel offset (blocks are stored in increasing order),
    // chunk count of the rows below, and this lane's chunk bound: no row of
    // node q starts before node q - 1 - N0 - N0 N1, so rows past the last
    // DOF of node col/3 + 1 + N0 + N0 N1 are zero in column col, and so are
    // the padding rows
    auto start = [&](int I, int64_t offI1, int64_t& offI, int& nco, int& rend) {
      const int rem = n - (I + 1) * TS;
      const int w = rem < s.bo ? rem : s.bo;
      offI = offI1 - (int64_t)TS * (TS + w);
      nco = w / V;
      const int col = I * TS + c, rbase = (I + 1) * TS;
      int last = 3 * (col / 3 + 1 + N0 + N0 * N1) + 2;
      if (last > s.ndof - 1) last = s.ndof - 1;
      int cnt = last + 1 - rbase;
      cnt = cnt < 0 ? 0 : (cnt > nco * V ? nco * V : cnt);
      rend = (cnt + V - 1) / V;
    };
    // chunk rr below block row I of this column, or zeros where its rows all
    // start after the column
    auto src = [&](int64_t offI, int I, int rr) -> const VT* {
      const VT* q = reinterpret_cast<const VT*>(P + offI + ((int64_t)(TS / V + rr) * TS + c) * V);
      return fcr[(I + 1) * TS / V + rr] <= I * TS + c ? q : zsrc;
    };
    int64_t off;
    int nco, rend;
    start(nb - 1, s.panel_len, off, nco, rend);
    const int rr0 = tid / TS;
    VT Lp[UNR];
    bool pre = rr0 + (UNR - 1) * RPT < rend;
    if (pre)
#pragma unroll
      for (int u = 0; u < UNR; ++u) Lp[u] = __builtin_nontemporal_load(src(off, nb - 1, rr0 + u * RPT));
    for (int I = nb - 1; I >= 0; --I) {
      const int rbase = (I + 1) * TS;
      VT dgv[DGU];
      if constexpr (!DIAG_PRE) {
        // chunk q = dc TS + row, needed where dc V + V - 1 >= row
        const VT* dsrc = reinterpret_cast<const VT*>(P + off);
#pragma unroll
        for (int u = 0; u < DGU; ++u) {
          const int q = tid + u * NT;
          if (q < DGV && (q / TS) * V + V - 1 >= q % TS) dgv[u] = __builtin_nontemporal_load(dsrc + q);
        }
      }
      T acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = T(0);
      int rr = rr0;
      if (pre) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(Lp[u], *reinterpret_cast<const VT*>(xs0 + k * VS + rbase + (rr + u * RPT) * V));
        rr += UNR * RPT;
      }
      for (; rr + (UNR - 1) * RPT < rend; rr += UNR * RPT) {
        VT L[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) L[u] = __builtin_nontemporal_load(src(off, I, rr + u * RPT));
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(L[u], *reinterpret_cast<const VT*>(xs0 + k * VS + rbase + (rr + u * RPT) * V));
      }
      if constexpr (DIAG_PRE && (NR > 1 || sizeof(T) == 8)) {
        for (; rr < rend; rr += RPT) {
          VT L = *src(off, I, rr);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            VT z = *reinterpret_cast<const VT*>(xs0 + k * VS + rbase + rr * V);
            acc[k] += vdot<VT, V>(L, z);
          }
        }
      } else if (rr < rend) {
        // this lane's last chunks as one batch (zeros past the end)
        VT L[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = rr + u * RPT;
          L[u] = __builtin_nontemporal_load(r < rend ? src(off, I, r) : zsrc);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = rr + u * RPT < rend ? rr + u * RPT : rr;
#pragma unroll
          for (int k = 0; k < NR; ++k)
            acc[k] += vdot<VT, V>(L[u], *reinterpret_cast<const VT*>(xs0 + k * VS + rbase + r * V));
        }
      }
      if constexpr (!DIAG_PRE) {
#pragma unroll
        for (int u = 0; u < DGU; ++u) {
          const int q = tid + u * NT;
          if (q < DGV && (q / TS) * V + V - 1 >= q % TS) *reinterpret_cast<VT*>(dg + (int64_t)q * V) = dgv[u];
        }
      }
      // the inverse transpose is upper: lane tid < TS needs the diagonal
      // chunks dc with dc V + V - 1 >= tid
      auto diag = [&](int dc) -> VT {
        if constexpr (DIAG_PRE)
          return (tid < TS && dc * V + V - 1 >= tid)
                     ? *reinterpret_cast<const VT*>(P + off + ((int64_t)dc * TS + tid) * V)
                     : VT(T(0));
        else
          return (tid < TS && dc * V + V - 1 >= tid) ? *reinterpret_cast<const VT*>(dg + ((int64_t)dc * TS + tid) * V)
                                                     : VT(T(0));
      };
      VT Ld[DIAG_PRE ? TS / V : 1];
      if (DIAG_PRE && tid < 64)
#pragma unroll
        for (int dc = 0; dc < (DIAG_PRE ? TS / V : 1); ++dc) Ld[dc] = diag(dc);
#pragma unroll
      for (int k = 0; k < NR; ++k) part0[k * NT + tid] = acc[k];
      __syncthreads();
      // the next block row's (I - 1) first batch
      int64_t offn = 0;
      int ncon = 0, rendn = 0;
      bool pren = false;
      if (I > 0) {
        start(I - 1, off, offn, ncon, rendn);
        pren = rr0 + (UNR - 1) * RPT < rendn;
        if (pren)
#pragma unroll
          for (int u = 0; u < UNR; ++u) Lp[u] = __builtin_nontemporal_load(src(offn, I - 1, rr0 + u * RPT));
      }
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
        for (int dc = 0; dc < TS / V; ++dc) {
          VT L;
          if constexpr (DIAG_PRE)
            L = Ld[dc];
          else
            L = diag(dc);
#pragma unroll
          for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) z[k] += L[v] * bcast<T>(a[k], dc * V + v);
        }
        if (tid < TS)
#pragma unroll
          for (int k = 0; k < NR; ++k) xs0[k * VS + I * TS + tid] = z[k];
      }
      __syncthreads();
      off = offn;
      nco = ncon;
      rend = rendn;
      pre = pren;
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

template <typename T, int NT, int NR, bool X = false>
static void launch_ts(const KsolveArgs<T>& b, int TS, size_t shm, hipStream_t st) {
  dim3 grid((unsigned)b.nsub), block(NT);
  // the diagonal tile's LDS copy of the tiles wider than 8 vectors of 16 bytes
  if ((size_t)TS * sizeof(T) > 128) shm += (size_t)TS * TS * sizeof(T);
  if (TS == 16) {
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)ksolve_kernel<T, 16, NT, NR, X>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    ksolve_kernel<T, 16, NT, NR, X><<<grid, block, shm, st>>>(b);
  } else if (TS == 32) {
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)ksolve_kernel<T, 32, NT, NR, X>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    ksolve_kernel<T, 32, NT, NR, X><<<grid, block, shm, st>>>(b);
  } else if constexpr (NT <= 512) {
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)ksolve_kernel<T, 64, NT, NR, X>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    ksolve_kernel<T, 64, NT, NR, X><<<grid, block, shm, st>>>(b);
  }
}

template <typename T>
void launch_ksolve(const KsolveArgs<T>& a, int TS, int threads, int npad_max, hipStream_t st) {
  // shared memory: NR vectors (npad_max entries each, rounded to 16 bytes)
  // + NR partial sums per thread + one envelope column per chunk of rows
  // (16-byte aligned) + the diagonal tile for the wide tiles; a second
  // right-hand side when lam2 is set
  // 1024 threads only with tiles of 16 or 32 rows (the 64-row kernel needs
  // more registers than 16 waves per compute unit leave)
  const int NT = (threads == 1024 && TS <= 32) ? 1024 : (threads == 512 ? 512 : 256);
  const int NR = a.lam2 ? 2 : 1;
  const size_t vec = ((size_t)npad_max * sizeof(T) + 15) / 16 * 16;
  size_t shm = NR * (vec + (size_t)NT * sizeof(T)) + (vec / 4 + 15) / 16 * 16;
  // x and one copy of y per tile-walking wavefront of the explicit
  // operators' product
  const int xw = TS >= 64 ? NT / 128 : 2;
  if (a.xuse) shm = std::max(shm, (size_t)(xw + 1) * a.x_mp * sizeof(double));
  KsolveArgs<T> b = a;
  b.vec_stride = (int32_t)(vec / sizeof(T));
  if (a.xuse) {
    // the F-apply of the PCGP loop (one right-hand side)
    if (NT == 1024)
      launch_ts<T, 1024, 1, true>(b, TS, shm, st);
    else if (NT == 512)
      launch_ts<T, 512, 1, true>(b, TS, shm, st);
    else
      launch_ts<T, 256, 1, true>(b, TS, shm, st);
  } else if (NR == 2) {
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

// Batched band Cholesky of the regularized subdomain tangents (Remark 1:
// once regularized, each block is factorized by a standard Cholesky method
// for nonsingular matrices).
//
// Storage: row-band, row r holds columns r-b..r (entry (r, k) at
// r Wb + k - r + b, k = r the diagonal) with the row stride Wb one more than
// a multiple of 16 (band_stride); rows are the subdomain DOFs in the factor
// ordering, padded with identity rows to a multiple of 64.
//
// One workgroup (256 threads) per band matrix, left-looking by block columns
// of NB.  Per block column J (the panel: the NB columns of every row the
// band reaches, at most NB + b rows):
//  U. the panel takes its updates from the finished columns in the band,
//     A_panel - L_panel,k L_tile,k^T over k in [J - b, J), on the FP64
//     matrix cores: the tile rows' L (negated) are staged in LDS, each
//     wavefront keeps the accumulators of its row blocks in registers
//     (initialized with the panel's entries) and streams the 16 x 16 tiles
//     of its rows of L that meet the band, slot by slot, a ring of DT tiles
//     in flight; the 16-column chunks start where every row's chunk is one
//     aligned 128-byte line;
//  F. the accumulators become the LDS panel;
//  D. the diagonal tile is factored by one wavefront in registers
//     (right-looking, one row per lane, cross-lane reads instead of LDS
//     round trips), which also carries panel rows NB..63 along; the same
//     wavefront forms the tile's inverse X, and the rows from 64 on are
//     L_below = A_below X^T on the matrix cores;
//  W. the panel is written back.
// Finished columns are only read, so the band is written once per entry
// and no store waits on the matrix-core chain.
#include "kernels.h"

namespace tfeti {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// a copy of v that the compiler cannot identify with v (no common
// subexpression, so values derived from v earlier need not stay live)
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// v, for the compiler computed only once dep is (orders independent work)
template <typename V>
__device__ __forceinline__ V after(V v, double dep) {
  asm volatile("" : "+v"(v) : "v"(dep));
  return v;
}

// lane l's v, for a lane index l known at compile time
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l), hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// row stride (doubles) of the staged tile rows: whole 16-column chunks
// covering b, plus 2 so that the 16 rows of a read start in distinct banks
__host__ __device__ inline int tile_stride(int bmax) { return ((bmax + 15) / 16 * 16 + 29) / 32 * 32 + 2; }

}  // namespace

template <int NB, int G, int DT>
__global__ __launch_bounds__(256, 2) void band_cholesky_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                            const int32_t* __restrict__ list,
                                                            double* __restrict__ W, int32_t* __restrict__ fail,
                                                            int LB) {
  static_assert(NB % 16 == 0 && NB <= 64, "tile of whole 16 x 16 blocks, one row per lane of a wavefront");
  static_assert(kPadRows % NB == 0, "whole block columns: the diagonal tile is always NB x NB");
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
  unsigned char* Abytes = reinterpret_cast<unsigned char*>(A);
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64, li = lane % 16,
            lk = lane / 16;
  if (tid == 0) s_fail = 0;

  for (int J = 0; J < n; J += NB) {
    const int jb = (n - J) < NB ? (n - J) : NB;
    int rend = J + jb + b;
    if (rend > n) rend = n;
    const int nr = rend - J;                      // panel rows (>= jb)
    const int nbr = (nr + 15) / 16;               // panel row blocks
    const int kbeg = J > b ? J - b : 0;           // first update column
    // 16-column chunks of the update columns start at kq0 <= kbeg, chosen
    // with kq0 + b a multiple of 16: with the band's row stride one more
    // than a multiple of 16 every row's chunk is then one aligned 128-byte
    // line (chunk entries before kbeg are masked)
    const int kq0 = kbeg - ((kbeg + b) & 15);
    const int nq = (J - kq0 + 15) / 16;           // chunks
    const bool multi = nbr > 4 * G;               // row blocks in several passes
    // entry (r, k) of the band, as a byte offset from its (uniform) start;
    // rows J - 1 .. n - 1 and columns kq0 .. J + 14 stay inside the storage
    auto eoff = [&](int r, int k) { return 8u * (uint32_t)(r * (Wb - 1) + k + b); };
    // ---- U. updates from the finished columns: the tile rows' L over the
    //      chunks, negated, to LDS (16-byte loads, all of a round in flight) ----
    constexpr int SU = 20;
    const int npair = NB * 8 * nq;
    for (int q0 = tid; q0 < npair; q0 += SU * 256) {
      double2 v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        int q = q0 + u * 256;
        q = q < npair ? q : npair - 1;
        const int c = q / (8 * nq), kk = 2 * (q - c * (8 * nq));
        v[u] = *reinterpret_cast<const double2*>(Abytes + eoff(J + c, kq0 + kk));
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int q = q0 + u * 256;
        const int c = q / (8 * nq), kk = 2 * (q - c * (8 * nq));
        const int row = J + c, k = kq0 + kk;
        if (q < npair) {
          Bt[c * LB + kk] = (c < jb && k >= kbeg && k < J && k >= row - b) ? -v[u].x : 0.0;
          Bt[c * LB + kk + 1] = (c < jb && k + 1 >= kbeg && k + 1 < J && k + 1 >= row - b) ? -v[u].y : 0.0;
        }
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
            const double v =
                *reinterpret_cast<const double*>(Abytes + 8u * (uint32_t)(rc * Wb + (cc - rc + b)));
            acc[g][jc][r] = in ? v : 0.0;
          }
      // The wavefront's tiles (16 rows x 16 update columns) that meet the
      // band, slot by slot: slot g's row block takes the chunks from the
      // first one its first row reaches (lo_of) to the last.  Each slot's
      // run is padded to whole turns of a ring of DT tiles (padding tiles
      // load the panel's first row and add zero), so that a slot always
      // starts at ring position 0 and its accumulators are updated in a
      // plain loop; loads run DT tiles ahead of the matrix cores across
      // slot boundaries.  All cursors are wavefront-uniform.
      auto lo_of = [&](int g) {
        const int R = row_block(pass, g);
        if (R >= nbr) return nq;
        const int x = J + 16 * R - b - kq0 - 15;
        const int lo = x <= 0 ? 0 : (x + 15) / 16;
        return lo < nq ? lo : nq;
      };
      auto run_of = [&](int g) { return (nq - lo_of(g) + DT - 1) / DT * DT; };
      auto next_slot = [&](int g) {  // first slot after g with a nonempty run (G: none)
        ++g;
        while (g < G && run_of(g) == 0) ++g;
        return g;
      };
      // One turn of requests: entries i0 .. i0 + DT - 1 of slot sl's run
      // into the ring (sl == G or entries past the run: the panel's first
      // row).  Lane (li, lk) fetches columns 4 lk .. 4 lk + 3 of row li as
      // two 16-byte loads; rows past the panel read its last row (their
      // products are never stored).  The loader always runs one turn ahead
      // of the matrix cores.
      const uint32_t edummy = eoff(J, kq0);
      auto load_turn = [&](int sl, int i0, double2 (&ring)[DT][2]) {
        int q0 = nq, row = J;
        if (sl < G) {
          q0 = lo_of(sl) + i0;
          row = J + 16 * row_block(pass, sl) + li;
        }
        const uint32_t e0 = eoff(row < rend ? row : rend - 1, kq0 + 4 * lk);
#pragma unroll
        for (int d = 0; d < DT; ++d) {
          const uint32_t e = q0 + d < nq ? e0 + 128u * (uint32_t)(q0 + d) : edummy;
          ring[d][0] = *reinterpret_cast<const double2*>(Abytes + e);
          ring[d][1] = *reinterpret_cast<const double2*>(Abytes + e + 16u);
        }
      };
      double2 ring[DT][2];
      load_turn(next_slot(-1), 0, ring);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int lo = lo_of(g), n = nq - lo, run = run_of(g), nx = next_slot(g);
        const int R = row_block(pass, g);
        for (int i0 = 0; i0 < run; i0 += DT) {
          const bool same = i0 + DT < run;
          const int ns = same ? g : nx, ni = same ? i0 + DT : 0;
          int nq0 = nq, nrow = J;
          if (ns < G) {
            nq0 = lo_of(ns) + ni;
            nrow = J + 16 * row_block(pass, ns) + li;
          }
          const uint32_t ne0 = eoff(nrow < rend ? nrow : rend - 1, kq0 + 4 * lk);
#pragma unroll
          for (int d = 0; d < DT; ++d) {
            const int i = i0 + d;
            const int q = lo + (i < n ? i : n - 1);
            double bq[NJ][4];
#pragma unroll
            for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
              for (int s = 0; s < 4; ++s) bq[jc][s] = Bt[(16 * jc + li) * LB + 16 * q + 4 * lk + s];
            // lane (li, lk) holds column k = kq0 + 16 q + 4 lk + s of row
            // J + 16 R + li; its band starts at k = row - b, i.e. the entry
            // counts when li - 4 lk - s <= ub.  The tile rows in LDS are zero
            // outside kbeg .. J - 1, so no other column needs a mask, and
            // rows past the panel are never stored.
            const int ub = i < n ? kq0 + 16 * q + b - J - 16 * R : -64;
            const double a[4] = {ring[d][0].x, ring[d][0].y, ring[d][1].x, ring[d][1].y};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const double av = (li - 4 * lk - s <= ub) ? a[s] : 0.0;
#pragma unroll
              for (int jc = 0; jc < NJ; ++jc) acc[g][jc] = mfma4(av, bq[jc][s], acc[g][jc]);
            }
            // the next turn's entry d into the freed ring position
            const uint32_t e = nq0 + d < nq ? ne0 + 128u * (uint32_t)(nq0 + d) : edummy;
            ring[d][0] = *reinterpret_cast<const double2*>(Abytes + e);
            ring[d][1] = *reinterpret_cast<const double2*>(Abytes + e + 16u);
          }
        }
      }
      if (multi) {
        // several passes: this pass's panel rows go back to memory and are
        // staged with the others below (lane indices re-derived, so that
        // nothing of the accumulators' set-up stays live across the loop)
        const int li2 = opaque(li), lk2 = opaque(lk);
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int R = row_block(pass, g);
              const int row = J + 16 * R + lk2 + 4 * r, col = J + 16 * jc + li2;
              if (R < nbr && row < rend && col < J + jb && col <= row && row - col <= b)
                A[(int64_t)row * Wb + (col - row + b)] = acc[g][jc][r];
            }
      }
    }
    __syncthreads();
    // ---- F. the LDS panel (zero outside the band and past jb) ----
    if (!multi) {
      const int li2 = opaque(li), lk2 = opaque(lk);
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int R = row_block(0, g);
            const int i = 16 * R + lk2 + 4 * r, j = 16 * jc + li2;
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
    // ---- D. the diagonal tile by wavefront 0, right-looking, one row per
    //      lane (lanes NB..63 carry panel rows NB..63 along): at column j the
    //      pivot is lane j's entry, 1/sqrt of it comes from the reciprocal
    //      square root refined by two Newton steps, and every later column k
    //      takes lane k's L[k][j] by a cross-lane read, so the chain has no
    //      LDS round trip.  Then lane c < NB forms column c of X = L^{-1}
    //      (forward substitution over the tile in LDS) and stores its strict
    //      lower part transposed in the tile's upper triangle; s_rcp holds
    //      X's diagonal. ----
    if (wave == 0) {
      // lane index re-derived here: nothing lane-dependent of this phase is
      // computed ahead of the block-column loop and kept live across it
      const int r = opaque(lane);
      const bool have = r < nr;
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = have ? P[(have ? r : 0) * LS + j] : 0.0;
      bool bad = false;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        double d = readlane_f64(x[j], j);
        if (!(d > 0.0)) {
          bad = true;
          d = 1.0;
        }
        double y = __builtin_amdgcn_rsq(d);
        y = y * fma(-0.5 * d * y, y, 1.5);
        y = y * fma(-0.5 * d * y, y, 1.5);
        x[j] = r == j ? d * y : x[j] * y;
        if (r == 0) s_rcp[j] = y;
        // the cross-lane reads go in groups of four, each group ordered
        // after the previous one's updates, so that few scalar registers
        // hold read values at a time
        double xj = x[j];
#pragma unroll
        for (int k0 = j + 1; k0 < NB; k0 += 4) {
#pragma unroll
          for (int k = k0; k < k0 + 4 && k < NB; ++k) x[k] = fma(-xj, readlane_f64(xj, k), x[k]);
          xj = after(xj, x[k0 + 3 < NB ? k0 + 3 : NB - 1]);
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (have && j <= r) P[r * LS + j] = x[j];
      if (bad) s_fail = 1;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if constexpr (NB == 32) {
        // X in 16 x 16 blocks: lanes 0..15 form the columns of X11 = L11^{-1}
        // and lanes 16..31 those of X22 = L22^{-1} (two 16-row chains at
        // once), then X21 = -X22 (L21 X11) on the matrix cores
        if (r < NB) {
          const int o = r & 16, c = r - o;
          double z[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            // row i of the block is read once z[i - 1] is known
            const int base = i >= 1 ? after((o + i) * LS + o, z[i - 1]) : o * LS + o;
            double s0 = i == c ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) {
              if (k & 1)
                s1 = fma(-P[base + k], z[k], s1);
              else
                s0 = fma(-P[base + k], z[k], s0);
            }
            z[i] = (s0 + s1) * s_rcp[o + i];
          }
#pragma unroll
          for (int i = 1; i < 16; ++i)
            if (i > c) P[(o + c) * LS + o + i] = z[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int mi = opaque(li), mk = opaque(lk);
        // T = L21 X11 (X11[k][n] is P[n][k] below its diagonal, s_rcp on it)
        d4 t = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = 4 * st + mk;
          const double bb = kk > mi ? P[mi * LS + kk] : (kk == mi ? s_rcp[mi] : 0.0);
          t = mfma4(P[(16 + mi) * LS + kk], bb, t);
        }
        // parked in the tile's upper right block, P[m][16 + n] = T[m][n]
#pragma unroll
        for (int q = 0; q < 4; ++q) P[(mk + 4 * q) * LS + 16 + mi] = t[q];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        d4 x = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = 4 * st + mk;
          const double aa = mi > kk ? P[(16 + kk) * LS + 16 + mi] : (mi == kk ? s_rcp[16 + mi] : 0.0);
          x = mfma4(aa, P[kk * LS + 16 + mi], x);
        }
        // X21[m][n] = -x, stored transposed: P[n][16 + m] (over T, whose
        // reads are done)
#pragma unroll
        for (int q = 0; q < 4; ++q) P[mi * LS + 16 + mk + 4 * q] = -x[q];
      } else {
        if (r < NB) {
          const int c = r;
          double z[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            // row i of the tile is read once z[i - 1] is known: one row in
            // flight, not the whole tile at once
            const int base = i >= 1 ? after(i * LS, z[i - 1]) : 0;
            double s0 = i == c ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) {
              if (k & 1)
                s1 = fma(-P[base + k], z[k], s1);
              else
                s0 = fma(-P[base + k], z[k], s0);
            }
            z[i] = (s0 + s1) * s_rcp[i];
          }
#pragma unroll
          for (int i = 1; i < NB; ++i)
            if (i > c) P[c * LS + i] = z[i];
        }
      }
    }
    __syncthreads();
    // ---- rows 64.. of the panel: L_below = A_below X^T on the matrix cores
    //      (B[k][n] = X[n][k], zero for k > n), one 16-row block at a time ----
    {
      const int nb2 = nr > 64 ? (nr - 64 + 15) / 16 : 0;
      if (nb2 > wave) {
        const int mi = opaque(li), mk = opaque(lk);
        double xb[NJ][KS];
#pragma unroll
        for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const int n = 16 * jc + mi, k = 4 * t + mk;
            xb[jc][t] = k < n ? P[k * LS + n] : (k == n ? s_rcp[n] : 0.0);
          }
        for (int rb = wave; rb < nb2; rb += 4) {
          const int row0 = 64 + 16 * rb;
          const int ra = row0 + mi < nr ? row0 + mi : nr - 1;
          d4 y[NJ];
#pragma unroll
          for (int jc = 0; jc < NJ; ++jc) y[jc] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const double av = P[ra * LS + 4 * t + mk];
#pragma unroll
            for (int jc = 0; jc < NJ; ++jc)
              if (4 * t <= 16 * jc + 15) y[jc] = mfma4(av, xb[jc][t], y[jc]);
          }
#pragma unroll
          for (int jc = 0; jc < NJ; ++jc)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = row0 + mk + 4 * q;
              if (row < nr) P[row * LS + 16 * jc + mi] = y[jc][q];
            }
        }
      }
    }
    __syncthreads();
    // ---- W. write the panel back ----
    {
      // eight LDS reads in flight per thread before the stores
      constexpr int WU = 8;
      const int nw = nr * NB;
      for (int q0 = tid; q0 < nw; q0 += WU * 256) {
        double v[WU];
#pragma unroll
        for (int u = 0; u < WU; ++u) {
          const int q = q0 + u * 256 < nw ? q0 + u * 256 : nw - 1;
          v[u] = P[(q / NB) * LS + q % NB];
        }
#pragma unroll
        for (int u = 0; u < WU; ++u) {
          const int q = q0 + u * 256, r = q / NB, j = q % NB;
          if (q < nw && j < jb && j <= r && r - j <= b)
            *reinterpret_cast<double*>(Abytes + eoff(J + r, J + j)) = v[u];
        }
      }
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

template <int NB, int G, int DT>
static int launch_nb(const SubDev* subs, int64_t nsub, const int32_t* list, double* band, int32_t* fail, int bmax,
                     hipStream_t st) {
  const size_t shm = chol_lds(NB, bmax);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)band_cholesky_kernel<NB, G, DT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  if (nsub > 0)
    band_cholesky_kernel<NB, G, DT><<<dim3((unsigned)nsub), dim3(256), shm, st>>>(subs, nsub, list, band, fail,
                                                                             tile_stride(bmax));
  return 0;
}

#ifndef CHOL_DT
#define CHOL_DT 2
#endif
template <typename T>
int launch_band_cholesky(const SubDev* subs, int64_t nsub, const int32_t* list, T* band, int32_t* fail, int bmax,
                         int nb, hipStream_t st) {
  static_assert(sizeof(T) == 8, "FP64 factors");
  if (nb <= 0) nb = band_cholesky_nb(bmax, sizeof(T));
  switch (nb) {
    case 32:
      return launch_nb<32, 5, CHOL_DT>(subs, nsub, list, band, fail, bmax, st);
    case 16:
      return launch_nb<16, 5, CHOL_DT>(subs, nsub, list, band, fail, bmax, st);
    default:
      return -1;
  }
}
template int launch_band_cholesky<double>(const SubDev*, int64_t, const int32_t*, double*, int32_t*, int, int,
                                          hipStream_t);

}  // namespace tfeti

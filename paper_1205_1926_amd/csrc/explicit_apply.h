// The explicit local dual operator's product (see explicit.hip) as a device
// function, shared by its own kernel and by the subdomain-solve kernel,
// which applies it to the subdomains whose kept elastic factor has one.
#pragma once

#include "kernels.h"

namespace tfeti {

// tile (I, J), I >= J, of the lower triangle of an mt x mt tile grid, tiles
// of one tile column contiguous
__host__ __device__ inline int64_t explicit_tile_index(int64_t I, int64_t J, int64_t mt) {
  return J * mt - J * (J - 1) / 2 + (I - J);
}

// y = Ft_p x for subdomain p (x = lam_sign B^T lam at its touched DOFs), the
// result at the touched DOFs; the workgroup's NT threads build x and sum
// the result, its first NW wavefronts walk the tiles (lane l holds row
// l / 4 and columns 4 (l % 4) .. + 3 of a tile; U tiles of a column are
// fetched together).  sh: LDS for x and NW copies of y, 16 (NW + 1)
// ceil(m_p / 16) doubles.
template <typename T, int NW, int NT, int U>
__device__ __forceinline__ void explicit_apply_body(const ExplicitApply& a, int p, double* sh) {
  static_assert(NT >= 64 * NW, "the tile-walking wavefronts are the first NW of the workgroup");
  constexpr int CH = (int)sizeof(T) * 256 / 16 / 64;  // 16-byte chunks per lane per tile
  typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type VT;
  const int m = a.subs[p].n_iface;
  const int mt = (m + 15) / 16, mp = 16 * mt;
  const int64_t ioff = a.subs[p].iface_off;
  const T* F = reinterpret_cast<const T*>(a.F) + a.foff[p];
  double* x = sh;
  double* y = sh + mp;  // NW copies
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, rr = lane / 4, cq = lane % 4;

  const double beta = a.fold.S ? a.fold.S->beta : 0.0;
  for (int i = tid; i < mp; i += NT) {
    double v = 0.0;
    if (i < m) {
      const int64_t it = a.sit[ioff + i];
      v = a.lam_sign * seg_dot<4>(a.if_rp[it], a.if_rp[it + 1], a.if_row, a.if_coef, [&](int32_t row) {
            return a.fold.S ? fma(beta, a.lam[row], a.fold.y[row]) : a.lam[row];
          });
    }
    x[i] = v;
#pragma unroll
    for (int w = 0; w < NW; ++w) y[w * mp + i] = 0.0;
  }
  __syncthreads();

  if (wave < NW) {
    double* yw = y + wave * mp;
    for (int J = wave; J < mt; J += NW) {
      double xj[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) xj[c] = x[16 * J + 4 * cq + c];
      double cp[4] = {0.0, 0.0, 0.0, 0.0};
      const T* col = F + explicit_tile_index(J, J, mt) * 256 + rr * 16 + 4 * cq;
      // tiles I = J .. mt - 1 of column J, U at a time (the diagonal tile
      // contributes its rows only: it is stored whole)
      for (int I0 = J; I0 < mt; I0 += U) {
        VT v[U][CH];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int I = I0 + u < mt ? I0 + u : mt - 1;
#pragma unroll
          for (int h = 0; h < CH; ++h) v[u][h] = reinterpret_cast<const VT*>(col + (int64_t)(I - J) * 256)[h];
        }
        // the batch's LDS traffic in three independent groups (x reads, y
        // reads, y writes; distinct rows), not one read-modify-write chain
        // per tile: rows past the last tile use the last row and add zero
        double xi[U], rp[U], yo[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xi[u] = x[16 * (I0 + u < mt ? I0 + u : mt - 1) + rr];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int I = I0 + u;
          double e[4];
#pragma unroll
          for (int h = 0; h < CH; ++h) {
            if constexpr (sizeof(T) == 8) {
              e[2 * h] = v[u][h].x;
              e[2 * h + 1] = v[u][h].y;
            } else {
              e[0] = v[u][h].x;
              e[1] = v[u][h].y;
              e[2] = v[u][h].z;
              e[3] = v[u][h].w;
            }
          }
          double r = e[0] * xj[0];
#pragma unroll
          for (int c = 1; c < 4; ++c) r = fma(e[c], xj[c], r);
          r += __shfl_xor(r, 1);
          r += __shfl_xor(r, 2);
          rp[u] = I < mt ? r : 0.0;
          // columns: the diagonal tile (I == J) contributes its rows only
          const double xu = (I > J && I < mt) ? xi[u] : 0.0;
#pragma unroll
          for (int c = 0; c < 4; ++c) cp[c] = fma(e[c], xu, cp[c]);
        }
        if (cq == 0) {
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (I0 + u < mt) yo[u] = yw[16 * (I0 + u) + rr];
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (I0 + u < mt) yw[16 * (I0 + u) + rr] = yo[u] + rp[u];
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double v = cp[c];
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        cp[c] = v;
      }
      if (rr == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) yw[16 * J + 4 * cq + c] += cp[c];
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < m; i += NT) {
    double v = y[i];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += y[w * mp + i];
    a.out_iface[a.sit[ioff + i]] = v;
  }
}

}  // namespace tfeti

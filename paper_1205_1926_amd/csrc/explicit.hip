// Explicit local dual operators (cheaper F-apply format).
//
// F = B K^+ B^T (Section 4.2) sums, over the subdomains, B_p K_p^+ B_p^T,
// and B_p only touches the DOFs of subdomain p that carry rows of B.  With
// K_p^+ the inverse of the regularized block (Remark 1: fixing nodes, then
// a Cholesky factor L L^T), the touched block of that inverse,
//
//   Ft_p = S_p^T K_reg,p^{-1} S_p     (S_p: the columns of I at the touched DOFs),
//
// is a dense symmetric m_p x m_p matrix, and one F-apply needs only
// Ft_p (B_p^T lambda)_touched per subdomain.  Stored as its lower triangle
// in 16 x 16 tiles it holds about 5.4 MB in FP64 for an interior 8^3
// subdomain (1158 touched DOFs), against the 8.6 MB of factor panels that
// the two triangular sweeps of a subdomain solve read.
//
// Touched DOFs are taken in ascending factor index ("sorted position"), so
// that column c of S_p has no entry before row f_c of the factor ordering:
// L^{-1} S_p is zero above f_c and its solves can start there.
//
// Forming (once per factorization of the subdomain, on the FP64 matrix
// cores, v_mfma_f64_16x16x4f64): each wavefront takes 16 consecutive sorted
// columns C and computes W = L^{-T} L^{-1} S_C by block forward and backward
// substitution over 16-row blocks of the band factor:
//   forward  Z_I = D_I (S_I - sum_K L_IK Z_K),        K in [I - kb, I)
//   backward W_I = D_I^T (Z_I - sum_K L_KI^T W_K),     K in (I, I + kb]
// with D_I the inverse of the diagonal 16 x 16 block (diag_inverse_kernel)
// and kb = ceil(b / 16).  The factor tiles of a block row are staged in LDS
// once for the workgroup's wavefronts, the last kb blocks of each
// wavefront's Z (then W) stay in its registers, and Z goes to a scratch
// buffer for the backward sweep.  The rows of W at touched DOFs of sorted
// position >= the first of C are the lower-triangle entries of columns C of
// Ft_p.
//
// Applying (once per F-apply, HBM bound): one workgroup per subdomain;
// each wavefront walks whole tile columns J and uses every off-diagonal
// tile (I, J) twice, y_I += T x_J and y_J += T^T x_I, so the lower triangle
// is read once.  Each wavefront accumulates into its own copy of y in LDS
// and the copies are summed in a fixed order: the result does not depend on
// scheduling.
#include "explicit_apply.h"

namespace tfeti {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// v, for the compiler computed only once dep is (keeps loads from being
// hoisted far ahead of their use)
__device__ __forceinline__ int after(int v, double dep) {
  asm volatile("" : "+v"(v) : "v"(dep));
  return v;
}


// Inverse X of each 16 x 16 diagonal block of the factor, in two orders
// that put a lane's four matrix-core operands next to each other:
//   block + 0:   X[i][g + 4 s]  at i * 16 + 4 g + s   (forward: X Z)
//   block + 256: X[g + 4 s][i]  at i * 16 + 4 g + s   (backward: X^T W)
// Rows past the last DOF are identity rows.  16 lanes per block, lane j
// computes column j by forward substitution.
__global__ __launch_bounds__(256) void diag_inverse_kernel(const SubDev* __restrict__ subs, int64_t count,
                                                           const int32_t* __restrict__ list,
                                                           const double* __restrict__ band,
                                                           const int64_t* __restrict__ doff,
                                                           double* __restrict__ dinv) {
  if ((int64_t)blockIdx.x >= count) return;
  const int64_t p = list ? list[blockIdx.x] : blockIdx.x;
  const int ndof = subs[p].ndof, b = subs[p].b, Wm = subs[p].Wb - 1;
  const double* A = band + subs[p].band_off;
  double* D = dinv + doff[p];
  const int nbr = (ndof + 15) / 16, j = threadIdx.x % 16;
  for (int I = threadIdx.x / 16; I < nbr; I += 16) {
    const int R0 = 16 * I;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int R = R0 + i;
      double acc = i == j ? 1.0 : 0.0;
      if (R < ndof) {
#pragma unroll
        for (int k = 0; k < i; ++k)
          if (R0 + k >= R - b) acc -= A[(int64_t)R * Wm + R0 + k + b] * x[k];
        acc /= A[(int64_t)R * Wm + R + b];
      }
      x[i] = acc;
    }
    double* X = D + (int64_t)I * 512;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      X[i * 16 + 4 * (j % 4) + j / 4] = x[i];
      X[256 + j * 16 + 4 * (i % 4) + i / 4] = x[i];
    }
  }
}

// One workgroup per (subdomain p, group of NW consecutive column blocks of
// 16 sorted touched DOFs), one wavefront per column block; the wavefronts
// walk the block rows together.  Per block row the KB factor tiles the
// update needs (forward: row block I, columns of blocks I - KB .. I - 1;
// backward: column block I, rows of blocks I + 1 .. I + KB) are read from
// the band once per workgroup, masked to the band, and staged in LDS (two
// buffers: the tiles of the next row are fetched into registers while the
// current row is computed).  Each wavefront keeps the last KB blocks of its
// Z (then W) in registers, block K in slot K mod KB (a compile-time index:
// the row loop is unrolled KB rows at a time), so that block K is the B
// operand of the product with tile K without any move:
// in step s of a 16 x 16 x 4 product lane l (row or column l % 16, group
// g = l / 16) supplies contraction index g + 4 s, which is register s of an
// accumulator (rows g + 4 r).  LDS holds tile k as [s][g][i] = T[i][g + 4 s],
// so that the 64 lanes' operands of one step are 64 consecutive doubles
// (no bank conflicts).  Rows a wavefront does not need
// (before its first touched DOF) are skipped by that wavefront only.
template <typename T, int KB, int NW>
__global__ __launch_bounds__(64 * NW) void explicit_form_kernel(ExplicitForm a, int64_t item0, int64_t n) {
  constexpr int NT = 64 * NW;
  constexpr int SE = (KB * 256 + NT - 1) / NT;   // staged entries per thread and row
  __shared__ __align__(16) double stage[2][KB * 256];
  extern __shared__ int posl[];                   // sorted position of each factor row (-1: untouched)
  // consecutive groups (of one subdomain) on one XCD: workgroups are dealt
  // to the eight XCDs in turn
  const int64_t per = (n + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= n) return;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, g = lane / 16;
  const int p = uniform(a.items[2 * (item0 + t)]), grp = uniform(a.items[2 * (item0 + t) + 1]);
  const int ndof = uniform(a.subs[p].ndof), b = uniform(a.subs[p].b), Wm = uniform(a.subs[p].Wb - 1);
  const int m = uniform(a.subs[p].n_iface);
  const int64_t ioff = a.subs[p].iface_off, doff_t = a.subs[p].dof_off;
  const double* A = a.band + a.subs[p].band_off;
  const double* D = a.dinv + a.doff[p];
  const int nbr = (ndof + 15) / 16, kb = (b + 15) / 16;
  const int mt = (m + 15) / 16;
  const int cb = NW * grp + wave;                // this wavefront's column block
  const bool has = cb < mt;
  const int c = 16 * cb + li;
  const int fj = c < m ? a.sfidx[ioff + c] : -1;
  const int Iw = has ? uniform(a.sfidx[ioff + 16 * cb]) / 16 : nbr;  // first row block of this wavefront
  const int Ig = uniform(a.sfidx[ioff + 16 * NW * grp]) / 16;         // of the group (sorted: the first)
  double* Zs = a.dinv + a.zs_off + (t * NW + wave) * a.zstride;
  T* F = reinterpret_cast<T*>(a.F) + a.foff[p];

  for (int r = tid; r < ndof; r += NT) posl[r] = a.pos[doff_t + r];
  double zr[KB][4];
#pragma unroll
  for (int k = 0; k < KB; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s) zr[k][s] = 0.0;
  // staging: entry e = tid + NT q of a row's KB tiles is entry (i, c) =
  // (e % 16, (e / 16) % 4 + 4 ((e / 64) % 4)) of tile e / 256 (forward: row
  // i, column c; backward: row c, column i), stored at LDS position e, so
  // that in step s lane l reads position 64 s + l: 64 consecutive doubles
  double sv[SE];
  double dv[4];

  // ---- forward
  {
    // tile k of row I: rows 16 I + i, columns 16 (I - KB + k) + c
    auto fetch = [&](int I) {
#pragma unroll
      for (int q = 0; q < SE; ++q) {
        const int e = tid + NT * q, k = e >> 8, i = e & 15, c = ((e >> 4) & 3) + 4 * ((e >> 6) & 3);
        const int R = 16 * I + i, col = 16 * (I - KB + k) + c;
        const int Rc = R < ndof ? R : ndof - 1, cc = col > Rc - b ? col : Rc - b;
        const double v = A[Rc * Wm + cc + b];
        sv[q] = (e < KB * 256 && R < ndof && col >= R - b && col >= 0) ? v : 0.0;
      }
    };
    auto put = [&](int buf) {
#pragma unroll
      for (int q = 0; q < SE; ++q) {
        const int e = tid + NT * q;
        if (e < KB * 256) stage[buf][e] = sv[q];
      }
    };
    auto fetch_d = [&](int I) {
#pragma unroll
      for (int s = 0; s < 4; ++s) dv[s] = D[(int64_t)(I < nbr ? I : 0) * 512 + li * 16 + 4 * g + s];
    };
    fetch(Ig);
    fetch_d(Ig);
    // rows in rounds of KB: block K lives in ring slot K mod KB, a
    // compile-time index within the round
    for (int I0r = Ig / KB * KB; I0r < nbr; I0r += KB) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int I = I0r + u;
        if (I >= Ig && I < nbr) {
          const int buf = I & 1;
          put(buf);
          if (I + 1 < nbr) fetch(I + 1);
          __syncthreads();
          if (I >= Iw) {
            d4 acc = {0, 0, 0, 0};
            const int tb = buf * KB * 256 + lane;
            // tiles k >= k0 take part; each tile's operands are read while
            // the products of the tile before it run
            const int k0 = KB - min(kb, I - Iw);
            double ac[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) ac[s] = stage[0][tb + min(k0, KB - 1) * 256 + 64 * s];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              if (k >= k0) {
                double an[4];
                const int nx = after(tb + min(k + 1, KB - 1) * 256, acc[0]);
#pragma unroll
                for (int s = 0; s < 4; ++s) an[s] = stage[0][nx + 64 * s];
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = mfma4(-ac[s], zr[(u + k) % KB][s], acc);
#pragma unroll
                for (int s = 0; s < 4; ++s) ac[s] = an[s];
              }
            }
            d4 tv = acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) tv[r] += (16 * I + g + 4 * r == fj) ? 1.0 : 0.0;
            d4 z = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 4; ++s) z = mfma4(dv[s], tv[s], z);
            fetch_d(I + 1);
            double* Zg = Zs + (int64_t)(I - Iw) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r) Zg[r * 64 + lane] = z[r];
#pragma unroll
            for (int s = 0; s < 4; ++s) zr[u][s] = z[s];
          } else if (I + 1 == Iw) {
            fetch_d(I + 1);
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- backward (the ring holds W_{I+1} .. W_{I+KB})
  {
#pragma unroll
    for (int k = 0; k < KB; ++k)
#pragma unroll
      for (int s = 0; s < 4; ++s) zr[k][s] = 0.0;
    double zv[4];
    // tile k of row I: rows 16 (I + 1 + k) + c, columns 16 I + i
    auto fetch = [&](int I) {
#pragma unroll
      for (int q = 0; q < SE; ++q) {
        const int e = tid + NT * q, k = e >> 8, i = e & 15, c = ((e >> 4) & 3) + 4 * ((e >> 6) & 3);
        const int R = 16 * (I + 1 + k) + c, col = 16 * I + i;
        const int Rc = R < ndof ? R : ndof - 1, cc = col > Rc - b ? col : Rc - b;
        const double v = A[Rc * Wm + cc + b];
        sv[q] = (e < KB * 256 && R < ndof && col >= R - b) ? v : 0.0;
      }
    };
    auto put = [&](int buf) {
#pragma unroll
      for (int q = 0; q < SE; ++q) {
        const int e = tid + NT * q;
        if (e < KB * 256) stage[buf][e] = sv[q];
      }
    };
    // the diagonal inverse and Z_I
    auto fetch_d = [&](int I) {
      const int Ic = I >= 0 ? I : 0, Iz = I >= Iw ? I : Iw;
#pragma unroll
      for (int s = 0; s < 4; ++s) dv[s] = D[(int64_t)Ic * 512 + 256 + li * 16 + 4 * g + s];
#pragma unroll
      for (int s = 0; s < 4; ++s) zv[s] = has ? Zs[(int64_t)(Iz - Iw) * 256 + s * 64 + lane] : 0.0;
    };
    fetch(nbr - 1);
    fetch_d(nbr - 1);
    // rows in rounds of KB from the top: block K in slot K mod KB
    for (int Itr = (nbr - 1) / KB * KB + KB - 1; Itr >= Ig; Itr -= KB) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int I = Itr - u;
        if (I >= Ig && I < nbr) {
          const int buf = I & 1;
          put(buf);
          if (I - 1 >= Ig) fetch(I - 1);
          __syncthreads();
          if (I >= Iw) {
            d4 acc = {zv[0], zv[1], zv[2], zv[3]};
            const int tb = buf * KB * 256 + lane;
            // tiles k < k1 take part
            const int k1 = min(kb, nbr - 1 - I);
            double ac[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) ac[s] = stage[0][tb + 64 * s];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              if (k < k1) {
                double an[4];
                const int nx = after(tb + min(k + 1, KB - 1) * 256, acc[0]);
#pragma unroll
                for (int s = 0; s < 4; ++s) an[s] = stage[0][nx + 64 * s];
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = mfma4(-ac[s], zr[(KB + k - u) % KB][s], acc);
#pragma unroll
                for (int s = 0; s < 4; ++s) ac[s] = an[s];
              }
            }
            const d4 tv = acc;
            d4 w = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 4; ++s) w = mfma4(dv[s], tv[s], w);
            fetch_d(I - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int R = 16 * I + g + 4 * r, q = R < ndof ? posl[R] : -1;
              if (q >= 0 && (q >> 4) >= cb)
                F[explicit_tile_index(q >> 4, cb, mt) * 256 + (q & 15) * 16 + li] = (T)w[r];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) zr[(KB - 1 - u) % KB][s] = w[s];
          }
        }
      }
    }
  }
}

// y = Ft_p x per subdomain: one workgroup of NW wavefronts per subdomain.
template <typename T, int NW, int U>
__global__ __launch_bounds__(64 * NW) void explicit_apply_kernel(ExplicitApply a) {
  if (a.done && *a.done) return;
  extern __shared__ double sh[];
  const int p = a.order ? a.order[blockIdx.x] : blockIdx.x;
  explicit_apply_body<T, NW, 64 * NW, U>(a, p, sh);
}

// the operator of each listed subdomain copied as 16-byte vectors (its
// storage is a multiple of 256 entries)
__global__ __launch_bounds__(256) void copy_explicit_kernel(const SubDev* __restrict__ subs, const int32_t* list,
                                                            const int64_t* __restrict__ foff, const int4* src,
                                                            int4* dst, int32_t per_tile) {
  const int p = list[blockIdx.x];
  const int64_t mt = (subs[p].n_iface + 15) / 16;
  const int64_t n = mt * (mt + 1) / 2 * per_tile, o = foff[p] / 256 * per_tile;
  for (int64_t i = threadIdx.x; i < n; i += 256) dst[o + i] = src[o + i];
}

}  // namespace

void launch_copy_explicit(const SubDev* subs, int64_t count, const int32_t* list, const int64_t* foff,
                          const void* src, void* dst, size_t elem, hipStream_t st) {
  if (count > 0)
    copy_explicit_kernel<<<dim3((unsigned)count), dim3(256), 0, st>>>(
        subs, list, foff, reinterpret_cast<const int4*>(src), reinterpret_cast<int4*>(dst),
        (int32_t)(256 * elem / 16));
}

int64_t explicit_tiles(int64_t m) {
  const int64_t mt = (m + 15) / 16;
  return mt * (mt + 1) / 2;
}

void launch_diag_inverse(const SubDev* subs, int64_t count, const int32_t* list, const double* band,
                         const int64_t* doff, double* dinv, hipStream_t st) {
  if (count > 0)
    diag_inverse_kernel<<<dim3((unsigned)count), dim3(256), 0, st>>>(subs, count, list, band, doff, dinv);
}

// tiles per staged row: the smallest instantiated count >= ceil(bmax / 16)
int explicit_form_kb(int bmax) {
  const int kb = (bmax + 15) / 16;
  for (int k : {4, 8, 12, 18, 21, 26})
    if (kb <= k) return k;
  return 0;
}

template <typename T>
void launch_explicit_form(const ExplicitForm& a, int64_t item0, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t per = (n + 7) / 8;
  const dim3 grid((unsigned)(8 * per)), block(64 * kExplicitWaves);
  const size_t lds = (size_t)a.max_ndof * sizeof(int);
  switch (a.kb) {
    case 4: explicit_form_kernel<T, 4, kExplicitWaves><<<grid, block, lds, st>>>(a, item0, n); break;
    case 8: explicit_form_kernel<T, 8, kExplicitWaves><<<grid, block, lds, st>>>(a, item0, n); break;
    case 12: explicit_form_kernel<T, 12, kExplicitWaves><<<grid, block, lds, st>>>(a, item0, n); break;
    case 18: explicit_form_kernel<T, 18, kExplicitWaves><<<grid, block, lds, st>>>(a, item0, n); break;
    case 21: explicit_form_kernel<T, 21, kExplicitWaves><<<grid, block, lds, st>>>(a, item0, n); break;
    default: explicit_form_kernel<T, 26, kExplicitWaves><<<grid, block, lds, st>>>(a, item0, n); break;
  }
}

template <typename T>
void launch_explicit_apply(const ExplicitApply& a, int max_iface, hipStream_t st) {
  // four wavefronts per subdomain when every subdomain's workgroup is then
  // still resident at once (two per compute unit, by registers, if the LDS
  // of x and four copies of y allows), else two: the launch ends with the
  // largest operators, which stream faster with more loads in flight (with
  // at most two workgroups per compute unit, registers allow batches of 16
  // tiles; with two wavefronts and many workgroups per unit, 8)
  static int cus = 0, lds_cu = 0;
  if (cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 1;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0)
      lds_cu = 65536;
  }
  const int mp = (max_iface + 15) / 16 * 16;
  const size_t lds4 = (size_t)5 * mp * sizeof(double);
  const int64_t per_cu = std::min<int64_t>(2, (int64_t)lds_cu / (int64_t)lds4);
  if (a.nsub <= per_cu * cus) {
    if (lds4 > 65536)
      (void)hipFuncSetAttribute((const void*)explicit_apply_kernel<T, 4, 16>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds4);
    explicit_apply_kernel<T, 4, 16><<<dim3((unsigned)a.nsub), dim3(256), lds4, st>>>(a);
  } else {
    const size_t lds2 = (size_t)3 * mp * sizeof(double);
    explicit_apply_kernel<T, 2, 8><<<dim3((unsigned)a.nsub), dim3(128), lds2, st>>>(a);
  }
}

template void launch_explicit_form<double>(const ExplicitForm&, int64_t, int64_t, hipStream_t);
template void launch_explicit_form<float>(const ExplicitForm&, int64_t, int64_t, hipStream_t);
template void launch_explicit_apply<double>(const ExplicitApply&, int, hipStream_t);
template void launch_explicit_apply<float>(const ExplicitApply&, int, hipStream_t);

}  // namespace tfeti

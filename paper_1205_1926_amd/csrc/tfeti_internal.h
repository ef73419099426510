// Internal definitions shared by the HIP sources of the TFETI library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tfeti.h"

namespace tfeti {

constexpr int kThreads = 256;     // threads per workgroup of the subdomain kernels
constexpr int kPadRows = 64;      // subdomain factors are padded to a multiple of this
// Row stride of a row-band matrix of half bandwidth b: b rounded up to a
// multiple of 16, plus one.  Entry (r, k) sits at r (stride - 1) + k + b, so
// with the band 16-entry aligned a column k that is a multiple of 16 minus b
// starts a 128-byte line in every row (the factorization streams 16-column
// chunks of many rows).
inline int32_t band_stride(int32_t b) { return (b + 15) / 16 * 16 + 1; }

// Per-subdomain description, identical on host and device.
struct SubDev {
  int32_t n[3];        // elements per local axis (x, y, z)
  int32_t N[3];        // nodes per local axis
  int32_t perm[3];     // factor ordering: perm[0] is the fastest axis
  int32_t fs[3];       // factor node stride of each local axis (x, y, z)
  int32_t ndof;        // 3 * nodes
  int32_t npad;        // ndof rounded up to kPadRows
  int32_t b;           // half bandwidth in the factor ordering
  int32_t Wb;          // row stride of the band, band_stride(b)
  int32_t bo;          // off-diagonal panel width (b rounded up to 4)
  int32_t n_iface;     // B-touched local DOFs
  int32_t n_elem;
  int32_t spare;
  int64_t dof_off;     // torn DOF offset
  int64_t elem_off;    // first element (global index)
  int64_t band_off;    // offset of the row-band matrices (entries)
  int64_t panel_off;   // offset of this subdomain's panels (entries of one layout)
  int64_t panel_len;   // entries of one layout for this subdomain
  int64_t iface_off;   // first touched DOF (global touched index)
  int32_t fix[9];      // factor indices of the fixing DOFs
  int32_t pad1;
};

// Factor index of local DOF (natural order a = i + Ni (j + Nj k), comp c).
// (fixed-index field accesses only, so device code keeps the struct in registers)
__host__ __device__ inline int32_t factor_index(const SubDev& s, int32_t ldof) {
  int32_t a = ldof / 3, c = ldof - 3 * a;
  int32_t i = a % s.N[0];
  int32_t t = a / s.N[0];
  int32_t j = t % s.N[1];
  int32_t k = t / s.N[1];
  return 3 * (i * s.fs[0] + j * s.fs[1] + k * s.fs[2]) + c;
}

// Rigid body modes of a box subdomain in closed form (the kernel of the
// floating subdomain's stiffness, Section 2): with node (i, j, k) at the
// coordinates (x, y, z) relative to the box centre, the three translations
// and the rotations (-y, x, 0), (0, -z, y), (z, 0, -x) are mutually
// orthogonal on a centred tensor grid, so scaling each by the inverse of its
// norm gives an orthonormal basis.  A touched DOF carries its doubled
// centred node coordinates 2 i - (N - 1) (signed 10-bit fields, so at most
// 512 nodes per axis) and its component in one packed word; the host's
// R values and the kernels use the same two roundings, x = (2 i - (N - 1))
// (h / 2) and then x * s.
__host__ __device__ inline uint32_t rigid_pack(int32_t xi, int32_t yi, int32_t zi, int32_t c) {
  return ((uint32_t)xi & 1023u) | (((uint32_t)yi & 1023u) << 10) | (((uint32_t)zi & 1023u) << 20) |
         ((uint32_t)c << 30);
}
// centred coordinates and component of a packed word; hh = half the element
// edge lengths
__host__ __device__ inline int32_t rigid_unpack(uint32_t pk, const double* hh, double& x, double& y, double& z) {
  x = (double)((int32_t)(pk << 22) >> 22) * hh[0];
  y = (double)((int32_t)(pk << 12) >> 22) * hh[1];
  z = (double)((int32_t)(pk << 2) >> 22) * hh[2];
  return (int32_t)(pk >> 30);
}
// the six mode values of one DOF; sc = (s_t, s_3, s_4, s_5), the inverse
// norms of the translations and of the three rotations (selects only, so
// device code keeps everything in registers)
__host__ __device__ inline void rigid_row(int32_t c, double x, double y, double z, const double (&sc)[4],
                                          double* R) {
  R[0] = c == 0 ? sc[0] : 0.0;
  R[1] = c == 1 ? sc[0] : 0.0;
  R[2] = c == 2 ? sc[0] : 0.0;
  const double r3a = -(y * sc[1]), r3b = x * sc[1];
  const double r4a = -(z * sc[2]), r4b = y * sc[2];
  const double r5a = z * sc[3], r5b = -(x * sc[3]);
  R[3] = c == 0 ? r3a : (c == 1 ? r3b : 0.0);
  R[4] = c == 1 ? r4a : (c == 2 ? r4b : 0.0);
  R[5] = c == 0 ? r5a : (c == 2 ? r5b : 0.0);
}

// Panel geometry: entries of one layout for tile TS, vector width V.
__host__ __device__ inline int64_t panel_entries(int32_t npad, int32_t bo, int32_t TS) {
  int64_t tot = 0;
  int32_t nb = npad / TS;
  for (int32_t I = 0; I < nb; ++I) {
    int32_t w = I * TS < bo ? I * TS : bo;
    tot += (int64_t)TS * (w + TS);
  }
  return tot;
}

struct PcgScalars {
  double ww, yw, yw_prev, pq, beta, gamma, r_ref, eps;
  double rr, tmp0, tmp1, tmp2;
  int32_t done, iters, maxit, nonfinite;
  int32_t spd_fail;
  int32_t pend;  // the updates r -= gamma q, lambda += gamma p are still to apply
  int32_t pad[2];
};

// Vector updates of a PCGP iteration folded into the kernels that read the
// vectors next (S == nullptr: none).  In the subdomain solve and the q
// gather, the direction is p = y + beta p (the gather stores it); in the
// first projection of the next iteration, r - gamma q replaces r and
// lambda + gamma p replaces lambda while S->pend is set.
struct PcgFold {
  const PcgScalars* S;
  const double* y;  // p = fma(beta, p, y)
  const double* q;  // r = fma(-gamma, q, r)
  double* p;        // lambda = fma(gamma, p, lambda)
  double* lam;
  double* r;
};

struct DeviceBuffers;

}  // namespace tfeti

struct tfeti_handle;

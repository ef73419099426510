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

// Per-subdomain description, identical on host and device.
struct SubDev {
  int32_t n[3];        // elements per local axis (x, y, z)
  int32_t N[3];        // nodes per local axis
  int32_t perm[3];     // factor ordering: perm[0] is the fastest axis
  int32_t fs[3];       // factor node stride of each local axis (x, y, z)
  int32_t ndof;        // 3 * nodes
  int32_t npad;        // ndof rounded up to kPadRows
  int32_t b;           // half bandwidth in the factor ordering
  int32_t Wb;          // row-band width b + 1
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
  int32_t spd_fail, pad[3];
};

struct DeviceBuffers;

}  // namespace tfeti

struct tfeti_handle;

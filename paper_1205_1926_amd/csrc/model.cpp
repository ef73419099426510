// Host-side construction of the TFETI model: structured Q1 mesh split into
// box subdomains, factor ordering, the orthonormal gluing matrix B
// (Section 4.1), rigid body modes (Section 4.2), index maps for the kernels,
// and the coarse matrix G G^T (Algorithm 3, first step).
#include "model.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace tfeti {

namespace {

inline int64_t gnode(const HostModel& M, int64_t i, int64_t j, int64_t k) {
  return i + (int64_t)(M.N[0] + 1) * (j + (int64_t)(M.N[1] + 1) * k);
}

// Shape-function gradients of the trilinear hexahedron on [-1,1]^3, nodes
// ordered (0,0,0),(1,0,0),(1,1,0),(0,1,0),(0,0,1),(1,0,1),(1,1,1),(0,1,1).
const int kNodeOff[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                            {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

void element_matrices(HostModel& M) {
  const double g = 1.0 / std::sqrt(3.0);
  for (int gp = 0; gp < 8; ++gp) {
    double xi[3] = {(gp & 1) ? g : -g, (gp & 2) ? g : -g, (gp & 4) ? g : -g};
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 24; ++c) M.Bg[gp][r][c] = 0.0;
    for (int a = 0; a < 8; ++a) {
      double s[3], f[3];
      for (int d = 0; d < 3; ++d) {
        s[d] = kNodeOff[a][d] ? 1.0 : -1.0;
        f[d] = 1.0 + xi[d] * s[d];
      }
      double dN[3];
      dN[0] = 0.125 * s[0] * f[1] * f[2] * (2.0 / M.h[0]);
      dN[1] = 0.125 * s[1] * f[0] * f[2] * (2.0 / M.h[1]);
      dN[2] = 0.125 * s[2] * f[0] * f[1] * (2.0 / M.h[2]);
      M.Bg[gp][0][3 * a + 0] = dN[0];
      M.Bg[gp][1][3 * a + 1] = dN[1];
      M.Bg[gp][2][3 * a + 2] = dN[2];
      M.Bg[gp][3][3 * a + 0] = dN[1];
      M.Bg[gp][3][3 * a + 1] = dN[0];
      M.Bg[gp][4][3 * a + 1] = dN[2];
      M.Bg[gp][4][3 * a + 2] = dN[1];
      M.Bg[gp][5][3 * a + 0] = dN[2];
      M.Bg[gp][5][3 * a + 2] = dN[0];
    }
  }
  M.wg = M.h[0] * M.h[1] * M.h[2] / 8.0;
}

// Orthonormalize the columns of an (n x k) row-major matrix in place by two
// passes of modified Gram-Schmidt.
void mgs(double* A, int n, int k) {
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < k; ++j) {
      for (int i = 0; i < j; ++i) {
        double d = 0.0;
        for (int r = 0; r < n; ++r) d += A[r * k + i] * A[r * k + j];
        for (int r = 0; r < n; ++r) A[r * k + j] -= d * A[r * k + i];
      }
      double nn = 0.0;
      for (int r = 0; r < n; ++r) nn += A[r * k + j] * A[r * k + j];
      nn = std::sqrt(nn);
      for (int r = 0; r < n; ++r) A[r * k + j] /= nn;
    }
}

}  // namespace

std::string build_model(const tfeti_problem& P, HostModel& M) {
  for (int a = 0; a < 3; ++a) {
    if (P.S[a] <= 0) return "S must be positive";
    if (!P.n_host[a]) return "n_host must not be NULL";
    if (!(P.extent[a] > 0.0)) return "extent must be positive";
    M.S[a] = P.S[a];
    M.slab[a].assign(P.n_host[a], P.n_host[a] + P.S[a]);
    M.N[a] = 0;
    for (int v : M.slab[a]) {
      if (v <= 0 || v > 64) return "slab element counts must be in 1..64";
      M.N[a] += v;
    }
    M.ext[a] = P.extent[a];
    M.h[a] = P.extent[a] / M.N[a];
  }
  if (!(P.mat.E > 0 && P.mat.nu > -1.0 && P.mat.nu < 0.5 && P.mat.sigma_y > 0 && P.mat.H > 0))
    return "material must satisfy E > 0, -1 < nu < 0.5, sigma_y > 0, H > 0";
  M.mat = P.mat;
  std::memcpy(M.dir, P.dirichlet, sizeof(M.dir));
  std::memcpy(M.trac, P.traction, sizeof(M.trac));
  element_matrices(M);

  const int64_t Nx1 = M.N[0] + 1, Ny1 = M.N[1] + 1, Nz1 = M.N[2] + 1;
  M.n_gnodes = Nx1 * Ny1 * Nz1;
  M.n_gdof = 3 * M.n_gnodes;
  const int64_t n_box = (int64_t)M.S[0] * M.S[1] * M.S[2];
  if (n_box > (1 << 20)) return "too many subdomains";
  M.n_sub = 0;
  for (int64_t q = 0; q < n_box; ++q) M.n_sub += (P.absent_host && P.absent_host[q]) ? 0 : 1;
  if (M.n_sub == 0) return "every box of the decomposition is absent";

  // ---- subdomains ----
  std::vector<int32_t> start[3];
  for (int a = 0; a < 3; ++a) {
    start[a].resize(M.S[a]);
    int acc = 0;
    for (int I = 0; I < M.S[a]; ++I) {
      start[a][I] = acc;
      acc += M.slab[a][I];
    }
  }
  M.subs.resize(M.n_sub);
  M.sub_e0.resize(3 * M.n_sub);
  int64_t dof_off = 0, elem_off = 0, band_off = 0;
  int64_t p = -1;
  for (int K = 0; K < M.S[2]; ++K)
    for (int J = 0; J < M.S[1]; ++J)
      for (int I = 0; I < M.S[0]; ++I) {
        if (P.absent_host && P.absent_host[I + (int64_t)M.S[0] * (J + (int64_t)M.S[1] * K)]) continue;
        ++p;
        SubDev& s = M.subs[p];
        std::memset(&s, 0, sizeof(SubDev));
        s.n[0] = M.slab[0][I];
        s.n[1] = M.slab[1][J];
        s.n[2] = M.slab[2][K];
        for (int a = 0; a < 3; ++a) s.N[a] = s.n[a] + 1;
        M.sub_e0[3 * p + 0] = start[0][I];
        M.sub_e0[3 * p + 1] = start[1][J];
        M.sub_e0[3 * p + 2] = start[2][K];
        // factor ordering: axes by increasing node count (stable), so that
        // the half bandwidth 3 (N0 N1 + N0 + 1) + 2 is the smallest
        int ord[3] = {0, 1, 2};
        std::stable_sort(ord, ord + 3, [&](int x, int y) { return s.N[x] < s.N[y]; });
        for (int a = 0; a < 3; ++a) s.perm[a] = ord[a];
        s.fs[ord[0]] = 1;
        s.fs[ord[1]] = s.N[ord[0]];
        s.fs[ord[2]] = s.N[ord[0]] * s.N[ord[1]];
        int64_t nn = (int64_t)s.N[0] * s.N[1] * s.N[2];
        s.ndof = (int32_t)(3 * nn);
        s.npad = (s.ndof + kPadRows - 1) / kPadRows * kPadRows;
        int32_t N0 = s.N[s.perm[0]], N1 = s.N[s.perm[1]], N2 = s.N[s.perm[2]];
        s.b = 3 * (N0 * N1 + N0 + 1) + 2;
        s.Wb = band_stride(s.b);
        s.bo = (s.b + 3) / 4 * 4;
        s.n_elem = s.n[0] * s.n[1] * s.n[2];
        s.dof_off = dof_off;
        s.elem_off = elem_off;
        s.band_off = band_off;
        dof_off += s.ndof;
        elem_off += s.n_elem;
        band_off += (int64_t)s.npad * s.Wb;
        // fixing nodes: three non-collinear corners of the last node layer
        int32_t last = N2 - 1;
        int32_t fn[3] = {0 + N0 * (0 + N1 * last), (N0 - 1) + N0 * (0 + N1 * last),
                         0 + N0 * ((N1 - 1) + N1 * last)};
        for (int q = 0; q < 3; ++q)
          for (int c = 0; c < 3; ++c) s.fix[3 * q + c] = 3 * fn[q] + c;
      }
  M.n_torn = dof_off;
  M.n_elem = elem_off;
  M.n_gp = 8 * elem_off;
  M.band_entries = band_off;
  if (M.n_torn >= (int64_t)1 << 31) return "torn vector too long for 32-bit indices";

  // skyline (envelope) size of the factors: per row, distance to the first
  // coupled column in the factor ordering
  M.skyline_entries = 0;
  M.skyline_sub.assign(M.subs.size(), 0);
  for (const SubDev& s : M.subs) {
    const int64_t sky0 = M.skyline_entries;
    int32_t N0 = s.N[s.perm[0]], N1 = s.N[s.perm[1]], N2 = s.N[s.perm[2]];
    for (int32_t c2 = 0; c2 < N2; ++c2)
      for (int32_t c1 = 0; c1 < N1; ++c1)
        for (int32_t c0 = 0; c0 < N0; ++c0) {
          int32_t f = c0 + N0 * (c1 + N1 * c2);
          int32_t g0 = std::max(c0 - 1, 0), g1 = std::max(c1 - 1, 0), g2 = std::max(c2 - 1, 0);
          // smallest neighbour node index: lowest in every axis, but the
          // neighbour must lie in an element shared with the node
          int32_t fmin = g0 + N0 * (g1 + N1 * g2);
          for (int c = 0; c < 3; ++c) M.skyline_entries += 3 * (f - fmin) + c + 1;
        }
    M.skyline_sub[&s - M.subs.data()] = M.skyline_entries - sky0;
  }

  // ---- global node -> copies (p ascending) ----
  std::vector<int32_t> cnt(M.n_gnodes + 1, 0);
  for (int64_t p = 0; p < M.n_sub; ++p) {
    const SubDev& s = M.subs[p];
    for (int32_t k = 0; k < s.N[2]; ++k)
      for (int32_t j = 0; j < s.N[1]; ++j)
        for (int32_t i = 0; i < s.N[0]; ++i)
          cnt[gnode(M, M.sub_e0[3 * p] + i, M.sub_e0[3 * p + 1] + j, M.sub_e0[3 * p + 2] + k) + 1]++;
  }
  for (int64_t g = 0; g < M.n_gnodes; ++g) cnt[g + 1] += cnt[g];
  std::vector<int32_t> cp_sub(cnt[M.n_gnodes]), cp_loc(cnt[M.n_gnodes]);
  {
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t p = 0; p < M.n_sub; ++p) {
      const SubDev& s = M.subs[p];
      for (int32_t k = 0; k < s.N[2]; ++k)
        for (int32_t j = 0; j < s.N[1]; ++j)
          for (int32_t i = 0; i < s.N[0]; ++i) {
            int64_t g = gnode(M, M.sub_e0[3 * p] + i, M.sub_e0[3 * p + 1] + j, M.sub_e0[3 * p + 2] + k);
            int32_t a = i + s.N[0] * (j + s.N[1] * k);
            cp_sub[fill[g]] = (int32_t)p;
            cp_loc[fill[g]] = a;
            fill[g]++;
          }
    }
  }

  // ---- Dirichlet mask per (global node, component) ----
  auto dirichlet = [&](int64_t g, int c) -> bool {
    int64_t i = g % Nx1, j = (g / Nx1) % Ny1, k = g / (Nx1 * Ny1);
    bool on[6] = {i == 0, i == M.N[0], j == 0, j == M.N[1], k == 0, k == M.N[2]};
    for (int f = 0; f < 6; ++f)
      if (on[f] && M.dir[f][c]) return true;
    return false;
  };

  // ---- B: Helmert gluing rows, then Dirichlet rows ----
  struct Ent {
    int32_t p, a, c;
    double v;
  };
  std::vector<int64_t> rpG{0}, rpU{0};
  std::vector<Ent> eG, eU;
  std::vector<int64_t> rnodeG, rnodeU;   // global node of each row
  std::vector<int8_t> rslotG, rslotU;    // slot 7 c + index within the node
  std::vector<uint8_t> gfree_full(M.n_gdof, 1);
  for (int64_t g = 0; g < M.n_gnodes; ++g) {
    int32_t k = cnt[g + 1] - cnt[g];
    for (int c = 0; c < 3; ++c) {
      if (dirichlet(g, c)) {
        gfree_full[3 * g + c] = 0;
        for (int32_t t = 0; t < k; ++t) {
          eU.push_back({cp_sub[cnt[g] + t], cp_loc[cnt[g] + t], c, 1.0});
          rpU.push_back((int64_t)eU.size());
          rnodeU.push_back(g);
          rslotU.push_back((int8_t)(7 * c + t));
        }
      } else if (k > 1) {
        for (int32_t j = 1; j < k; ++j) {
          double cj = 1.0 / std::sqrt((double)(j * (j + 1)));
          for (int32_t t = 0; t < j; ++t) eG.push_back({cp_sub[cnt[g] + t], cp_loc[cnt[g] + t], c, cj});
          eG.push_back({cp_sub[cnt[g] + j], cp_loc[cnt[g] + j], c, -(double)j * cj});
          rpG.push_back((int64_t)eG.size());
          rnodeG.push_back(g);
          rslotG.push_back((int8_t)(7 * c + (j - 1)));
        }
      }
    }
  }
  M.mG = (int64_t)rpG.size() - 1;
  M.mU = (int64_t)rpU.size() - 1;
  M.m = M.mG + M.mU;
  if (M.m >= (int64_t)1 << 31) return "too many multipliers";
  int64_t nnz = (int64_t)eG.size() + (int64_t)eU.size();
  M.b_rowptr.resize(M.m + 1);
  M.b_col.resize(nnz);
  M.b_val.resize(nnz);
  std::vector<int32_t> e_sub(nnz), e_ldof(nnz);
  for (int64_t r = 0; r <= M.mG; ++r) M.b_rowptr[r] = rpG[r];
  for (int64_t r = 1; r <= M.mU; ++r) M.b_rowptr[M.mG + r] = (int64_t)eG.size() + rpU[r];
  for (int64_t e = 0; e < nnz; ++e) {
    const Ent& x = e < (int64_t)eG.size() ? eG[e] : eU[e - eG.size()];
    e_sub[e] = x.p;
    e_ldof[e] = 3 * x.a + x.c;
    M.b_col[e] = M.subs[x.p].dof_off + 3 * x.a + x.c;
    M.b_val[e] = x.v;
  }

  // ---- touched DOFs per subdomain ----
  std::vector<int32_t> tidx(M.n_torn, -1);
  for (int64_t e = 0; e < nnz; ++e) tidx[M.b_col[e]] = 0;
  M.n_iface = 0;
  for (int64_t p = 0; p < M.n_sub; ++p) {
    SubDev& s = M.subs[p];
    s.iface_off = M.n_iface;
    int32_t cntp = 0;
    for (int32_t ld = 0; ld < s.ndof; ++ld)
      if (tidx[s.dof_off + ld] >= 0) {
        tidx[s.dof_off + ld] = (int32_t)(M.n_iface + cntp);
        M.if_ldof.push_back(ld);
        M.if_fidx.push_back(factor_index(s, ld));
        ++cntp;
      }
    s.n_iface = cntp;
    M.n_iface += cntp;
  }
  M.b_iface.resize(nnz);
  for (int64_t e = 0; e < nnz; ++e) M.b_iface[e] = tidx[M.b_col[e]];
  // B^T per touched DOF: entries (row, coef) in row order
  M.if_rp.assign(M.n_iface + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) M.if_rp[M.b_iface[e] + 1]++;
  for (int64_t t = 0; t < M.n_iface; ++t) M.if_rp[t + 1] += M.if_rp[t];
  M.if_row.resize(nnz);
  M.if_coef.resize(nnz);
  {
    std::vector<int32_t> fill(M.if_rp.begin(), M.if_rp.end() - 1);
    for (int64_t r = 0; r < M.m; ++r)
      for (int64_t e = M.b_rowptr[r]; e < M.b_rowptr[r + 1]; ++e) {
        int32_t t = M.b_iface[e];
        M.if_row[fill[t]] = (int32_t)r;
        M.if_coef[fill[t]] = M.b_val[e];
        fill[t]++;
      }
  }

  // ---- rigid body modes: closed form on the centred box grid ----
  M.R_full.assign(6 * M.n_torn, 0.0);
  M.rscale.assign(4 * M.n_sub, 0.0);
  M.QQt.assign(81 * M.n_sub, 0.0);
  const double hh[3] = {0.5 * M.h[0], 0.5 * M.h[1], 0.5 * M.h[2]};
  auto node_pack = [&](const SubDev& s, int32_t ldof) {
    int32_t a = ldof / 3, c = ldof - 3 * a;
    int32_t i = a % s.N[0], j = (a / s.N[0]) % s.N[1], k = a / (s.N[0] * s.N[1]);
    return rigid_pack(2 * i - (s.N[0] - 1), 2 * j - (s.N[1] - 1), 2 * k - (s.N[2] - 1), c);
  };
  for (int64_t p = 0; p < M.n_sub; ++p) {
    const SubDev& s = M.subs[p];
    if (s.N[0] > 512 || s.N[1] > 512 || s.N[2] > 512) return "a subdomain has more than 512 nodes on an axis";
    int64_t nn = s.ndof / 3;
    double sxy = 0.0, syz = 0.0, sxz = 0.0;
    for (int32_t a = 0; a < nn; ++a) {
      double x, y, z;
      rigid_unpack(node_pack(s, 3 * a), hh, x, y, z);
      sxy += x * x + y * y;
      syz += y * y + z * z;
      sxz += x * x + z * z;
    }
    const double sc[4] = {1.0 / std::sqrt((double)nn), 1.0 / std::sqrt(sxy), 1.0 / std::sqrt(syz),
                          1.0 / std::sqrt(sxz)};
    for (int q = 0; q < 4; ++q) M.rscale[4 * p + q] = sc[q];
    double* R = &M.R_full[6 * s.dof_off];
    for (int32_t ld = 0; ld < s.ndof; ++ld) {
      double x, y, z;
      const int32_t c = rigid_unpack(node_pack(s, ld), hh, x, y, z);
      rigid_row(c, x, y, z, sc, R + 6 * ld);
    }
    // Q: orthonormal basis of the rows of R at the fixing DOFs
    double Rs[9 * 6];
    for (int q = 0; q < 9; ++q) {
      // find the local natural DOF of factor index s.fix[q]
      int32_t f = s.fix[q], fnode = f / 3, c = f % 3;
      int32_t N0 = s.N[s.perm[0]], N1 = s.N[s.perm[1]];
      int32_t co[3];
      co[s.perm[0]] = fnode % N0;
      co[s.perm[1]] = (fnode / N0) % N1;
      co[s.perm[2]] = fnode / (N0 * N1);
      int32_t a = co[0] + s.N[0] * (co[1] + s.N[1] * co[2]);
      for (int j = 0; j < 6; ++j) Rs[6 * q + j] = R[6 * (3 * a + c) + j];
    }
    mgs(Rs, 9, 6);
    double* Q = &M.QQt[81 * p];
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) {
        double v = 0.0;
        for (int c = 0; c < 6; ++c) v += Rs[6 * i + c] * Rs[6 * j + c];
        Q[9 * i + j] = v;
      }
  }
  // packed node coordinates of every B entry and of every B^T entry
  M.b_sub.resize(nnz);
  M.b_pk.resize(nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    M.b_sub[e] = e_sub[e];
    M.b_pk[e] = node_pack(M.subs[e_sub[e]], e_ldof[e]);
  }
  M.if_pk.resize(nnz);
  for (int64_t p = 0; p < M.n_sub; ++p) {
    const SubDev& s = M.subs[p];
    for (int32_t t = 0; t < s.n_iface; ++t) {
      const int64_t it = s.iface_off + t;
      const uint32_t pk = node_pack(s, M.if_ldof[it]);
      for (int32_t e = M.if_rp[it]; e < M.if_rp[it + 1]; ++e) M.if_pk[e] = pk;
    }
  }

  // ---- K_bb (lumped preconditioner): per touched DOF, the touched nodes
  //      among the 27 nodes around its own (bit 9 (dk+1) + 3 (dj+1) + di+1)
  //      and three values (the three components) per such node.  The touched
  //      DOFs of a subdomain are sorted by their node count (stable) and cut
  //      into groups of 64, one wavefront each; a group stores its values
  //      slot-major, value (3 b + c) of lane l at off + (3 b + c) 64 + l,
  //      padded with zeros to the group's largest count. ----
  {
    std::vector<uint8_t> node_touched(M.n_torn / 3, 0);
    for (int64_t e = 0; e < nnz; ++e) node_touched[M.b_col[e] / 3] = 1;
    M.kbb_g0.assign(M.n_sub + 1, 0);
    M.kbb_row.clear();
    M.kbb_mask.clear();
    M.kbb_node.clear();
    M.kbb_goff.assign(1, 0);
    M.kbb_gnb.clear();
    M.kbb_gsub.clear();
    for (int64_t p = 0; p < M.n_sub; ++p) {
      const SubDev& s = M.subs[p];
      std::vector<uint32_t> mask(s.n_iface);
      std::vector<int32_t> ord(s.n_iface);
      for (int32_t t = 0; t < s.n_iface; ++t) {
        const int64_t it = s.iface_off + t;
        int32_t a = M.if_ldof[it] / 3;
        int32_t i = a % s.N[0], j = (a / s.N[0]) % s.N[1], k = a / (s.N[0] * s.N[1]);
        uint32_t mk = 0;
        for (int dk = -1; dk <= 1; ++dk)
          for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
              int32_t ii = i + di, jj = j + dj, kk = k + dk;
              if (ii < 0 || jj < 0 || kk < 0 || ii >= s.N[0] || jj >= s.N[1] || kk >= s.N[2]) continue;
              int32_t a2 = ii + s.N[0] * (jj + s.N[1] * kk);
              if (node_touched[s.dof_off / 3 + a2]) mk |= 1u << (9 * (dk + 1) + 3 * (dj + 1) + (di + 1));
            }
        mask[t] = mk;
        ord[t] = t;
      }
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
        return __builtin_popcount(mask[x]) > __builtin_popcount(mask[y]);
      });
      const int32_t ng = (s.n_iface + 63) / 64;
      for (int32_t g = 0; g < ng; ++g) {
        int32_t nb = 0;
        for (int32_t l = 0; l < 64; ++l) {
          const int32_t q = 64 * g + l;
          if (q < s.n_iface) {
            M.kbb_row.push_back((int32_t)(s.iface_off + ord[q]));
            M.kbb_mask.push_back(mask[ord[q]]);
            M.kbb_node.push_back(M.if_ldof[s.iface_off + ord[q]] / 3);
            nb = std::max(nb, __builtin_popcount(mask[ord[q]]));
          } else {
            M.kbb_row.push_back(-1);
            M.kbb_mask.push_back(0u);
            M.kbb_node.push_back(0);
          }
        }
        M.kbb_gnb.push_back(nb);
        M.kbb_gsub.push_back((int32_t)p);
        M.kbb_goff.push_back(M.kbb_goff.back() + (int64_t)3 * nb * 64);
      }
      M.kbb_g0[p + 1] = M.kbb_g0[p] + ng;
    }
  }

  // ---- Dirichlet preconditioner: interior boxes and the couplings of the
  //      interior with the touched nodes ----
  {
    std::vector<uint8_t> node_touched(M.n_torn / 3, 0);
    for (int64_t e = 0; e < nnz; ++e) node_touched[M.b_col[e] / 3] = 1;
    M.isubs.assign(M.n_sub, SubDev{});
    M.ilo.assign(3 * M.n_sub, 0);
    int64_t ioff = 0, iband = 0;
    for (int64_t p = 0; p < M.n_sub; ++p) {
      const SubDev& s = M.subs[p];
      SubDev& si = M.isubs[p];
      std::memset(&si, 0, sizeof(SubDev));
      // bounding box of the nodes without a row of B
      int32_t lo[3] = {s.N[0], s.N[1], s.N[2]}, hi[3] = {-1, -1, -1};
      int64_t cnt_in = 0;
      for (int32_t k = 0; k < s.N[2]; ++k)
        for (int32_t j = 0; j < s.N[1]; ++j)
          for (int32_t i = 0; i < s.N[0]; ++i) {
            const int32_t a = i + s.N[0] * (j + s.N[1] * k);
            if (node_touched[s.dof_off / 3 + a]) continue;
            ++cnt_in;
            const int32_t c[3] = {i, j, k};
            for (int d = 0; d < 3; ++d) {
              lo[d] = std::min(lo[d], c[d]);
              hi[d] = std::max(hi[d], c[d]);
            }
          }
      if (cnt_in == 0) continue;
      int64_t box = 1;
      for (int d = 0; d < 3; ++d) box *= hi[d] - lo[d] + 1;
      if (box != cnt_in) {
        // a hole's edge or corner leaves interface nodes between free faces:
        // the lumped preconditioner still applies, the Dirichlet one is refused
        M.interior_error = "the interior nodes of subdomain " + std::to_string(p) +
                           " do not form a box (Dirichlet preconditioner unavailable)";
        break;
      }
      for (int d = 0; d < 3; ++d) {
        M.ilo[3 * p + d] = lo[d];
        si.N[d] = hi[d] - lo[d] + 1;
        si.n[d] = si.N[d] - 1;
      }
      int ord[3] = {0, 1, 2};
      std::stable_sort(ord, ord + 3, [&](int x, int y) { return si.N[x] < si.N[y]; });
      for (int d = 0; d < 3; ++d) si.perm[d] = ord[d];
      si.fs[ord[0]] = 1;
      si.fs[ord[1]] = si.N[ord[0]];
      si.fs[ord[2]] = si.N[ord[0]] * si.N[ord[1]];
      si.ndof = (int32_t)(3 * cnt_in);
      si.npad = (si.ndof + kPadRows - 1) / kPadRows * kPadRows;
      const int32_t N0 = si.N[si.perm[0]], N1 = si.N[si.perm[1]];
      si.b = std::min(3 * (N0 * N1 + N0 + 1) + 2, si.npad - 1);
      si.Wb = band_stride(si.b);
      si.bo = (si.b + 3) / 4 * 4;
      si.dof_off = ioff;
      si.band_off = iband;
      ioff += si.ndof;
      iband += (int64_t)si.npad * si.Wb;
    }
    if (!M.interior_error.empty()) {
      M.isubs.assign(M.n_sub, SubDev{});
      M.ilo.assign(3 * M.n_sub, 0);
      ioff = iband = 0;
    }
    M.n_int = ioff;
    M.iband_entries = iband;
    // rows in groups of 64 sorted by neighbour count; cols(p, node) tells
    // whether a neighbour node is a column node
    auto build = [&](NbGroupsHost& G, bool keep_empty, auto rows_of, auto is_col) {
      G = NbGroupsHost{};
      G.g0.assign(M.n_sub + 1, 0);
      for (int64_t p = 0; p < M.n_sub; ++p) {
        const SubDev& s = M.subs[p];
        std::vector<int32_t> ld, out;
        rows_of(p, ld, out);
        std::vector<uint32_t> mask(ld.size(), 0u);
        std::vector<int32_t> ord;
        for (size_t t = 0; t < ld.size(); ++t) {
          const int32_t a = ld[t] / 3;
          const int32_t i = a % s.N[0], j = (a / s.N[0]) % s.N[1], k = a / (s.N[0] * s.N[1]);
          uint32_t mk = 0;
          for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
              for (int di = -1; di <= 1; ++di) {
                const int32_t ii = i + di, jj = j + dj, kk = k + dk;
                if (ii < 0 || jj < 0 || kk < 0 || ii >= s.N[0] || jj >= s.N[1] || kk >= s.N[2]) continue;
                if (is_col(p, ii + s.N[0] * (jj + s.N[1] * kk)))
                  mk |= 1u << (9 * (dk + 1) + 3 * (dj + 1) + (di + 1));
              }
          mask[t] = mk;
          if (mk || keep_empty) ord.push_back((int32_t)t);
        }
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
          return __builtin_popcount(mask[x]) > __builtin_popcount(mask[y]);
        });
        const int32_t nrow = (int32_t)ord.size(), ng = (nrow + 63) / 64;
        for (int32_t g = 0; g < ng; ++g) {
          int32_t nb = 0;
          for (int32_t l = 0; l < 64; ++l) {
            const int32_t q = 64 * g + l;
            if (q < nrow) {
              G.out.push_back(out[ord[q]]);
              G.ldof.push_back(ld[ord[q]]);
              G.mask.push_back(mask[ord[q]]);
              nb = std::max(nb, __builtin_popcount(mask[ord[q]]));
            } else {
              G.out.push_back(-1);
              G.ldof.push_back(ld[ord[0]]);
              G.mask.push_back(0u);
            }
          }
          G.gnb.push_back(nb);
          G.gsub.push_back((int32_t)p);
          G.goff.push_back(G.goff.back() + (int64_t)3 * nb * 64);
        }
        G.g0[p + 1] = G.g0[p] + ng;
      }
    };
    auto interior = [&](int64_t p, int32_t a) { return M.isubs[p].ndof > 0 && !node_touched[M.subs[p].dof_off / 3 + a]; };
    if (M.interior_error.empty()) {
    // K_it: every DOF of an interior node (rows without a touched neighbour
    // too, so that every interior entry is written); output at its interior DOF
    build(M.kit, true,
          [&](int64_t p, std::vector<int32_t>& ld, std::vector<int32_t>& out) {
            const SubDev& s = M.subs[p];
            const SubDev& si = M.isubs[p];
            const int32_t* lo = &M.ilo[3 * p];
            for (int32_t li = 0; li < si.ndof; ++li) {
              const int32_t ai = li / 3, c = li % 3;
              const int32_t ii = ai % si.N[0], jj = (ai / si.N[0]) % si.N[1], kk = ai / (si.N[0] * si.N[1]);
              const int32_t a = (ii + lo[0]) + s.N[0] * ((jj + lo[1]) + s.N[1] * (kk + lo[2]));
              ld.push_back(3 * a + c);
              out.push_back((int32_t)(si.dof_off + li));
            }
          },
          [&](int64_t p, int32_t a) { return node_touched[M.subs[p].dof_off / 3 + a] != 0; });
    // K_ti: the touched DOFs next to an interior node; output at the touched index
    build(M.kti, false,
          [&](int64_t p, std::vector<int32_t>& ld, std::vector<int32_t>& out) {
            const SubDev& s = M.subs[p];
            for (int32_t t = 0; t < s.n_iface; ++t) {
              ld.push_back(M.if_ldof[s.iface_off + t]);
              out.push_back((int32_t)(s.iface_off + t));
            }
          },
          interior);
    }
    if (M.n_int >= (int64_t)1 << 31) return "too many interior DOFs for 32-bit indices";
  }

  // ---- untorn maps: the global DOFs of the nodes in some subdomain (all of
  //      them unless boxes are absent), node ascending ----
  int64_t used_nodes = 0;
  for (int64_t g = 0; g < M.n_gnodes; ++g) used_nodes += cnt[g + 1] > cnt[g] ? 1 : 0;
  M.n_gdof = 3 * used_nodes;
  M.g_first.resize(M.n_gdof);
  M.g_rp.assign(M.n_gdof + 1, 0);
  M.g_free.assign(M.n_gdof, 1);
  M.g_copies.clear();
  M.g_copies.reserve(3 * cp_sub.size());
  for (int64_t g = 0, gu = 0; g < M.n_gnodes; ++g) {
    if (cnt[g + 1] == cnt[g]) continue;
    for (int c = 0; c < 3; ++c) {
      const int64_t gd = 3 * gu + c;
      for (int32_t t = cnt[g]; t < cnt[g + 1]; ++t)
        M.g_copies.push_back(M.subs[cp_sub[t]].dof_off + 3 * cp_loc[t] + c);
      M.g_first[gd] = M.subs[cp_sub[cnt[g]]].dof_off + 3 * cp_loc[cnt[g]] + c;
      M.g_rp[gd + 1] = (int32_t)M.g_copies.size();
      M.g_free[gd] = gfree_full[3 * g + c];
    }
    ++gu;
  }

  // ---- colouring of elements ----
  M.elem_sub.resize(M.n_elem);
  for (int c = 0; c < 8; ++c) M.colour_elems[c].clear();
  for (int64_t p = 0; p < M.n_sub; ++p) {
    const SubDev& s = M.subs[p];
    for (int32_t k = 0; k < s.n[2]; ++k)
      for (int32_t j = 0; j < s.n[1]; ++j)
        for (int32_t i = 0; i < s.n[0]; ++i) {
          int64_t e = s.elem_off + i + s.n[0] * (j + s.n[1] * k);
          M.elem_sub[e] = (int32_t)p;
          M.colour_elems[(i & 1) | ((j & 1) << 1) | ((k & 1) << 2)].push_back((int32_t)e);
        }
  }

  // ---- load at factor 1: each subdomain integrates its own loaded faces ----
  M.f1.assign(M.n_torn, 0.0);
  const double gq = 1.0 / std::sqrt(3.0);
  for (int64_t p = 0; p < M.n_sub; ++p) {
    const SubDev& s = M.subs[p];
    for (int face = 0; face < 6; ++face) {
      const double* t = M.trac[face];
      if (t[0] == 0.0 && t[1] == 0.0 && t[2] == 0.0) continue;
      int ax = face / 2, side = face % 2;
      int loc = side ? s.n[ax] : 0;
      if (M.sub_e0[3 * p + ax] + loc != (side ? M.N[ax] : 0)) continue;
      int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
      double jac = M.h[a1] * M.h[a2] / 4.0;
      const double ref[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
      double fl[4] = {0, 0, 0, 0};
      for (int gj = 0; gj < 2; ++gj)
        for (int gi = 0; gi < 2; ++gi) {
          double u = gi ? gq : -gq, v = gj ? gq : -gq;
          for (int q = 0; q < 4; ++q) fl[q] += 0.25 * (1 + u * ref[q][0]) * (1 + v * ref[q][1]) * jac;
        }
      const int dd[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
      for (int ib = 0; ib < s.n[a2]; ++ib)
        for (int ia = 0; ia < s.n[a1]; ++ia)
          for (int q = 0; q < 4; ++q) {
            int co[3];
            co[ax] = loc;
            co[a1] = ia + dd[q][0];
            co[a2] = ib + dd[q][1];
            int32_t a = co[0] + s.N[0] * (co[1] + s.N[1] * co[2]);
            for (int c = 0; c < 3; ++c) M.f1[s.dof_off + 3 * a + c] += fl[q] * t[c];
          }
    }
  }

  // ---- coarse matrix G G^T (G = R^T B^T), lower row-band ----
  // The coarse unknowns are numbered by the boxes in lexicographic order with
  // the axis of fewest boxes fastest, which keeps the band of G G^T narrow on
  // flat decompositions (20 x 20 x 2 boxes: neighbours 43 positions apart
  // instead of 421); the inverse is gathered back to subdomain order.
  M.lc = (int32_t)(6 * M.n_sub);
  {
    int ax[3] = {0, 1, 2};
    std::stable_sort(ax, ax + 3, [&](int x, int y) { return M.S[x] < M.S[y]; });
    std::vector<int32_t> box_p((size_t)n_box, -1);
    {
      int64_t q = 0;
      for (int K = 0; K < M.S[2]; ++K)
        for (int J = 0; J < M.S[1]; ++J)
          for (int I = 0; I < M.S[0]; ++I) {
            const int64_t bi = I + (int64_t)M.S[0] * (J + (int64_t)M.S[1] * K);
            if (!(P.absent_host && P.absent_host[bi])) box_p[bi] = (int32_t)q++;
          }
    }
    M.cpos.assign(M.n_sub, 0);
    int32_t pos = 0;
    int c[3];
    for (c[ax[2]] = 0; c[ax[2]] < M.S[ax[2]]; ++c[ax[2]])
      for (c[ax[1]] = 0; c[ax[1]] < M.S[ax[1]]; ++c[ax[1]])
        for (c[ax[0]] = 0; c[ax[0]] < M.S[ax[0]]; ++c[ax[0]]) {
          const int32_t q = box_p[c[0] + (int64_t)M.S[0] * (c[1] + (int64_t)M.S[1] * c[2])];
          if (q >= 0) M.cpos[q] = pos++;
        }
  }
  int64_t maxdp = 0;
  for (int64_t r = 0; r < M.m; ++r)
    for (int64_t e = M.b_rowptr[r]; e < M.b_rowptr[r + 1]; ++e)
      for (int64_t e2 = M.b_rowptr[r]; e2 < M.b_rowptr[r + 1]; ++e2)
        maxdp = std::max<int64_t>(maxdp, std::abs((int64_t)M.cpos[e_sub[e]] - M.cpos[e_sub[e2]]));
  M.bc = (int32_t)(6 * maxdp + 5);
  M.lc_pad = (M.lc + kPadRows - 1) / kPadRows * kPadRows;
  M.Wc = band_stride(M.bc);
  const int64_t Wc = M.Wc;
  M.GGt_band.assign((int64_t)M.lc_pad * Wc, 0.0);
  for (int64_t r = 0; r < M.m; ++r) {
    // column r of G: for entry (p, ldof, v): v * R_p[ldof, :] at rows 6p..6p+5
    int64_t e0 = M.b_rowptr[r], e1 = M.b_rowptr[r + 1];
    for (int64_t e = e0; e < e1; ++e)
      for (int64_t e2 = e0; e2 < e1; ++e2) {
        const int64_t pa = M.cpos[e_sub[e]], pb = M.cpos[e_sub[e2]];
        if (pa < pb) continue;
        const double* Ra = &M.R_full[6 * M.b_col[e]];
        const double* Rb = &M.R_full[6 * M.b_col[e2]];
        double va = M.b_val[e], vb = M.b_val[e2];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 6; ++j) {
            int64_t gi = 6 * pa + i, gj = 6 * pb + j;
            if (gj > gi) continue;
            M.GGt_band[gi * Wc + (gj - gi + M.bc)] += (va * Ra[i]) * (vb * Rb[j]);
          }
      }
  }
  for (int64_t i = M.lc; i < M.lc_pad; ++i) M.GGt_band[i * Wc + M.bc] = 1.0;

  // ---- interface nodes of the learned warm start ----
  {
    std::vector<int32_t> node_of(M.n_gnodes, -1);
    std::vector<int64_t> wn_g;
    auto visit = [&](int64_t g) {
      if (node_of[g] < 0) {
        node_of[g] = (int32_t)wn_g.size();
        wn_g.push_back(g);
      }
      return node_of[g];
    };
    for (int64_t r = 0; r < M.mG; ++r) visit(rnodeG[r]);
    for (int64_t r = 0; r < M.mU; ++r) visit(rnodeU[r]);
    M.n_wnodes = (int64_t)wn_g.size();
    M.wn_rows.assign(21 * M.n_wnodes, -1);
    M.wn_class.assign(M.n_wnodes, 0);
    std::vector<uint8_t> has_dir(M.n_wnodes, 0);
    for (int64_t r = 0; r < M.mG; ++r) M.wn_rows[21 * node_of[rnodeG[r]] + rslotG[r]] = (int32_t)r;
    for (int64_t r = 0; r < M.mU; ++r) {
      M.wn_rows[21 * node_of[rnodeU[r]] + rslotU[r]] = (int32_t)(M.mG + r);
      has_dir[node_of[rnodeU[r]]] = 1;
    }
    M.wn_erp.assign(M.n_wnodes + 1, 0);
    M.wn_elems.clear();
    for (int64_t q = 0; q < M.n_wnodes; ++q) {
      const int64_t g = wn_g[q];
      const int32_t k = cnt[g + 1] - cnt[g];
      int8_t cls;
      if (has_dir[q])
        cls = (int8_t)(k >= 4 ? 5 : (k >= 2 ? 4 : 3));
      else
        cls = (int8_t)(k >= 8 ? 2 : (k >= 4 ? 1 : 0));
      M.wn_class[q] = cls;
      for (int32_t t = cnt[g]; t < cnt[g + 1]; ++t) {
        const SubDev& s = M.subs[cp_sub[t]];
        const int32_t a = cp_loc[t];
        const int32_t i = a % s.N[0], j = (a / s.N[0]) % s.N[1], kk = a / (s.N[0] * s.N[1]);
        for (int dk = 0; dk < 2; ++dk)
          for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
              int32_t ei = i - di, ej = j - dj, ek = kk - dk;
              if (ei < 0 || ej < 0 || ek < 0 || ei >= s.n[0] || ej >= s.n[1] || ek >= s.n[2]) continue;
              M.wn_elems.push_back((int32_t)(s.elem_off + ei + s.n[0] * (ej + s.n[1] * ek)));
            }
      }
      M.wn_erp[q + 1] = (int32_t)M.wn_elems.size();
    }
    // load scale: traction of the loaded face (the largest one) and its element face area
    double best = 0.0;
    for (int f = 0; f < 6; ++f) {
      double n2 = M.trac[f][0] * M.trac[f][0] + M.trac[f][1] * M.trac[f][1] + M.trac[f][2] * M.trac[f][2];
      if (n2 > best) {
        best = n2;
        for (int c = 0; c < 3; ++c) M.load_dir[c] = M.trac[f][c];
        int ax = f / 2;
        int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
        M.load_area = M.h[a1] * M.h[a2];
      }
    }
    if (best == 0.0) M.load_area = M.h[0] * M.h[1];
  }

  // ---- sanity checks of every index map against its target ----
  for (int64_t e = 0; e < nnz; ++e)
    if (M.b_col[e] < 0 || M.b_col[e] >= M.n_torn || M.b_iface[e] < 0 || M.b_iface[e] >= M.n_iface)
      return "internal: B map out of range";
  for (int64_t t = 0; t < M.n_iface; ++t)
    if (M.if_fidx[t] < 0) return "internal: touched DOF map";
  for (int64_t p = 0; p < M.n_sub; ++p) {
    const SubDev& s = M.subs[p];
    for (int32_t t = 0; t < s.n_iface; ++t)
      if (M.if_fidx[s.iface_off + t] >= s.ndof) return "internal: factor index out of range";
    for (int q = 0; q < 9; ++q)
      if (s.fix[q] < 0 || s.fix[q] >= s.ndof) return "internal: fixing DOF out of range";
  }
  for (size_t q = 0; q < M.wn_rows.size(); ++q)
    if (M.wn_rows[q] < -1 || M.wn_rows[q] >= M.m) return "internal: warm-start row map out of range";
  for (size_t q = 0; q < M.wn_elems.size(); ++q)
    if (M.wn_elems[q] < 0 || M.wn_elems[q] >= M.n_elem) return "internal: warm-start element map out of range";
  return "";
}

int64_t assign_interior_panels(HostModel& M, int TS) {
  int64_t off = 0;
  for (SubDev& s : M.isubs) {
    s.panel_off = off;
    s.panel_len = s.ndof > 0 ? panel_entries(s.npad, s.bo, TS) : 0;
    off += s.panel_len;
  }
  return off;
}

int64_t assign_panels(HostModel& M, int TS) {
  int64_t off = 0;
  for (SubDev& s : M.subs) {
    s.panel_off = off;
    s.panel_len = panel_entries(s.npad, s.bo, TS);
    off += s.panel_len;
  }
  return off;
}

}  // namespace tfeti

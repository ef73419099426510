// Host-side model: mesh, box decomposition, factor ordering, gluing matrix
// B, rigid modes, index maps and the coarse matrix G G^T.  Built once by
// tfeti_setup; only integer maps and FP64 constants, no device state.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "tfeti_internal.h"

namespace tfeti {

// Sparse rows in wavefront groups of 64 (the layout of the lumped K_bb):
// per lane slot the output index (-1 past the end), the local natural DOF of
// the row and its mask of column nodes among the 27 around its node (bit
// 9 (dk+1) + 3 (dj+1) + di+1); per group the value offset, the neighbour
// count and the subdomain; per subdomain its first group.  Values are stored
// slot-major: value (3 b + c) of lane l at goff + (3 b + c) 64 + l.
struct NbGroupsHost {
  std::vector<int32_t> out, ldof;
  std::vector<uint32_t> mask;
  std::vector<int64_t> goff{0};
  std::vector<int32_t> gnb, gsub, g0;
};

struct HostModel {
  // problem
  int32_t S[3];
  std::vector<int32_t> slab[3];
  double ext[3];
  tfeti_material mat;
  int32_t dir[6][3];
  double trac[6][3];
  // mesh
  int32_t N[3];          // global elements per axis
  double h[3];           // element edge lengths
  int64_t n_gnodes = 0, n_gdof = 0;
  int64_t n_torn = 0, n_elem = 0, n_gp = 0, n_sub = 0;
  std::vector<SubDev> subs;
  std::vector<int32_t> sub_e0;           // 3 per subdomain: first global element index per axis
  // B in CSR (rows of B_G then B_U)
  int64_t m = 0, mG = 0, mU = 0;
  std::vector<int64_t> b_rowptr;        // m + 1
  std::vector<int64_t> b_col;           // torn DOF per entry
  std::vector<double> b_val;
  std::vector<int32_t> b_iface;         // global touched index per entry
  // touched DOFs ("interface"): per subdomain ascending local DOF
  int64_t n_iface = 0;
  std::vector<int32_t> if_fidx;         // factor index
  std::vector<int32_t> if_ldof;         // local natural DOF
  std::vector<int32_t> if_rp;           // n_iface + 1: entries of B^T per touched DOF
  std::vector<int32_t> if_row;          // row of each entry
  std::vector<double> if_coef;
  // rigid modes
  std::vector<double> R_full;           // n_torn * 6 (torn order)
  std::vector<double> rscale;           // 4 per subdomain: inverse norms of the raw modes
  std::vector<int32_t> b_sub;           // subdomain of each B entry
  std::vector<uint32_t> b_pk;           // packed centred node coordinates of each B entry
  std::vector<uint32_t> if_pk;          // the same for each B^T entry (if_row order)
  // K_bb (lumped preconditioner) in wavefront groups of 64 touched DOFs
  // sorted by neighbour count: per lane slot the touched DOF (-1 past the
  // end) and its 27-neighbour mask of touched nodes; per group the value
  // offset, the block count and the subdomain; per subdomain its first group
  std::vector<int32_t> kbb_row;         // 64 per group
  std::vector<uint32_t> kbb_mask;       // 64 per group
  std::vector<int32_t> kbb_node;        // 64 per group: local node of the slot's DOF (0 past the end)
  std::vector<int64_t> kbb_goff;        // groups + 1
  std::vector<int32_t> kbb_gnb;         // groups
  std::vector<int32_t> kbb_gsub;        // groups
  std::vector<int32_t> kbb_g0;          // n_sub + 1
  // untorn maps
  std::vector<int64_t> g_first;         // n_gdof: torn index of the lowest-p copy
  std::vector<int32_t> g_rp;            // n_gdof + 1
  std::vector<int64_t> g_copies;        // torn indices of all copies
  std::vector<uint8_t> g_free;          // 1 if not Dirichlet
  // element colouring (2x2x2 parity classes share no node)
  std::vector<int32_t> colour_elems[8];
  std::vector<int32_t> elem_sub;
  // fixing nodes: rho-free regularization block Q Q^T (9x9) per subdomain
  std::vector<double> QQt;
  // strain-displacement matrices of the (uniform) element, weights
  double Bg[8][6][24];
  double wg;
  // load at factor 1, torn
  std::vector<double> f1;
  // coarse matrix G G^T in lower row-band form
  int32_t lc = 0, bc = 0, lc_pad = 0, Wc = 0;  // Wc: row stride of GGt_band
  std::vector<int32_t> cpos;            // coarse position of each subdomain: boxes in
                                        // lexicographic order, fewest boxes fastest
  std::vector<double> GGt_band;         // lc_pad rows of Wc
  // interface nodes of the learned warm start: nodes carrying multiplier rows
  int64_t n_wnodes = 0;
  std::vector<int32_t> wn_rows;         // n_wnodes * 21: row in slot 7 c + j, or -1
  std::vector<int8_t> wn_class;         // glue k = 2/4/8 -> 0/1/2, Dirichlet copies 1/2/4 -> 3/4/5
  std::vector<int32_t> wn_erp;          // n_wnodes + 1
  std::vector<int32_t> wn_elems;        // elements containing the node (all copies)
  double load_dir[3] = {0, 0, 0};       // traction of the loaded face at factor 1
  double load_area = 0.0;               // element face area of that face
  // Dirichlet preconditioner (Section 4.2): the interior nodes of each
  // subdomain (those carrying no row of B) form a box of the node lattice,
  // solved as a problem of its own
  std::vector<SubDev> isubs;            // n_sub; ndof 0 where no node is interior
  std::vector<int32_t> ilo;             // 3 per subdomain: first interior node per local axis
  int64_t n_int = 0;                    // interior DOFs of all subdomains
  std::string interior_error;           // non-empty: some interior is not a box
  int64_t iband_entries = 0;            // sum npad * Wb of the interior problems
  NbGroupsHost kit;                     // K_it: interior rows x touched neighbour nodes
  NbGroupsHost kti;                     // K_ti: touched rows x interior neighbour nodes
  // sizes
  int64_t band_entries = 0;             // sum npad * Wb
  int64_t skyline_entries = 0;          // sum of envelope widths of the factors
  std::vector<int64_t> skyline_sub;      // envelope entries of each subdomain's factor
};

// Build the host model; returns an empty string on success, else a message.
std::string build_model(const tfeti_problem& prob, HostModel& M);

// Assign panel offsets for tile TS; returns entries of one layout.
int64_t assign_panels(HostModel& M, int TS);
// The same for the interior problems of the Dirichlet preconditioner.
int64_t assign_interior_panels(HostModel& M, int TS);

}  // namespace tfeti

// mesh_prep.h -- host-side preparation of a (batch of) cloth sheet(s): rest
// geometry, hinges, block sparsity pattern, element-to-block maps, solver plan.
#pragma once

#include <string>
#include <vector>

namespace phisft {

constexpr int kMidSize = 16;  // vertices per aggregate of the middle level

struct HostSheet {
  int nv = 0, nt = 0;
  std::vector<int> tris;      // [nt][3]
  std::vector<double> rest;   // [nv][3]
  std::vector<int> pins;
  double mat[3] = {0, 0, 0};  // k_s, k_b, d
};

// Concatenated, validated layout (global indices). Field meaning as in Mesh.
struct HostLayout {
  int nv = 0, nt = 0, nh = 0, ninst = 0, maxnz = 0;
  std::vector<double> varea;
  std::vector<int> pinned, vert_inst, vinc_ptr, vinc_ref, ell_col, slot_ptr, slot_ref, diag_k;
  std::vector<int> tri_v;
  std::vector<double> tri_B, tri_area;
  std::vector<int> tri_inst;
  std::vector<int> hin_v;
  std::vector<double> hin_ce, hin_rest;
  std::vector<int> hin_inst;
  std::vector<int> inst_voff, inst_nv, inst_toff, inst_nt, inst_hoff, inst_nh;
  std::vector<double> mat;    // [ninst][3] create-time materials
  // anisotropic material frames: per triangle the strain measure tensors N_1..N_4 in its
  // local frame [12][nt] (N_00, N_01, N_11 each), per hinge the bending direction
  // weights of the 0, 45 and 90 degree tables [3][nh]
  std::vector<double> tri_N, hin_dw;
  // vertex order: internal index -> caller's (global) index
  std::vector<int> vold;
  // coarse space: aggregates are runs of consecutive internal vertices of one sheet
  int nagg = 0, max_nc = 0;
  std::vector<int> agg_v0;     // [nagg+1] first vertex
  std::vector<int> agg_inst;   // [nagg]
  std::vector<int> agg_modes;  // [nagg] 6 (rigid motions), 3 (translations) or 0
  std::vector<int> vert_agg;   // [nv]
  std::vector<int> inst_agg0, inst_nagg, inst_nc;  // [ninst]; nc = 6 * aggregates
  std::vector<int> inst_np;                         // [ninst] nc rounded up to 32 (stored size)
  std::vector<long long> inst_coff;                 // [ninst] offset of the dense np x np blocks
  long long coarse_doubles = 0;
  // aggregate pairs (a <= b, adjacent) and the matrix slots s = k*nv + i (i in a, col in b)
  std::vector<int> pair_a, pair_b, pair_ptr, pair_slot;
  // middle level: runs of kMidSize vertices from each sheet's start (compact 4x4 patches
  // of the grid sheets); the slots coupling two free vertices of the same run
  int nmid = 0;
  std::vector<int> mid_v0, mid_modes, mid_ptr, mid_slot, inst_mid0, vert_mid;
};

struct HostPlan {
  int rows = 0, nwg = 0, mat_home = 1, occ = 1;   // mat_home: MatrixHome
  int split = 0;   // register rows over two wavefront teams (SolverPlan::split)
  int barrier_slots = 0;   // root slots + group counter/flag slots
  std::vector<int> wg_inst, wg_row0, wg_nrows, inst_wg0, inst_nwg, inst_grp0;
  std::vector<int> group_wg0;  // solver launches: workgroup ranges of whole sheets
  // overlap of workgroup row ranges and aggregates (both are runs of vertices)
  int max_wg_agg = 0, max_agg_wg = 0;
  std::vector<int> wg_agg0, wg_nagg;   // [nwg] first aggregate touched, count
  std::vector<int> agg_wg0, agg_nwg;   // [nagg] first workgroup touching, count
  // neighbour rows owned by other workgroups (the halo) and the local column table:
  // lcol[k][i] = j - row0 for a column j of the workgroup's own rows, rows + h for the
  // h-th halo row, the row's own local index for a padding slot
  int max_halo = 0;
  std::vector<int> halo_ptr, halo_idx, lcol;
  // > 0: the solver keeps the FP32 rows of the coarse inverse that each workgroup
  // uses in LDS (6 x max_wg_agg x the largest coarse dimension floats)
  int xl_floats = 0;
};

// Splits the sheets (in order) into solver launches of at most `capacity`
// co-resident workgroups; false if one sheet alone exceeds it.
bool group_plan(HostPlan& P, int capacity, int max_groups);

// Returns 0 on success, -1 (invalid argument) or -2 (mesh error) with a message.
// Vertices of every sheet are renumbered by recursive coordinate bisection of the
// rest positions into compact runs of `agg_size` vertices (the aggregates of the
// coarse space; 0: no coarse space, runs of 64 still order the vertices). A sheet
// with more than max_aggs runs uses proportionally larger ones.
int build_layout(const std::vector<HostSheet>& sheets, int agg_size, int max_aggs,
                 HostLayout& out, std::string& err);

// Checks every index table against its bounds (run before any upload).
bool check_layout(const HostLayout& L, std::string& err);

HostPlan make_plan(const HostLayout& L, int rows, int group);

}  // namespace phisft

// sim_internal.h -- device-side data layout shared by the host runtime and the kernels.
//
// All per-instance arrays of a handle are concatenated (vertices, triangles,
// hinges) and indexed globally. Geometry is stored in FP64; the state
// trajectory, the assembled system matrix and its block-Jacobi inverse are
// stored in the handle's precision T (float or double); element intermediates
// and all solver vectors are FP64.
#pragma once

#include <cstdint>

namespace phisft {

// Sticky device status bits. A status array holds the handle-wide word at
// index 0 and one word per instance after it.
enum : int {
  ST_NOT_CONVERGED = 1,
  ST_INDEFINITE = 2,
  ST_NONFINITE = 4,
  ST_TIMEOUT = 8,  // a solver workgroup waited too long at a cluster barrier
};

// Element reference encodings (slot contributions and vertex incidences):
//   triangle block (t, a, b): t * 9 + a * 3 + b          (>= 0)
//   hinge block    (e, a, b): -(e * 16 + a * 4 + b) - 1   (< 0)
//   triangle vertex (t, a):   t * 3 + a                   (>= 0)
//   hinge vertex    (e, a):   -(e * 4 + a) - 1            (< 0)

// Anisotropic material (the Wang-style tables): four strain measures x six strain
// segments, three bending directions x five angle segments, then the density.
constexpr int kWangStretch = 24, kWangBend = 15, kWangParams = 40;

struct Mesh {
  int nv, nt, nh, ninst, maxnz;
  int tension;                  // 1: tension-clamped membrane block in K_sys, 0: exact Hessian
  int wang;                     // 1: anisotropic strain-dependent material
  int matn;                     // doubles per instance in the material arrays (3 or 40);
                                // the density is the last
  const double* tri_N;          // [12][nt] strain measure tensors (anisotropic material)
  const double* hin_dw;         // [3][nh]  bending direction weights (anisotropic)
  // vertices
  const double* varea;          // [nv] lumped area (a third of incident triangle areas)
  const int* pinned;            // [nv] 1 = Dirichlet vertex
  const int* vert_inst;         // [nv]
  const int* vinc_ptr;          // [nv+1] incident element vertices
  const int* vinc_ref;          // encoded (t,a) / (e,a)
  const int* ell_col;           // [maxnz][nv] block columns (padding: own row, zero block)
  const int* slot_ptr;          // [maxnz*nv+1] contributions of slot s = k*nv + i
  const int* slot_ref;          // encoded (t,a,b) / (e,a,b)
  const int* diag_k;            // [nv] slot index of the diagonal block
  // triangles
  const int* tri_v;             // [3][nt] global vertex ids (a, b, c), CCW
  const double* tri_B;          // [4][nt] inverse rest frame B = D_m^-1, row-major
  const double* tri_area;       // [nt] rest area
  const int* tri_inst;          // [nt]
  // hinges: edge (v0, v1), wings v2 (triangle v0 v1 v2) and v3 (triangle v1 v0 v3)
  const int* hin_v;             // [4][nh]
  const double* hin_ce;         // [nh] 3 |e|^2 / (A1 + A2)
  const double* hin_rest;       // [nh] rest dihedral angle
  const int* hin_inst;          // [nh]
  // instances
  const int* inst_voff;
  const int* inst_nv;
  const int* inst_toff;
  const int* inst_nt;
  const int* inst_hoff;
  const int* inst_nh;
  const int* vold;              // [nv] caller's index of each vertex (I/O arrays use it)
};

// Per-step element scratch (FP64).
struct Elem {
  double* tri_f;    // [9][nt]  force on (a, b, c)
  double* tri_K;    // [81][nt] system stiffness blocks (a,b) row-major 3x3
  double* hin_g;    // [12][nh] grad theta
  double* hin_f;    // [12][nh] bending force
  double* hin_w;    // [nh]     2 k_b c_e
  // adjoint
  double* tri_ag;   // [9][nt]  state-gradient contribution
  double* tri_ak;   // [9][nt]  K_sys mu contribution
  double* hin_ag;   // [12][nh]
  double* hin_ak;   // [12][nh]
  double* acc_ks;   // [nt] dL/dk_s partial sums over steps
  double* acc_kb;   // [nh]
  double* acc_d;    // [nv]
  double* acc_ws;   // [24][nt] anisotropic material: dL/dS partial sums
  double* acc_wb;   // [15][nh] dL/dB partial sums
  // wind (aerodynamic force of each triangle, used when the rollout has a wind)
  double* tri_fw;   // [3][nt]  a vertex's share (a third) of the triangle's wind force
  double* tri_wn;   // [4][nt]  unit normal n and c = 2 rho area |s| / 9: every 3x3 block
                    //          of the triangle's -df/dv is c n n^T
  double* tri_wv;   // [3][nt]  adjoint: each vertex's velocity-gradient term
  double* acc_w;    // [3][nt]  dL/dw partial sums over steps
};

// Coarse space of the two-level preconditioner M^-1 = B^-1 + P A_c^-1 P^T (B: the
// 3x3 block diagonal of A). An aggregate is a run of consecutive vertices of one
// sheet; its six modes are the rigid motions t + w x (x_i - c) about its centroid c
// at the step's positions (P_i = 0 on pinned vertices; an aggregate with fewer than
// three free, non-collinear vertices keeps translations only, one without free
// vertices keeps none). A_c = P^T A P is dense per sheet (nc = 6 x aggregates).
constexpr int kMaxWgAgg = 4;      // aggregates overlapping one solver workgroup
constexpr int kMaxAggWg = 4;      // solver workgroups overlapping one aggregate
constexpr int kGjTile = 32;       // tile of the blocked symmetric sweep (coarse inverse)
constexpr int kSwMaxTiles = 4;    // tiles one sweep workgroup holds in LDS at most
constexpr int kSwFlag = 32;       // ints between two sweep flags (one cache line each)
constexpr int kMid = 16;          // vertices per aggregate of the middle level

struct Coarse {
  int nagg;                    // 0: no coarse space
  int max_nc;
  int max_nb;                  // largest number of 32-tiles per side
  const int* agg_v0;           // [nagg+1]
  const int* agg_inst;         // [nagg]
  const int* agg_modes;        // [nagg] 6, 3 or 0
  const int* vert_agg;         // [nv]
  const int* inst_agg0;        // [ninst]
  const int* inst_nagg;        // [ninst]
  const int* inst_nc;          // [ninst] coarse dimension (6 x aggregates)
  const int* inst_np;          // [ninst] stored dimension: nc rounded up to 32 (identity pad)
  const long long* inst_coff;  // [ninst] offset of the sheet's np x np matrix
  int npair;
  const int* pair_a;           // [npair] aggregate pairs a <= b of one sheet
  const int* pair_b;
  const int* pair_ptr;         // [npair+1]
  const int* pair_slot;        // matrix slots k*nv + i, i in a, column in b
  // blocked symmetric sweep: workgroup w holds the tiles sw_ij[w * sw_tpw ..] (i * 65536
  // + j, i <= j, or -1) of sheet sw_inst[w]; sw_sync:
  // per sheet sw_stride ints (flags kSwFlag apart: pivot, then one per panel)
  int sw_tpw;
  int sw_stride;
  const int* sw_inst;
  const int* sw_ij;
  int* sw_sync;
  // solver-plan overlaps
  const int* wg_agg0;          // [nwg]
  const int* wg_nagg;          // [nwg]
  const int* agg_wg0;          // [nagg]
  const int* agg_nwg;          // [nagg]
  // per-step data
  double* crel;                // [3][nv] x_i - c (zero where the rotations are not used)
  double* mat;                 // A_c as assembled (FP64); the sweep reads its upper tiles
                               // once and keeps them in LDS
  float* xinv;                 // symmetrised FP32 copy of A_c^-1 read by the solver
  double* gj_c;                // per sheet (at inst_coff) [nb steps][nb][32][32] C_t = M_tK P
  double* gj_r;                // the same for the column panels D_t = M_tK
  double* gj_pinv;             // per sheet (at inst_boff) [nb steps][32][32] inverse pivots
  const long long* inst_boff;  // [ninst] offset of the sheet's inverse pivots (32 np)
  int* ok;                     // [ninst] 1 when this step's inversion succeeded
  double* part;                // [nwg][kMaxWgAgg][6] restriction partial sums
  // middle level: the six rigid motions of runs of kMid vertices, each with the
  // inverse of its own 6x6 diagonal block of P1^T A P1 (purely local to a workgroup)
  int nmid;
  const int* mid_v0;           // [nmid+1]
  const int* mid_modes;        // [nmid]
  const int* mid_ptr;          // [nmid+1] slots of the run's diagonal block
  const int* mid_slot;
  const int* vert_mid;         // [nv]
  double* mid_crel;            // [3][nv] x_i - centroid of the run (per step)
  double* mid_inv;             // [nmid][36] inverse diagonal blocks (per step)
};

// Cluster-barrier layout: counters 128 bytes apart; sheets with more than
// kBarrierGroup workgroups arrive in groups of that size.
constexpr int kBarrierSlot = 32;   // ints per counter slot
constexpr int kBarrierGroup = 32;

constexpr int kMaxSolverGroups = 64;

// Where the persistent solver keeps its workgroup's matrix rows during a solve:
// streamed from the assembled array in global memory at every product, copied once
// into LDS, or copied once into each row's lane registers (one workgroup per CU,
// rows of at most kRegRowBlocks blocks).
enum MatrixHome { kMatStream = 0, kMatLds = 1, kMatReg = 2 };

// Persistent solver launch description.
struct SolverPlan {
  int nwg;                 // workgroups over all solver groups
  int wg_base;             // first workgroup of the current launch
  int ngroups;             // launches per solve: sets of whole sheets that fit co-resident
  int group_wg0_host[kMaxSolverGroups + 1];  // workgroup ranges of the groups
  int mat_home;            // where the solver reads the matrix rows: MatrixHome
  int occ;                 // 1 or 2 workgroups of 256 threads per CU (kernel variant)
  int split;               // 1: register rows over two wavefront teams (rows <= 128)
  int rows;                // rows per workgroup (LDS stride; block = rows rounded up to 64)
  const int* wg_inst;      // [nwg]
  const int* wg_row0;      // [nwg]
  const int* wg_nrows;     // [nwg]
  const int* inst_wg0;     // [ninst]
  const int* inst_nwg;     // [ninst]
  const int* inst_grp0;    // [ninst] first group slot (counter, flag pairs) of the sheet
  int max_halo;            // largest halo (neighbour rows of other workgroups)
  const int* halo_ptr;     // [nwg+1]
  const int* halo_idx;     // halo rows of each workgroup (global vertex ids)
  const int* lcol;         // [maxnz][nv] local columns: own row j - row0, halo rows + h
  int xl_floats;           // > 0: LDS floats holding the rows of the coarse inverse that
                           // a workgroup uses (6 x its aggregates x the coarse dimension);
                           // 0: those rows are read from global memory every iteration
};

// Solver scratch (device).
// tagged partials of one workgroup: 3 dot products, then 6 per overlapped aggregate
constexpr int kTagSlots = 3 + 6 * kMaxWgAgg;

struct SolverWork {
  double* zbuf;            // [3][nv]     preconditioned initial residual, gathered once
  double* pbuf;            // [2][3][nv]  m = M^-1 w of even / odd iterations
  unsigned long long* tbuf;  // [2][4][nv] the same, published as tagged 64-bit words
                             // (tag << 32 | 32 data bits), zeroed before each launch
  double* red;             // [2][nwg][3] per-workgroup partial sums
  unsigned long long* tred;  // [2][nwg][kTagSlots][2] the same and the coarse restriction
                             // partials as tagged words (coarse space), zeroed per launch
  int* barrier;            // counter slots: [ninst] roots, then group counter/flag pairs
  int barrier_ints;        // ints to zero before each launch
  int tred_ints;           // ints of tred
  int* abort_flag;         // [1]
};

}  // namespace phisft

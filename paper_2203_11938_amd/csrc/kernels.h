// kernels.h -- launchers of the gfx950 kernels (definitions in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "sim_internal.h"

namespace phisft {

template <typename T, typename TM>
struct AssembleArgs {
  const double* v;     // [3][nv] velocity v_{t-1} (zero on pins)
  const T* forces;     // [3][nv] corrective forces of the step, or nullptr
  const double* mat;   // [ninst][3] (k_s, k_b, d)
  double h;
  double g[3];
  int want_rhs;        // 0: matrix and preconditioner only (adjoint re-assembly)
  int wind;            // 1: add the elements' wind force and damping blocks (h D)
  TM* A;               // [maxnz][9][nv]
  TM* Jinv;            // [9][nv]
  double* b;           // [3][nv]
  int* status;
};

template <typename TM>
struct PcgArgs {
  const TM* A;
  const TM* Jinv;
  const double* rhs;   // [3][nv]
  double* sol;         // [3][nv]
  double tol;
  int max_iter;
  int* iters;          // [ninst] or nullptr
  double* resid;       // [ninst] or nullptr
  int* status;
};

template <typename T>
struct AdjArgs {
  const double* x;     // x_{s-1}
  const double* vp;    // v_{s-1}
  const double* vs;    // v_s
  const double* mu;    // adjoint solution of step s
  const double* u;     // its right-hand side
  const double* mat;
  double h;
  double g[3];
  double* gx;          // [3][nv] running dL/dx
  double* gv;          // [3][nv] running dL/dv
  T* dl_dF;            // [3][nv] slice of dL/dF for step s, or nullptr
  const double* wind;  // [ninst][3] wind velocity, or nullptr (no aerodynamic force)
  double rho;          // air density
};

void launch_fill_int(int* p, int n, int v, hipStream_t st);
void launch_fill_double(double* p, long n, double v, hipStream_t st);

// Element pass at (x, v): forces and stiffness blocks, and with a wind velocity
// (wind != nullptr, [ninst][3]) the triangles' aerodynamic force and damping blocks.
void launch_elements(const Mesh& m, const Elem& el, const double* x, const double* v,
                     const double* mat, const double* wind, double rho, int* status,
                     hipStream_t st);
template <typename T, typename TM>
void launch_assemble(const Mesh& m, const Elem& el, const AssembleArgs<T, TM>& a, hipStream_t st);
template <typename TM>
size_t pcg_lds_bytes(int maxnz, int rows, int mat_home, int coarse_nc, int max_halo,
                     int xl_floats);
// threads of a solver block: its rows rounded up to whole 64-lane wavefronts
inline int pcg_threads(int rows) { return (rows + 63) / 64 * 64; }
// Rows may couple at most this many vertices (grid sheets: 13).
constexpr int kMaxRowBlocks = 32;
// Rows of at most this many blocks can hold them in registers (kMatReg).
constexpr int kRegRowBlocks = 13;
// Every product A v sums a row's slots [0, kSpmvSplit) and [kSpmvSplit, maxnz)
// separately and then adds the two (all matrix homes, so they agree bit for bit).
// Register-resident rows in workgroups of at most kSplitRows rows may run twice the
// wavefronts (SolverPlan::split): the second half holds and multiplies the rows'
// second slot range.
constexpr int kSpmvSplit = 7;
constexpr int kSplitRows = 128;
inline bool pcg_can_split(int rows, int mat_home) {
  return mat_home == kMatReg && pcg_threads(rows) <= kSplitRows;
}
// threads of a solver launch's workgroup
inline int pcg_block(int rows, bool split) {
  return split ? 2 * pcg_threads(rows) : pcg_threads(rows);
}
template <typename TM>
hipError_t pcg_prepare(size_t lds, int maxnz, int mat_home, bool coarse, int occ);
template <typename TM>
hipError_t pcg_occupancy(int rows, size_t lds, int maxnz, int mat_home, bool coarse, int occ,
                         bool split, int* blocks_per_cu);
template <typename TM>
void launch_pcg(const Mesh& m, const SolverPlan& plan, const SolverWork& w, const Coarse& cs,
                const PcgArgs<TM>& a, hipStream_t st);
// Coarse operator of the step at positions x and assembled matrix A: frames,
// Galerkin product and its in-place blocked symmetric sweep (one launch per group of
// sheets; sweep_groups: first workgroup of each group, then the total). No-op without
// a coarse space.
template <typename TM>
void launch_coarse_setup(const Mesh& m, const Coarse& c, const double* x, const TM* A,
                         long long coarse_doubles, const std::vector<int>& sweep_groups,
                         hipStream_t st);
// Dynamic LDS of the sweep kernel and its co-resident workgroups per CU for a given
// number of tiles held per workgroup.
size_t gj_sweep_lds(int tiles_per_wg);
hipError_t gj_sweep_occupancy(int tiles_per_wg, int* blocks_per_cu);
// Caller-layout arrays (x0, v0, x_out, dL/dx) are indexed through m.vold.
template <typename T>
void launch_update(const Mesh& m, const double* xp, const double* vp, const double* dv, double h,
                   double* xn, double* vn, T* xout, int* status, hipStream_t st);
template <typename T>
void launch_init_state(const Mesh& m, const T* x0, const T* v0, double* xs, double* vs,
                       int* status, hipStream_t st);
template <typename T>
void launch_adj_pre(const Mesh& m, const T* dl, double h, double* gx, const double* gv, double* u,
                    int* status, hipStream_t st);
template <typename T>
void launch_adj_elements(const Mesh& m, const Elem& el, const AdjArgs<T>& a, hipStream_t st);
template <typename T>
void launch_adj_rows(const Mesh& m, const Elem& el, const AdjArgs<T>& a, hipStream_t st);
template <typename T>
void launch_adj_final(const Mesh& m, const double* gx, const double* gv, T* dx0, T* dv0,
                      hipStream_t st);
// Per-sheet sums of the material (out_mat [ninst][3]) and wind (out_wind [ninst][3])
// gradient partials; either output may be nullptr.
void launch_material_sum(const Mesh& m, const Elem& el, double* out_mat, double* out_wind,
                         hipStream_t st);

// Per loss frame and sheet: E = sum over the sheet's vertices of |x - target|^2 (FP64,
// fixed order) into energy [nframes][ninst], and dl = 2 (x - target) when dl != nullptr.
// Arrays [nframes][3][nv] in the caller's vertex order; voff/vcount: device [ninst].
template <typename T>
void launch_frame_loss(const T* x, const T* tgt, int nv, const int* voff, const int* vcount,
                       int ninst, int nframes, double* energy, T* dl, hipStream_t st);

// Bytes of the static device array behind the allocation-free rollout's solver
// exchange buffers (one copy per GPU, held for the process's lifetime).
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
// Device address of that array on the current device (looked up once per device).
hipError_t noalloc_scratch(void** out);

}  // namespace phisft

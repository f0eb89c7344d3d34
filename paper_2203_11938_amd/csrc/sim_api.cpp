// sim_api.cpp -- the C ABI (include/phisft_sim.h): handles, workspace, and the
// step sequencing of rollout and adjoint on the caller's HIP stream.
//
// Rollout: for s = 1..n, one linearised backward-Euler step (Sec. 3.1, Eq. 4-5):
// element pass, row assembly, persistent PCG, update. States are kept either
// for every step or every k-th step (checkpoints); the adjoint walks the steps
// backwards (implicit differentiation of Eq. 4), recomputing each checkpoint
// segment forward first when checkpoints are used. The recomputation runs the
// same kernels on the same inputs, so it reproduces the forward states bitwise.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/phisft_sim.h"
#include "kernels.h"
#include "mesh_prep.h"
#include "sim_internal.h"

using namespace phisft;

static_assert(kMid == kMidSize, "device and host sizes of the middle level differ");
static_assert(kMatStream + 1 == SIM_MATRIX_STREAMED && kMatLds + 1 == SIM_MATRIX_LDS &&
                  kMatReg + 1 == SIM_MATRIX_REGISTERS,
              "solver matrix homes and their public values differ");

struct sim_s {
  HostLayout L;
  HostPlan plan_h;
  int prec = SIM_FP32;   // caller arrays
  int mprec = SIM_FP64;  // system matrix and block-Jacobi inverse
  size_t tsize = 4;
  size_t msize = 8;
  double h = 0.01;
  double grav[3] = {0.0, 0.0, -9.81};
  double cg_tol = 1e-7;
  int cg_max_iter = 20000;
  int ckpt = 0;
  int max_steps = 0;
  double rho_air = 1.0;      // air density of the aerodynamic force
  bool coarse_keep_all = false;

  std::vector<void*> allocs;
  size_t dev_bytes = 0;      // device memory held by the handle
  Mesh mesh{};
  Elem el{};
  SolverPlan plan{};
  SolverWork sw{};
  Coarse coarse{};
  long long gj_doubles = 0;               // per-sheet [np][32] blocks of the inversion
  // per-step coarse operators kept for the adjoint (inverse, offsets, flags); slot of
  // step s: s - 1 (every state stored) or (s - 1) % k (checkpoints every k)
  int cslots = 0;
  float* cmat_store = nullptr;
  double* crel_store = nullptr;
  int* cok_store = nullptr;
  double* mrel_store = nullptr;
  double* minv_store = nullptr;
  std::vector<int> slot_step;             // step held by each slot, 0 = none
  std::vector<int> sweep_groups;          // first sweep workgroup of each launch, then total
  void* A = nullptr;
  void* Jinv = nullptr;
  double* rhs = nullptr;
  double* sol = nullptr;
  double* mat_default = nullptr;
  double* gx = nullptr;
  double* gv = nullptr;
  int* status = nullptr;
  int* it_fwd = nullptr;   // [max_steps][ninst]
  int* it_rec = nullptr;
  int* it_adj = nullptr;
  double* res_fwd = nullptr;
  double* res_adj = nullptr;
  double* res_rec = nullptr;
  // state storage: each state is x [3][nv] followed by v [3][nv]
  void* traj = nullptr;    // store-all: max_steps + 1 states
  void* ckpts = nullptr;   // checkpoints: max_steps / k + 1 states
  void* tmp = nullptr;     // checkpoints: 2 rolling states + 1 final
  void* seg = nullptr;     // checkpoints: k recomputed states

  // most recent rollout
  bool have_rollout = false;
  bool have_adjoint = false;   // an adjoint ran since that rollout (its statistics count)
  int n_steps = 0;
  std::vector<int> frames;
  const void* forces = nullptr;
  const double* material = nullptr;
  const double* wind = nullptr;   // [ninst][3] wind velocity, or nullptr: no aerodynamic force
  hipStream_t stream = nullptr;

  // HIP graphs of the last rollout and adjoint (graph option): replayed when a call
  // repeats the captured arguments
  struct GraphCache {
    bool valid = false;
    std::vector<uintptr_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int> slot_after;   // host slot bookkeeping after the captured call
  };
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  GraphCache gfwd, gadj;
  long long graph_captures = 0, graph_replays = 0;

  sim_stats stats{};
  std::vector<int> inst_status;
  // solver timing: event pairs recorded around each solver launch
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  std::string err;
};

namespace {

// aggregates per sheet at most (coarse dimension 6 x 320 = 1920): beyond it the dense
// coarse inverse costs more per step and per iteration than its fewer iterations save
constexpr int kCoarseMaxAggs = 320;
// device memory for coarse operators kept between the forward pass and the adjoint
constexpr double kCoarseStoreCap = 16.0 * (1 << 30);

sim_status bits_to_status(int bits) {
  if (bits & ST_TIMEOUT) return SIM_E_HIP;
  if (bits & ST_NONFINITE) return SIM_E_NONFINITE;
  if (bits & ST_INDEFINITE) return SIM_E_INDEFINITE;
  if (bits & ST_NOT_CONVERGED) return SIM_E_NOT_CONVERGED;
  return SIM_OK;
}

sim_status hip_fail(sim_t* s, hipError_t e, const char* where) {
  if (s) s->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? SIM_E_NOMEM : SIM_E_HIP;
}

#define HIPCHECK(s, call)                                \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail((s), e_, #call); \
  } while (0)

template <typename V>
sim_status upload(sim_t* s, const std::vector<V>& h, const V** out) {
  void* d = nullptr;
  size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(V);
  HIPCHECK(s, hipMalloc(&d, bytes));
  s->allocs.push_back(d);
  s->dev_bytes += bytes;
  if (!h.empty()) HIPCHECK(s, hipMemcpy(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  *out = static_cast<const V*>(d);
  return SIM_OK;
}

sim_status alloc(sim_t* s, size_t bytes, void** out) {
  void* d = nullptr;
  HIPCHECK(s, hipMalloc(&d, std::max<size_t>(bytes, 8)));
  s->allocs.push_back(d);
  s->dev_bytes += std::max<size_t>(bytes, 8);
  *out = d;
  return SIM_OK;
}

#define TRY(x)                      \
  do {                              \
    sim_status st_ = (x);           \
    if (st_ != SIM_OK) return st_;  \
  } while (0)

// states are FP64 in every precision mode: x [3][nv] then v [3][nv]
size_t state_bytes(const sim_t* s) { return 6 * (size_t)s->L.nv * sizeof(double); }

char* state_at(void* base, const sim_t* s, long k) {
  return static_cast<char*>(base) + (size_t)k * state_bytes(s);
}

// State of step index k (0..n) during the forward pass of an n-step rollout.
char* fwd_state(sim_t* s, int k, int n) {
  if (s->ckpt == 0) return state_at(s->traj, s, k);
  if (k % s->ckpt == 0) return state_at(s->ckpts, s, k / s->ckpt);
  if (k == n) return state_at(s->tmp, s, 2);
  return state_at(s->tmp, s, k % 2);
}

// State of step index k during the adjoint sweep over the segment that starts at c0.
char* adj_state(sim_t* s, int k, int c0, int n) {
  if (s->ckpt == 0) return state_at(s->traj, s, k);
  if (k % s->ckpt == 0) return state_at(s->ckpts, s, k / s->ckpt);
  if (k == n) return state_at(s->tmp, s, 2);
  return state_at(s->seg, s, k - c0);
}

// Uploads a solver plan's tables and (re)allocates its plan-sized buffers.
sim_status apply_plan(sim_t* s, const HostPlan& P) {
  const HostLayout& L = s->L;
  const bool coarse = L.nagg > 0;
  SolverPlan& p = s->plan;
  p.nwg = P.nwg;
  p.rows = P.rows;
  p.mat_home = P.mat_home;
  p.occ = P.occ;
  p.split = P.split;
  p.wg_base = 0;
  p.ngroups = (int)P.group_wg0.size() - 1;
  for (int g = 0; g <= p.ngroups; ++g) p.group_wg0_host[g] = P.group_wg0[g];
  TRY(upload(s, P.inst_grp0, &p.inst_grp0));
  TRY(upload(s, P.wg_inst, &p.wg_inst));
  TRY(upload(s, P.wg_row0, &p.wg_row0));
  TRY(upload(s, P.wg_nrows, &p.wg_nrows));
  TRY(upload(s, P.inst_wg0, &p.inst_wg0));
  TRY(upload(s, P.inst_nwg, &p.inst_nwg));
  p.max_halo = P.max_halo;
  p.xl_floats = coarse ? P.xl_floats : 0;
  TRY(upload(s, P.halo_ptr, &p.halo_ptr));
  TRY(upload(s, P.halo_idx, &p.halo_idx));
  TRY(upload(s, P.lcol, &p.lcol));
  void* q = nullptr;
  TRY(alloc(s, 6 * (size_t)p.nwg * 8, &q));
  s->sw.red = (double*)q;
  TRY(alloc(s, 2 * (size_t)p.nwg * kTagSlots * 16, &q));
  s->sw.tred = (unsigned long long*)q;
  s->sw.tred_ints = 2 * p.nwg * kTagSlots * 4;
  s->sw.barrier_ints = P.barrier_slots * kBarrierSlot;
  TRY(alloc(s, (size_t)s->sw.barrier_ints * 4, &q));
  s->sw.barrier = (int*)q;
  if (coarse) {
    Coarse& cs = s->coarse;
    TRY(upload(s, P.wg_agg0, &cs.wg_agg0));
    TRY(upload(s, P.wg_nagg, &cs.wg_nagg));
    TRY(upload(s, P.agg_wg0, &cs.agg_wg0));
    TRY(upload(s, P.agg_nwg, &cs.agg_nwg));
    TRY(alloc(s, (size_t)p.nwg * kMaxWgAgg * 6 * 8, &q));
    cs.part = (double*)q;
  }
  const int lm = P.mat_home;
  const int cnc = coarse ? L.max_nc : 0;
  hipError_t e = s->mprec == SIM_FP64
      ? pcg_prepare<double>(pcg_lds_bytes<double>(L.maxnz, P.rows, lm, cnc, P.max_halo, P.xl_floats),
                            L.maxnz, lm, coarse, P.occ)
      : pcg_prepare<float>(pcg_lds_bytes<float>(L.maxnz, P.rows, lm, cnc, P.max_halo, P.xl_floats),
                           L.maxnz, lm, coarse, P.occ);
  if (e != hipSuccess) return hip_fail(s, e, "solver LDS attribute");
  s->plan_h = P;
  s->stats.rows_per_block = p.rows;
  s->stats.blocks = p.nwg;
  s->stats.solver_matrix_home = p.mat_home + 1;   // MatrixHome -> sim_matrix_home
  s->stats.solver_wg_per_cu = p.occ;
  s->stats.solver_row_teams = p.split ? 2 : 1;
  s->stats.coarse_rows_lds = p.xl_floats > 0 ? 1 : 0;
  s->stats.solver_launches_per_solve = p.ngroups;
  return SIM_OK;
}

// Measuring autotuner: builds the step system of the rest state (the sheets at rest,
// zero velocity, gravity) with the real kernels, then times kTuneIters PCG
// iterations of every feasible launch shape and keeps the fastest.
constexpr int kTuneIters = 40;

template <typename TM>
sim_status autotune(sim_t* s, const std::vector<HostPlan>& cands, const std::vector<double>& xr,
                    int* pick) {
  const int nv = s->L.nv;
  void* q = nullptr;
  TRY(alloc(s, 3 * (size_t)nv * 8, &q));
  double* x = (double*)q;
  HIPCHECK(s, hipMemcpy(x, xr.data(), 3 * (size_t)nv * 8, hipMemcpyHostToDevice));
  hipStream_t st = nullptr;
  launch_fill_double(s->gv, 3L * nv, 0.0, st);
  launch_elements(s->mesh, s->el, x, s->gv, s->mat_default, nullptr, 0.0, s->status, st);
  AssembleArgs<double, TM> a{};
  a.v = s->gv;
  a.forces = nullptr;
  a.mat = s->mat_default;
  a.h = s->h;
  for (int k = 0; k < 3; ++k) a.g[k] = s->grav[k];
  a.want_rhs = 1;
  a.A = static_cast<TM*>(s->A);
  a.Jinv = static_cast<TM*>(s->Jinv);
  a.b = s->rhs;
  a.status = s->status;
  launch_assemble<double, TM>(s->mesh, s->el, a, st);
  launch_coarse_setup<TM>(s->mesh, s->coarse, x, a.A, s->L.coarse_doubles, s->sweep_groups, st);
  PcgArgs<TM> c{};
  c.A = a.A;
  c.Jinv = a.Jinv;
  c.rhs = s->rhs;
  c.sol = s->sol;
  c.tol = 0.0;  // never met: every trial runs kTuneIters iterations
  c.max_iter = kTuneIters;
  c.status = s->status;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(s, hipEventCreate(&e0));
  HIPCHECK(s, hipEventCreate(&e1));
  float best_ms = 1e30f;
  for (size_t k = 0; k < cands.size(); ++k) {
    TRY(apply_plan(s, cands[k]));
    launch_pcg<TM>(s->mesh, s->plan, s->sw, s->coarse, c, st);  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 3; ++r) launch_pcg<TM>(s->mesh, s->plan, s->sw, s->coarse, c, st);
    (void)hipEventRecord(e1, st);
    HIPCHECK(s, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHECK(s, hipEventElapsedTime(&ms, e0, e1));
    int bits = 0;
    HIPCHECK(s, hipMemcpy(&bits, s->status, 4, hipMemcpyDeviceToHost));
    // a trial stops at kTuneIters (not converged by design); any other condition
    // disqualifies the candidate
    if ((bits & ~ST_NOT_CONVERGED) == 0 && ms < best_ms) {
      best_ms = ms;
      *pick = (int)k;
    }
    HIPCHECK(s, hipMemset(s->status, 0, 4 * (s->L.ninst + 1)));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->stats.autotune_ms_per_iter = best_ms / (3.0 * kTuneIters);
  return SIM_OK;
}

sim_status setup(sim_t* s, const std::vector<HostSheet>& sheets, double dt, const sim_options* opt) {
  sim_options o;
  sim_default_options(&o);
  if (opt) o = *opt;
  if (!(dt > 0.0) || !std::isfinite(dt)) {
    s->err = "dt must be positive";
    return SIM_E_INVALID;
  }
  if ((o.precision != SIM_FP32 && o.precision != SIM_FP64) || !(o.cg_tol > 0.0) ||
      o.cg_max_iter < 1 || o.checkpoint_every < 0 || o.max_steps < 1 ||
      !(o.rows_per_block == 0 ||
        (o.rows_per_block >= 64 && o.rows_per_block <= 256 && o.rows_per_block % 16 == 0)) ||
      (o.membrane_system != SIM_MEMBRANE_EXACT && o.membrane_system != SIM_MEMBRANE_TENSION) ||
      (o.matrix_precision != SIM_FP32 && o.matrix_precision != SIM_FP64) ||
      !(o.coarse_size == 0 || (o.coarse_size >= 16 && o.coarse_size <= (1 << 20))) ||
      (o.autotune != 0 && o.autotune != 1) || (o.graph != 0 && o.graph != 1) ||
      o.matrix_home < SIM_MATRIX_AUTO || o.matrix_home > SIM_MATRIX_REGISTERS ||
      !(o.air_density >= 0.0) || !std::isfinite(o.air_density) ||
      (o.coarse_keep_all != 0 && o.coarse_keep_all != 1) ||
      (o.material_model != SIM_MATERIAL_ISOTROPIC && o.material_model != SIM_MATERIAL_WANG) ||
      (o.material_model == SIM_MATERIAL_WANG && o.membrane_system == SIM_MEMBRANE_TENSION)) {
    s->err = "invalid options";
    return SIM_E_INVALID;
  }
  s->prec = o.precision;
  s->use_graph = o.graph != 0;
  s->tsize = o.precision == SIM_FP64 ? 8 : 4;
  s->mprec = o.matrix_precision;
  s->msize = o.matrix_precision == SIM_FP64 ? 8 : 4;
  s->h = dt;
  for (int k = 0; k < 3; ++k) s->grav[k] = o.gravity[k];
  s->cg_tol = o.cg_tol;
  s->cg_max_iter = o.cg_max_iter;
  s->ckpt = o.checkpoint_every;
  s->max_steps = o.max_steps;
  s->rho_air = o.air_density;
  s->coarse_keep_all = o.coarse_keep_all != 0;

  int rc = build_layout(sheets, o.coarse_size, kCoarseMaxAggs, s->L, s->err);
  if (rc != 0) return rc == -1 ? SIM_E_INVALID : SIM_E_MESH;
  if (!check_layout(s->L, s->err)) return SIM_E_MESH;
  HostLayout& L = s->L;
  if (L.maxnz > kMaxRowBlocks) {
    s->err = "a vertex couples to more than 32 vertices (valence too high for the solver)";
    return SIM_E_MESH;
  }

  // solver launch shape: rows per workgroup bounded by the LDS budget and co-residency
  int dev = 0, ncu = 0;
  HIPCHECK(s, hipGetDevice(&dev));
  HIPCHECK(s, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const bool coarse = L.nagg > 0;
  // dynamic LDS budget: 160 KB less the kernel's static buffers
  const size_t lds_cap = 160 * 1024 - (coarse ? 4096 : 1024);
  // Largest feasible block first (fewer workgroups meet faster at the per-iteration
  // barrier); matrix rows in registers (rows of at most kRegRowBlocks blocks, one
  // workgroup per CU), in LDS when they fit, else streamed from global memory.
  // A plan needing fewer solver launches wins; then that order of homes; then larger
  // blocks.
  std::vector<int> cands;
  if (o.rows_per_block) cands.push_back(o.rows_per_block);
  else cands = {256, 224, 192, 160, 152, 128, 96, 64};
  std::vector<HostPlan> feasible;
  int best = -1, best_groups = 1 << 30;
  for (int mode : {kMatReg, kMatLds, kMatStream}) {
    if (o.matrix_home != SIM_MATRIX_AUTO && mode != o.matrix_home - 1) continue;
    if (mode == kMatReg && L.maxnz > kRegRowBlocks) continue;
    for (int rows : cands) {
      const bool m64 = s->mprec == SIM_FP64;
      const int lm = mode;
      const int cnc = coarse ? L.max_nc : 0;
      if (L.nmid > 0 && rows % kMidSize != 0) continue;  // workgroups hold whole runs
      HostPlan P0 = make_plan(L, rows, kBarrierGroup);
      P0.mat_home = mode;
      if (P0.max_wg_agg > kMaxWgAgg || P0.max_agg_wg > kMaxAggWg) continue;
      // the rows of the coarse inverse in LDS as well (when that fits), or streamed
      const int xl_full = coarse ? 6 * P0.max_wg_agg * L.max_nc : 0;
      for (int xl : {xl_full, 0}) {
        const size_t lds = m64 ? pcg_lds_bytes<double>(L.maxnz, rows, lm, cnc, P0.max_halo, xl)
                               : pcg_lds_bytes<float>(L.maxnz, rows, lm, cnc, P0.max_halo, xl);
        if (lds > lds_cap) continue;
        // the one-workgroup-per-CU variant, and the two-per-CU one where it adds
        // co-resident workgroups; register rows of small workgroups also over two
        // wavefront teams (tried first: equal launch counts then prefer it)
        int prev_cap = 0;
        const int nvar = mode == kMatReg ? (pcg_can_split(rows, mode) ? 2 : 1) : 2;
        for (int var = 0; var < nvar; ++var) {
          const int occ = mode == kMatReg ? 1 : var + 1;
          const bool split = mode == kMatReg && nvar == 2 && var == 0;
          // split teams hand their second products over in 6 KB of static LDS
          if (split && lds + 6 * kSplitRows * sizeof(double) > lds_cap) continue;
          HostPlan P = P0;
          P.xl_floats = xl;
          P.occ = occ;
          P.split = split ? 1 : 0;
          hipError_t e = m64 ? pcg_prepare<double>(lds, L.maxnz, lm, coarse, occ)
                             : pcg_prepare<float>(lds, L.maxnz, lm, coarse, occ);
          if (e != hipSuccess) return hip_fail(s, e, "solver LDS attribute");
          int per_cu = 0;
          e = m64 ? pcg_occupancy<double>(rows, lds, L.maxnz, lm, coarse, occ, split, &per_cu)
                  : pcg_occupancy<float>(rows, lds, L.maxnz, lm, coarse, occ, split, &per_cu);
          if (e != hipSuccess) return hip_fail(s, e, "solver occupancy");
          if (occ == 2 && per_cu <= prev_cap) continue;
          prev_cap = per_cu;
          if (!group_plan(P, per_cu * ncu, kMaxSolverGroups)) continue;
          const int ng = (int)P.group_wg0.size() - 1;
          feasible.push_back(P);
          if (ng < best_groups) {
            best = (int)feasible.size() - 1;
            best_groups = ng;
          }
        }
        if (xl_full == 0) break;   // both options are the same plan
      }
    }
  }
  if (best < 0) {
    s->err = o.matrix_home != SIM_MATRIX_AUTO
                 ? "no co-resident solver launch shape keeps the matrix where requested"
                 : o.rows_per_block != 0
                       ? "no co-resident solver launch shape with the requested rows per workgroup "
                         "(a workgroup may overlap at most 4 coarse aggregates, an aggregate at "
                         "most 4 workgroups)"
                       : "mesh too large for the co-resident solver";
    return SIM_E_INVALID;
  }

  // ---- upload geometry and tables
  Mesh& m = s->mesh;
  m.nv = L.nv;
  m.nt = L.nt;
  m.nh = L.nh;
  m.ninst = L.ninst;
  m.maxnz = L.maxnz;
  m.tension = o.membrane_system == SIM_MEMBRANE_TENSION ? 1 : 0;
  m.wang = o.material_model == SIM_MATERIAL_WANG ? 1 : 0;
  m.matn = m.wang ? kWangParams : 3;
  s->stats.material_params = m.matn;
  TRY(upload(s, L.varea, &m.varea));
  TRY(upload(s, L.pinned, &m.pinned));
  TRY(upload(s, L.vert_inst, &m.vert_inst));
  TRY(upload(s, L.vinc_ptr, &m.vinc_ptr));
  TRY(upload(s, L.vinc_ref, &m.vinc_ref));
  TRY(upload(s, L.ell_col, &m.ell_col));
  TRY(upload(s, L.slot_ptr, &m.slot_ptr));
  TRY(upload(s, L.slot_ref, &m.slot_ref));
  TRY(upload(s, L.diag_k, &m.diag_k));
  TRY(upload(s, L.tri_v, &m.tri_v));
  TRY(upload(s, L.tri_B, &m.tri_B));
  TRY(upload(s, L.tri_area, &m.tri_area));
  TRY(upload(s, L.tri_inst, &m.tri_inst));
  TRY(upload(s, L.hin_v, &m.hin_v));
  TRY(upload(s, L.hin_ce, &m.hin_ce));
  TRY(upload(s, L.hin_rest, &m.hin_rest));
  TRY(upload(s, L.hin_inst, &m.hin_inst));
  TRY(upload(s, L.inst_voff, &m.inst_voff));
  TRY(upload(s, L.inst_nv, &m.inst_nv));
  TRY(upload(s, L.inst_toff, &m.inst_toff));
  TRY(upload(s, L.inst_nt, &m.inst_nt));
  TRY(upload(s, L.inst_hoff, &m.inst_hoff));
  TRY(upload(s, L.inst_nh, &m.inst_nh));
  TRY(upload(s, L.vold, &m.vold));
  const double* md = nullptr;
  if (m.wang) {
    // the create-time (k_s, k_b, d) as anisotropic tables that reproduce the isotropic
    // model: warp, weft and shear at k_s, no area term, every bend entry k_b
    std::vector<double> wm;
    for (int b = 0; b < L.ninst; ++b) {
      for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 6; ++j) wm.push_back(k < 3 ? L.mat[3 * b] : 0.0);
      for (int j = 0; j < kWangBend; ++j) wm.push_back(L.mat[3 * b + 1]);
      wm.push_back(L.mat[3 * b + 2]);
    }
    TRY(upload(s, wm, &md));
    TRY(upload(s, L.tri_N, &m.tri_N));
    TRY(upload(s, L.hin_dw, &m.hin_dw));
  } else {
    TRY(upload(s, L.mat, &md));
    m.tri_N = m.hin_dw = nullptr;
  }
  s->mat_default = const_cast<double*>(md);

  // ---- coarse space
  Coarse& cs = s->coarse;
  cs.nagg = L.nagg;
  cs.max_nc = L.max_nc;
  if (coarse) {
    TRY(upload(s, L.agg_v0, &cs.agg_v0));
    TRY(upload(s, L.agg_inst, &cs.agg_inst));
    TRY(upload(s, L.agg_modes, &cs.agg_modes));
    TRY(upload(s, L.vert_agg, &cs.vert_agg));
    TRY(upload(s, L.inst_agg0, &cs.inst_agg0));
    TRY(upload(s, L.inst_nagg, &cs.inst_nagg));
    TRY(upload(s, L.inst_nc, &cs.inst_nc));
    TRY(upload(s, L.inst_coff, &cs.inst_coff));
    cs.npair = (int)L.pair_a.size();
    TRY(upload(s, L.pair_a, &cs.pair_a));
    TRY(upload(s, L.pair_b, &cs.pair_b));
    TRY(upload(s, L.pair_ptr, &cs.pair_ptr));
    TRY(upload(s, L.pair_slot, &cs.pair_slot));
    TRY(upload(s, L.inst_np, &cs.inst_np));
    // blocked symmetric sweep: the upper tiles of each sheet spread over co-resident
    // workgroups (tile e of a sheet in row order -> workgroup e mod n, slot e / n), the
    // fewest tiles per workgroup with which the largest sheet fits one launch; sheets
    // grouped into launches of co-resident workgroups
    int max_nb = 0;
    for (int b = 0; b < L.ninst; ++b) max_nb = std::max(max_nb, L.inst_np[b] / kGjTile);
    cs.max_nb = max_nb;
    int tpw = 0, cap = 0;
    const long long most_tiles = (long long)max_nb * (max_nb + 1) / 2;
    for (int t = 1; t <= kSwMaxTiles && tpw == 0; ++t) {
      int per_cu = 0;
      HIPCHECK(s, gj_sweep_occupancy(t, &per_cu));
      if ((long long)per_cu * ncu * t >= most_tiles && per_cu > 0) {
        tpw = t;
        cap = per_cu * ncu;
      }
    }
    if (tpw == 0) {
      s->err = "coarse operator too large for the co-resident sweep";
      return SIM_E_INVALID;
    }
    cs.sw_tpw = tpw;
    cs.sw_stride = (1 + max_nb) * kSwFlag;   // pivot, panels
    std::vector<int> sw_inst, sw_ij;
    s->sweep_groups.assign(1, 0);
    for (int b = 0; b < L.ninst; ++b) {
      const int nb = L.inst_np[b] / kGjTile;
      const int ntile = nb * (nb + 1) / 2;
      const int n = (ntile + tpw - 1) / tpw;
      if (n == 0) continue;
      if ((int)sw_inst.size() + n - s->sweep_groups.back() > cap)
        s->sweep_groups.push_back((int)sw_inst.size());
      const size_t w0 = sw_inst.size();
      sw_inst.resize(w0 + n, b);
      sw_ij.resize((w0 + n) * tpw, -1);
      int e = 0;
      for (int i = 0; i < nb; ++i)
        for (int j = i; j < nb; ++j, ++e) sw_ij[(w0 + e % n) * tpw + e / n] = i * 65536 + j;
    }
    s->sweep_groups.push_back((int)sw_inst.size());
    TRY(upload(s, sw_inst, &cs.sw_inst));
    TRY(upload(s, sw_ij, &cs.sw_ij));
    std::vector<long long> boff;
    for (int b = 0; b < L.ninst; ++b) {
      boff.push_back(s->gj_doubles);
      s->gj_doubles += (long long)kGjTile * L.inst_np[b];
    }
    TRY(upload(s, boff, &cs.inst_boff));
    cs.nmid = L.nmid;
    TRY(upload(s, L.mid_v0, &cs.mid_v0));
    TRY(upload(s, L.mid_modes, &cs.mid_modes));
    TRY(upload(s, L.mid_ptr, &cs.mid_ptr));
    TRY(upload(s, L.mid_slot, &cs.mid_slot));
    TRY(upload(s, L.vert_mid, &cs.vert_mid));
  }

  // ---- workspace
  const size_t nv = L.nv, nt = L.nt, nh = L.nh, ni = L.ninst;
  void* q = nullptr;
  Elem& el = s->el;
  TRY(alloc(s, 9 * nt * 8, &q)); el.tri_f = (double*)q;
  TRY(alloc(s, 81 * nt * 8, &q)); el.tri_K = (double*)q;
  TRY(alloc(s, 12 * nh * 8, &q)); el.hin_g = (double*)q;
  TRY(alloc(s, 12 * nh * 8, &q)); el.hin_f = (double*)q;
  TRY(alloc(s, nh * 8, &q)); el.hin_w = (double*)q;
  TRY(alloc(s, 9 * nt * 8, &q)); el.tri_ag = (double*)q;
  TRY(alloc(s, 9 * nt * 8, &q)); el.tri_ak = (double*)q;
  TRY(alloc(s, 12 * nh * 8, &q)); el.hin_ag = (double*)q;
  TRY(alloc(s, 12 * nh * 8, &q)); el.hin_ak = (double*)q;
  TRY(alloc(s, nt * 8, &q)); el.acc_ks = (double*)q;
  TRY(alloc(s, nh * 8, &q)); el.acc_kb = (double*)q;
  TRY(alloc(s, nv * 8, &q)); el.acc_d = (double*)q;
  el.acc_ws = el.acc_wb = nullptr;
  if (s->mesh.wang) {
    TRY(alloc(s, (size_t)kWangStretch * nt * 8, &q)); el.acc_ws = (double*)q;
    TRY(alloc(s, (size_t)kWangBend * std::max<size_t>(nh, 1) * 8, &q)); el.acc_wb = (double*)q;
  }
  TRY(alloc(s, 3 * nt * 8, &q)); el.tri_fw = (double*)q;
  TRY(alloc(s, 4 * nt * 8, &q)); el.tri_wn = (double*)q;
  TRY(alloc(s, 3 * nt * 8, &q)); el.tri_wv = (double*)q;
  TRY(alloc(s, 3 * nt * 8, &q)); el.acc_w = (double*)q;
  TRY(alloc(s, (size_t)L.maxnz * 9 * nv * s->msize, &s->A));
  TRY(alloc(s, 9 * nv * s->msize, &s->Jinv));
  TRY(alloc(s, 3 * nv * 8, &q)); s->rhs = (double*)q;
  TRY(alloc(s, 3 * nv * 8, &q)); s->sol = (double*)q;
  TRY(alloc(s, 3 * nv * 8, &q)); s->gx = (double*)q;
  TRY(alloc(s, 3 * nv * 8, &q)); s->gv = (double*)q;
  TRY(alloc(s, 3 * nv * 8, &q)); s->sw.zbuf = (double*)q;
  TRY(alloc(s, 6 * nv * 8, &q)); s->sw.pbuf = (double*)q;
  TRY(alloc(s, 8 * nv * 8, &q)); s->sw.tbuf = (unsigned long long*)q;   // [2][4][nv]
  TRY(alloc(s, 4, &q)); s->sw.abort_flag = (int*)q;
  if (coarse) {
    TRY(alloc(s, 3 * nv * 8, &q)); cs.crel = (double*)q;
    TRY(alloc(s, (size_t)L.coarse_doubles * 8, &q)); cs.mat = (double*)q;
    TRY(alloc(s, (size_t)L.coarse_doubles * 4, &q)); cs.xinv = (float*)q;
    // every sweep step's panels (as many doubles as the sheet's matrix) and inverse pivot
    TRY(alloc(s, (size_t)L.coarse_doubles * 8, &q)); cs.gj_c = (double*)q;
    TRY(alloc(s, (size_t)L.coarse_doubles * 8, &q)); cs.gj_r = (double*)q;
    TRY(alloc(s, (size_t)s->gj_doubles * 8, &q)); cs.gj_pinv = (double*)q;
    TRY(alloc(s, 4 * (size_t)ni * cs.sw_stride, &q)); cs.sw_sync = (int*)q;
    TRY(alloc(s, 4 * ni, &q)); cs.ok = (int*)q;
    TRY(alloc(s, 3 * nv * 8, &q)); cs.mid_crel = (double*)q;
    TRY(alloc(s, (size_t)L.nmid * 36 * 8, &q)); cs.mid_inv = (double*)q;
    // Store-all: one slot per step when they fit the cap (the adjoint reuses the
    // forward's operators). With checkpointing: one per step of a checkpoint segment
    // (memory bounded by the interval; the recomputed steps rebuild theirs, the adjoint
    // reuses those), or, with coarse_keep_all, one per step when they fit (the
    // recompute reuses the forward's too). Else none (every step rebuilds).
    const double slot_bytes =
        4.0 * (double)L.coarse_doubles + 8.0 * (6.0 * nv + 36.0 * L.nmid) + 4.0 * ni;
    int want = s->max_steps;
    if (s->ckpt > 0 && (!s->coarse_keep_all || want * slot_bytes > kCoarseStoreCap))
      want = std::min(s->ckpt, s->max_steps);
    if (want * slot_bytes <= kCoarseStoreCap) {
      s->cslots = want;
      TRY(alloc(s, (size_t)want * L.coarse_doubles * 4, &q)); s->cmat_store = (float*)q;
      TRY(alloc(s, (size_t)want * 3 * nv * 8, &q)); s->crel_store = (double*)q;
      TRY(alloc(s, (size_t)want * ni * 4, &q)); s->cok_store = (int*)q;
      TRY(alloc(s, (size_t)want * 3 * nv * 8, &q)); s->mrel_store = (double*)q;
      TRY(alloc(s, (size_t)want * L.nmid * 36 * 8, &q)); s->minv_store = (double*)q;
      s->slot_step.assign(want, 0);
    }
  }
  TRY(alloc(s, 4 * (ni + 1), &q)); s->status = (int*)q;
  const size_t st = (size_t)s->max_steps * ni;
  TRY(alloc(s, st * 4, &q)); s->it_fwd = (int*)q;
  TRY(alloc(s, st * 4, &q)); s->it_rec = (int*)q;
  TRY(alloc(s, st * 4, &q)); s->it_adj = (int*)q;
  TRY(alloc(s, st * 8, &q)); s->res_fwd = (double*)q;
  TRY(alloc(s, st * 8, &q)); s->res_rec = (double*)q;
  TRY(alloc(s, st * 8, &q)); s->res_adj = (double*)q;
  if (s->ckpt == 0) {
    TRY(alloc(s, (size_t)(s->max_steps + 1) * state_bytes(s), &s->traj));
  } else {
    TRY(alloc(s, (size_t)(s->max_steps / s->ckpt + 1) * state_bytes(s), &s->ckpts));
    TRY(alloc(s, 3 * state_bytes(s), &s->tmp));
    TRY(alloc(s, (size_t)s->ckpt * state_bytes(s), &s->seg));
  }
  HIPCHECK(s, hipMemset(s->status, 0, 4 * (ni + 1)));
  HIPCHECK(s, hipMemset(s->it_fwd, 0, st * 4));
  HIPCHECK(s, hipMemset(s->it_rec, 0, st * 4));
  HIPCHECK(s, hipMemset(s->it_adj, 0, st * 4));
  HIPCHECK(s, hipMemset(s->res_fwd, 0, st * 8));
  HIPCHECK(s, hipMemset(s->res_rec, 0, st * 8));
  HIPCHECK(s, hipMemset(s->res_adj, 0, st * 8));
  HIPCHECK(s, hipDeviceSynchronize());

  // ---- solver launch shape: the rule's choice, or the fastest candidate measured on
  // the step system of the rest state
  s->stats.autotune_candidates = (int)feasible.size();
  if (o.autotune && feasible.size() > 1) {
    std::vector<double> xr(3 * nv);
    for (int b = 0; b < L.ninst; ++b)
      for (int q2 = 0; q2 < L.inst_nv[b]; ++q2) {
        const int i = L.inst_voff[b] + q2, src = L.vold[i] - L.inst_voff[b];
        for (int c = 0; c < 3; ++c) xr[(size_t)c * nv + i] = sheets[b].rest[3 * (size_t)src + c];
      }
    int pick = best;
    TRY(s->mprec == SIM_FP64 ? autotune<double>(s, feasible, xr, &pick)
                             : autotune<float>(s, feasible, xr, &pick));
    best = pick;
    s->stats.autotuned = 1;
  }
  TRY(apply_plan(s, feasible[best]));
  HIPCHECK(s, hipDeviceSynchronize());
  s->stats.n_instances = L.ninst;
  long nnzb = 0;
  for (int c : L.ell_col) nnzb += c >= 0;
  s->stats.nnz_blocks = nnzb;
  s->stats.coarse_aggregates = L.nagg;
  s->stats.coarse_max_dim = L.max_nc;
  s->stats.coarse_store_slots = s->cslots;
  return SIM_OK;
}

// The coarse operator of step `step`: its stored slot when the handle keeps them
// (*have: the slot already holds that step), else the shared per-step buffers.
Coarse coarse_for_step(sim_t* s, int step, bool* have) {
  Coarse c = s->coarse;
  *have = false;
  if (s->cslots == 0 || c.nagg == 0) return c;
  const int slot = (step - 1) % s->cslots;
  c.xinv = s->cmat_store + (size_t)slot * s->L.coarse_doubles;
  c.crel = s->crel_store + (size_t)slot * 3 * s->L.nv;
  c.ok = s->cok_store + (size_t)slot * s->L.ninst;
  c.mid_crel = s->mrel_store + (size_t)slot * 3 * s->L.nv;
  c.mid_inv = s->minv_store + (size_t)slot * s->L.nmid * 36;
  *have = s->slot_step[slot] == step;
  s->slot_step[slot] = step;
  return c;
}

// Solver launch bracketed by timing events when timing is enabled.
template <typename TM>
void timed_pcg(sim_t* s, const Coarse& cs, const PcgArgs<TM>& c, hipStream_t st) {
  if (s->timing) {
    if (s->ev_used + 2 > s->ev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        s->ev.push_back(e);
      }
    }
    if (s->ev_used + 2 <= s->ev.size()) {
      (void)hipEventRecord(s->ev[s->ev_used], st);
      launch_pcg<TM>(s->mesh, s->plan, s->sw, cs, c, st);
      (void)hipEventRecord(s->ev[s->ev_used + 1], st);
      s->ev_used += 2;
      return;
    }
  }
  launch_pcg<TM>(s->mesh, s->plan, s->sw, cs, c, st);
}

// ---------------------------------------------------------- step sequences
// reuse: a recomputed step, whose coarse operator the forward pass of the same rollout
// may have kept (the forward pass always builds its own)
template <typename T, typename TM>
void forward_step(sim_t* s, int step, const char* sp, char* sn, const T* F, const double* mat,
                  T* xout, int* iters, double* resid, bool reuse, hipStream_t st) {
  const int nv = s->L.nv;
  const double* xp = reinterpret_cast<const double*>(sp);
  const double* vp = xp + 3 * (size_t)nv;
  double* xn = reinterpret_cast<double*>(sn);
  double* vn = xn + 3 * (size_t)nv;
  launch_elements(s->mesh, s->el, xp, vp, mat, s->wind, s->rho_air, s->status, st);
  AssembleArgs<T, TM> a{};
  a.v = vp;
  a.forces = F;
  a.mat = mat;
  a.h = s->h;
  for (int k = 0; k < 3; ++k) a.g[k] = s->grav[k];
  a.want_rhs = 1;
  a.wind = s->wind ? 1 : 0;
  a.A = static_cast<TM*>(s->A);
  a.Jinv = static_cast<TM*>(s->Jinv);
  a.b = s->rhs;
  a.status = s->status;
  launch_assemble<T, TM>(s->mesh, s->el, a, st);
  bool have = false;
  const Coarse cs = coarse_for_step(s, step, &have);
  if (!(reuse && have))
    launch_coarse_setup<TM>(s->mesh, cs, xp, a.A, s->L.coarse_doubles, s->sweep_groups, st);
  PcgArgs<TM> c{};
  c.A = a.A;
  c.Jinv = a.Jinv;
  c.rhs = s->rhs;
  c.sol = s->sol;
  c.tol = s->cg_tol;
  c.max_iter = s->cg_max_iter;
  c.iters = iters;
  c.resid = resid;
  c.status = s->status;
  timed_pcg<TM>(s, cs, c, st);
  launch_update<T>(s->mesh, xp, vp, s->sol, s->h, xn, vn, xout, s->status, st);
}

template <typename T>
const T* force_slice(const sim_t* s, int step) {
  if (!s->forces) return nullptr;
  return static_cast<const T*>(s->forces) + (size_t)(step - 1) * 3 * s->L.nv;
}

template <typename T, typename TM>
sim_status rollout_impl(sim_t* s, int n, const void* x0, const void* v0, void* x_out,
                        hipStream_t st) {
  const int nv = s->L.nv, ni = s->L.ninst;
  char* s0 = fwd_state(s, 0, n);
  launch_init_state<T>(s->mesh, static_cast<const T*>(x0), static_cast<const T*>(v0),
                       reinterpret_cast<double*>(s0), reinterpret_cast<double*>(s0) + 3 * (size_t)nv,
                       s->status, st);
  size_t f = 0;
  for (int k = 1; k <= n; ++k) {
    T* xo = nullptr;
    if (f < s->frames.size() && s->frames[f] == k) {
      xo = static_cast<T*>(x_out) + f * 3 * (size_t)nv;
      ++f;
    }
    forward_step<T, TM>(s, k, fwd_state(s, k - 1, n), fwd_state(s, k, n), force_slice<T>(s, k),
                    s->material, xo, s->it_fwd + (size_t)(k - 1) * ni,
                    s->res_fwd + (size_t)(k - 1) * ni, false, st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(s, e, "rollout launch");
  return SIM_OK;
}

template <typename T, typename TM>
void adjoint_step(sim_t* s, int k, const char* sp, const char* sn, const T* dl, T* dlF,
                  hipStream_t st) {
  const int nv = s->L.nv, ni = s->L.ninst;
  const double* xp = reinterpret_cast<const double*>(sp);
  const double* vp = xp + 3 * (size_t)nv;
  const double* vs = reinterpret_cast<const double*>(sn) + 3 * (size_t)nv;
  double* u = s->rhs;  // the adjoint right-hand side reuses the forward rhs buffer
  launch_adj_pre<T>(s->mesh, dl, s->h, s->gx, s->gv, u, s->status, st);
  launch_elements(s->mesh, s->el, xp, vp, s->material, s->wind, s->rho_air, s->status, st);
  AssembleArgs<T, TM> a{};
  a.v = vp;
  a.forces = nullptr;
  a.mat = s->material;
  a.h = s->h;
  for (int q = 0; q < 3; ++q) a.g[q] = s->grav[q];
  a.want_rhs = 0;
  a.wind = s->wind ? 1 : 0;
  a.A = static_cast<TM*>(s->A);
  a.Jinv = static_cast<TM*>(s->Jinv);
  a.b = nullptr;
  a.status = s->status;
  launch_assemble<T, TM>(s->mesh, s->el, a, st);
  // the step's coarse operator: kept from the forward pass or the recompute when the
  // handle stores them, else rebuilt (the same kernels on the same inputs)
  bool have = false;
  const Coarse cs = coarse_for_step(s, k, &have);
  if (!have)
    launch_coarse_setup<TM>(s->mesh, cs, xp, a.A, s->L.coarse_doubles, s->sweep_groups, st);
  PcgArgs<TM> c{};
  c.A = a.A;
  c.Jinv = a.Jinv;
  c.rhs = u;
  c.sol = s->sol;
  c.tol = s->cg_tol;
  c.max_iter = s->cg_max_iter;
  c.iters = s->it_adj + (size_t)(k - 1) * ni;
  c.resid = s->res_adj + (size_t)(k - 1) * ni;
  c.status = s->status;
  timed_pcg<TM>(s, cs, c, st);
  AdjArgs<T> j{};
  j.x = xp;
  j.vp = vp;
  j.vs = vs;
  j.mu = s->sol;
  j.u = u;
  j.mat = s->material;
  j.h = s->h;
  for (int q = 0; q < 3; ++q) j.g[q] = s->grav[q];
  j.gx = s->gx;
  j.gv = s->gv;
  j.dl_dF = dlF;
  j.wind = s->wind;
  j.rho = s->rho_air;
  launch_adj_elements<T>(s->mesh, s->el, j, st);
  launch_adj_rows<T>(s->mesh, s->el, j, st);
}

template <typename T, typename TM>
sim_status adjoint_impl(sim_t* s, const void* dl_dx, void* dl_dmat, void* dl_dwind, void* dl_dF,
                        void* dl_dx0, void* dl_dv0, hipStream_t st) {
  const int nv = s->L.nv, ni = s->L.ninst, n = s->n_steps;
  launch_fill_double(s->gx, 3L * nv, 0.0, st);
  launch_fill_double(s->gv, 3L * nv, 0.0, st);
  if (s->wind) launch_fill_double(s->el.acc_w, 3L * s->L.nt, 0.0, st);
  launch_fill_double(s->el.acc_ks, s->L.nt, 0.0, st);
  launch_fill_double(s->el.acc_kb, s->L.nh, 0.0, st);
  if (s->mesh.wang) {
    launch_fill_double(s->el.acc_ws, (long)kWangStretch * s->L.nt, 0.0, st);
    launch_fill_double(s->el.acc_wb, (long)kWangBend * s->L.nh, 0.0, st);
  }
  launch_fill_double(s->el.acc_d, nv, 0.0, st);
  const T* dl = static_cast<const T*>(dl_dx);
  int f = (int)s->frames.size() - 1;
  const int k = s->ckpt == 0 ? n : s->ckpt;
  const int nseg = (n + k - 1) / k;
  for (int c = nseg - 1; c >= 0; --c) {
    const int c0 = c * k, c1 = std::min(n, c0 + k);
    if (s->ckpt != 0) {
      // recompute the interior states of the segment from its checkpoint
      for (int q = c0 + 1; q < c1; ++q)
        forward_step<T, TM>(s, q, adj_state(s, q - 1, c0, n), adj_state(s, q, c0, n), force_slice<T>(s, q),
                        s->material, nullptr, s->it_rec + (size_t)(q - 1) * ni,
                        s->res_rec + (size_t)(q - 1) * ni, true, st);
    }
    for (int q = c1; q > c0; --q) {
      const T* dlq = nullptr;
      if (f >= 0 && s->frames[f] == q) {
        dlq = dl + (size_t)f * 3 * nv;
        --f;
      }
      T* dlF = dl_dF ? static_cast<T*>(dl_dF) + (size_t)(q - 1) * 3 * nv : nullptr;
      adjoint_step<T, TM>(s, q, adj_state(s, q - 1, c0, n), adj_state(s, q, c0, n), dlq, dlF, st);
    }
  }
  launch_adj_final<T>(s->mesh, s->gx, s->gv, static_cast<T*>(dl_dx0), static_cast<T*>(dl_dv0), st);
  launch_material_sum(s->mesh, s->el, static_cast<double*>(dl_dmat), static_cast<double*>(dl_dwind),
                      st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(s, e, "adjoint launch");
  return SIM_OK;
}

void graph_release(sim_t::GraphCache& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = sim_t::GraphCache{};
}

// Runs body(stream) directly, or (graph option, timing off) replays the cached graph
// when the key matches, else captures body on the handle's capture stream, keeps the
// graph and launches it on the caller's stream. Nothing in the step sequences
// allocates, synchronises or records memsets, so they capture as plain kernel nodes.
template <class Body>
sim_status graphed(sim_t* s, sim_t::GraphCache& gc, const std::vector<uintptr_t>& key,
                   hipStream_t user, Body&& body) {
  if (!s->use_graph || s->timing) return body(user);
  if (gc.valid && gc.key == key) {
    s->slot_step = gc.slot_after;
    HIPCHECK(s, hipGraphLaunch(gc.exec, user));
    ++s->graph_replays;
    return SIM_OK;
  }
  graph_release(gc);
  if (!s->cap_stream) HIPCHECK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  HIPCHECK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
  const sim_status st = body(s->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
  if (st != SIM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(s, e, "hipStreamEndCapture");
  gc.graph = g;
  HIPCHECK(s, hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0));
  gc.key = key;
  gc.slot_after = s->slot_step;
  gc.valid = true;
  ++s->graph_captures;
  HIPCHECK(s, hipGraphLaunch(gc.exec, user));
  return SIM_OK;
}

// Argument checks and bookkeeping shared by the rollout entry points.
sim_status begin_rollout(sim_t* s, int n_steps, const void* x0, const void* forces,
                         const void* material, const void* wind, const int32_t* loss_frames,
                         int n_loss, void* x_out, void* stream) {
  if (!s) return SIM_E_INVALID;
  if (n_steps < 1 || n_steps > s->max_steps || !x0 || n_loss < 0 ||
      (n_loss > 0 && (!loss_frames || !x_out))) {
    s->err = "invalid rollout arguments";
    return SIM_E_INVALID;
  }
  int prev = 0;
  for (int k = 0; k < n_loss; ++k) {
    if (loss_frames[k] <= prev || loss_frames[k] > n_steps) {
      s->err = "loss frames must be strictly increasing within 1..n_steps";
      return SIM_E_INVALID;
    }
    prev = loss_frames[k];
  }
  s->have_rollout = false;
  s->have_adjoint = false;
  s->n_steps = n_steps;
  s->frames.assign(loss_frames, loss_frames + n_loss);
  s->forces = forces;
  s->material = material ? static_cast<const double*>(material) : s->mat_default;
  s->wind = static_cast<const double*>(wind);
  s->stream = static_cast<hipStream_t>(stream);
  return SIM_OK;
}

sim_status run_rollout(sim_t* s, int n_steps, const void* x0, const void* v0, void* x_out,
                       hipStream_t q) {
  if (s->prec == SIM_FP64)
    return s->mprec == SIM_FP64 ? rollout_impl<double, double>(s, n_steps, x0, v0, x_out, q)
                                : rollout_impl<double, float>(s, n_steps, x0, v0, x_out, q);
  return s->mprec == SIM_FP64 ? rollout_impl<float, double>(s, n_steps, x0, v0, x_out, q)
                              : rollout_impl<float, float>(s, n_steps, x0, v0, x_out, q);
}

// The solver's exchange buffers (the ones sim_create allocates for the handle: the
// global copies of the preconditioned vectors, the tagged publications, the partial
// sums, the barrier counters and abort flag, the coarse restriction partials) laid
// out 256-byte aligned in the scratch array at base, of cap bytes. Every launch of
// the solver clears what must start at zero (counters, flag, tagged words) with a
// fill kernel; the rest is written before it is read.
sim_status noalloc_work(sim_t* s, char* base, size_t cap, SolverWork* w, double** part) {
  const size_t nv = s->L.nv, nwg = s->plan.nwg;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  *w = s->sw;
  w->zbuf = reinterpret_cast<double*>(take(3 * nv * 8));
  w->pbuf = reinterpret_cast<double*>(take(6 * nv * 8));
  w->tbuf = reinterpret_cast<unsigned long long*>(take(8 * nv * 8));
  w->red = reinterpret_cast<double*>(take(6 * nwg * 8));
  w->tred = reinterpret_cast<unsigned long long*>(take(2 * nwg * kTagSlots * 16));
  w->barrier = reinterpret_cast<int*>(take((size_t)s->sw.barrier_ints * 4));
  w->abort_flag = reinterpret_cast<int*>(take(4));
  *part = s->L.nagg > 0 ? reinterpret_cast<double*>(take(nwg * kMaxWgAgg * 6 * 8)) : nullptr;
  if (off > cap) {
    s->err = "the solver's exchange buffers (" + std::to_string(off) +
             " bytes) exceed the allocation-free rollout's scratch array (" +
             std::to_string(cap) + " bytes)";
    return SIM_E_INVALID;
  }
  return SIM_OK;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

void sim_default_options(sim_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = SIM_FP32;
  o->cg_tol = 1e-7;
  o->cg_max_iter = 20000;
  o->checkpoint_every = 0;
  o->gravity[0] = 0.0;
  o->gravity[1] = 0.0;
  o->gravity[2] = -9.81;
  o->max_steps = 1000;
  o->rows_per_block = 0;
  o->membrane_system = SIM_MEMBRANE_EXACT;
  o->matrix_precision = SIM_FP64;
  o->coarse_size = 64;
  o->matrix_home = SIM_MATRIX_AUTO;
  o->air_density = 1.0;
  o->coarse_keep_all = 0;
  o->material_model = SIM_MATERIAL_ISOTROPIC;
}

sim_status sim_create_batch(int32_t n, const sim_mesh* meshes, const double* const* rest_pos,
                            const int32_t* const* pins, const int32_t* n_pins,
                            const sim_material* mats, double dt, const sim_options* opt,
                            sim_t** out) {
  if (!out) return SIM_E_INVALID;
  *out = nullptr;
  if (n < 1 || !meshes || !rest_pos || !mats) return SIM_E_INVALID;
  std::vector<HostSheet> sheets(n);
  for (int b = 0; b < n; ++b) {
    const sim_mesh& m = meshes[b];
    if (m.n_verts < 3 || m.n_tris < 1 || !m.tris || !rest_pos[b]) return SIM_E_INVALID;
    int np = n_pins ? n_pins[b] : 0;
    if (np < 0 || (np > 0 && (!pins || !pins[b]))) return SIM_E_INVALID;
    HostSheet& s = sheets[b];
    s.nv = m.n_verts;
    s.nt = m.n_tris;
    s.tris.assign(m.tris, m.tris + 3 * (size_t)m.n_tris);
    s.rest.assign(rest_pos[b], rest_pos[b] + 3 * (size_t)m.n_verts);
    if (np > 0) s.pins.assign(pins[b], pins[b] + np);
    s.mat[0] = mats[b].stretch;
    s.mat[1] = mats[b].bend;
    s.mat[2] = mats[b].density;
    if (!std::isfinite(s.mat[0]) || !std::isfinite(s.mat[1]) || !std::isfinite(s.mat[2]) ||
        !(s.mat[2] > 0.0))
      return SIM_E_INVALID;
  }
  sim_t* s = new (std::nothrow) sim_t();
  if (!s) return SIM_E_NOMEM;
  sim_status st = setup(s, sheets, dt, opt);
  if (st != SIM_OK) {
    std::fprintf(stderr, "sim_create: %s\n", s->err.c_str());
    sim_destroy(s);
    return st;
  }
  *out = s;
  return SIM_OK;
}

sim_status sim_create(const sim_mesh* mesh, const double* rest_pos, const int32_t* pins,
                      int32_t n_pins, const sim_material* mat, double dt, const sim_options* opt,
                      sim_t** out) {
  if (!mesh || !mat) return SIM_E_INVALID;
  const double* rp[1] = {rest_pos};
  const int32_t* pp[1] = {pins};
  int32_t np[1] = {n_pins};
  return sim_create_batch(1, mesh, rp, pp, np, mat, dt, opt, out);
}

sim_status sim_rollout(sim_t* s, int32_t n_steps, const void* x0, const void* v0,
                       const void* forces, const void* material, const void* wind,
                       const int32_t* loss_frames, int32_t n_loss, void* x_out, void* stream) {
  TRY(begin_rollout(s, n_steps, x0, forces, material, wind, loss_frames, n_loss, x_out, stream));
  std::vector<uintptr_t> key = {(uintptr_t)n_steps, (uintptr_t)x0, (uintptr_t)v0,
                                (uintptr_t)forces, (uintptr_t)s->material, (uintptr_t)wind,
                                (uintptr_t)x_out};
  key.insert(key.end(), s->frames.begin(), s->frames.end());
  const sim_status st = graphed(s, s->gfwd, key, s->stream, [&](hipStream_t q) {
    return run_rollout(s, n_steps, x0, v0, x_out, q);
  });
  if (st == SIM_OK) s->have_rollout = true;
  return st;
}

sim_status sim_rollout_noalloc(sim_t* s, int32_t n_steps, const void* x0, const void* v0,
                               const void* forces, const void* material, const void* wind,
                               const int32_t* loss_frames, int32_t n_loss, void* x_out,
                               void* stream) {
  if (!s) return SIM_E_INVALID;
  if (s->use_graph) {
    s->err = "sim_rollout_noalloc needs a handle without the graph option";
    return SIM_E_INVALID;
  }
  TRY(begin_rollout(s, n_steps, x0, forces, material, wind, loss_frames, n_loss, x_out, stream));
  void* base = nullptr;
  HIPCHECK(s, noalloc_scratch(&base));
  SolverWork w{};
  double* part = nullptr;
  TRY(noalloc_work(s, static_cast<char*>(base), kNoAllocScratchBytes, &w, &part));
  // the handle's own exchange buffers are swapped out while the launches are enqueued
  // (kernels take them by value); no timing events are recorded
  const SolverWork saved = s->sw;
  double* saved_part = s->coarse.part;
  const bool saved_timing = s->timing;
  s->sw = w;
  s->coarse.part = part;
  s->timing = false;
  const sim_status st = run_rollout(s, n_steps, x0, v0, x_out, s->stream);
  s->sw = saved;
  s->coarse.part = saved_part;
  s->timing = saved_timing;
  if (st == SIM_OK) s->have_rollout = true;
  return st;
}

sim_status sim_adjoint(sim_t* s, const void* dl_dx, void* dl_dmaterial, void* dl_dwind,
                       void* dl_dforces, void* dl_dx0, void* dl_dv0, void* stream) {
  if (!s) return SIM_E_INVALID;
  if (!s->have_rollout) {
    s->err = "sim_adjoint needs a preceding sim_rollout";
    return SIM_E_STATE;
  }
  if (dl_dwind && !s->wind) {
    s->err = "dl_dwind needs a rollout with a wind velocity";
    return SIM_E_INVALID;
  }
  if (!s->frames.empty() && !dl_dx) {
    s->err = "dl_dx is required when the rollout has loss frames";
    return SIM_E_INVALID;
  }
  s->stream = static_cast<hipStream_t>(stream);
  // the adjoint reads the rollout's states, forces and material: its key includes them
  std::vector<uintptr_t> key = {(uintptr_t)dl_dx, (uintptr_t)dl_dmaterial, (uintptr_t)dl_dwind,
                                (uintptr_t)dl_dforces, (uintptr_t)dl_dx0, (uintptr_t)dl_dv0};
  key.insert(key.end(), s->gfwd.key.begin(), s->gfwd.key.end());
  s->have_adjoint = true;
  return graphed(s, s->gadj, key, s->stream, [&](hipStream_t q) {
    if (s->prec == SIM_FP64)
      return s->mprec == SIM_FP64
                 ? adjoint_impl<double, double>(s, dl_dx, dl_dmaterial, dl_dwind, dl_dforces,
                                                dl_dx0, dl_dv0, q)
                 : adjoint_impl<double, float>(s, dl_dx, dl_dmaterial, dl_dwind, dl_dforces,
                                               dl_dx0, dl_dv0, q);
    return s->mprec == SIM_FP64
               ? adjoint_impl<float, double>(s, dl_dx, dl_dmaterial, dl_dwind, dl_dforces, dl_dx0,
                                             dl_dv0, q)
               : adjoint_impl<float, float>(s, dl_dx, dl_dmaterial, dl_dwind, dl_dforces, dl_dx0,
                                            dl_dv0, q);
  });
}

sim_status sim_sync_status(sim_t* s) {
  if (!s) return SIM_E_INVALID;
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "hipStreamSynchronize");
  const int ni = s->L.ninst;
  std::vector<int> words(ni + 1, 0);
  e = hipMemcpy(words.data(), s->status, 4 * (ni + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(s, e, "status readback");
  e = hipMemset(s->status, 0, 4 * (ni + 1));
  if (e != hipSuccess) return hip_fail(s, e, "status reset");
  s->inst_status.assign(ni, SIM_OK);
  for (int b = 0; b < ni; ++b) s->inst_status[b] = bits_to_status(words[1 + b]);
  const int bits = words[0];
  // statistics of the most recent calls
  const int n = s->n_steps;
  std::vector<int> itf((size_t)n * ni), itr((size_t)n * ni), ita((size_t)n * ni);
  std::vector<double> rf((size_t)n * ni), ra((size_t)n * ni);
  if (n > 0) {
    (void)hipMemcpy(itf.data(), s->it_fwd, itf.size() * 4, hipMemcpyDeviceToHost);
    (void)hipMemcpy(rf.data(), s->res_fwd, rf.size() * 8, hipMemcpyDeviceToHost);
    if (s->have_adjoint) {
      // the adjoint's solves (and the checkpoint recompute's) belong to this rollout only
      // once an adjoint has run since it
      (void)hipMemcpy(itr.data(), s->it_rec, itr.size() * 4, hipMemcpyDeviceToHost);
      (void)hipMemcpy(ita.data(), s->it_adj, ita.size() * 4, hipMemcpyDeviceToHost);
      (void)hipMemcpy(ra.data(), s->res_adj, ra.size() * 8, hipMemcpyDeviceToHost);
    }
  }
  sim_stats& S = s->stats;
  S.n_steps = n;
  S.cg_iters_forward = S.cg_iters_recompute = S.cg_iters_adjoint = 0;
  S.cg_iters_max = 0;
  S.max_rel_residual = 0.0;
  for (size_t q = 0; q < itf.size(); ++q) {
    S.cg_iters_forward += itf[q];
    S.cg_iters_recompute += itr[q];
    S.cg_iters_adjoint += ita[q];
    S.cg_iters_max = std::max(S.cg_iters_max, std::max(itf[q], ita[q]));
    S.max_rel_residual = std::max(S.max_rel_residual, std::max(rf[q], ra[q]));
  }
  for (size_t q = 0; q + 1 < s->ev_used; q += 2) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, s->ev[q], s->ev[q + 1]) == hipSuccess) {
      S.solver_ms += ms;
      S.solver_launches += 1;
    }
  }
  s->ev_used = 0;
  sim_status st = bits_to_status(bits);
  if (bits & ST_TIMEOUT) s->err = "solver workgroups timed out at a cluster barrier";
  S.device_status = st;
  return st;
}

sim_status sim_frame_loss(sim_t* s, int32_t n_frames, const void* x, const void* target,
                          double* energy, void* dl_dx, void* stream) {
  if (!s) return SIM_E_INVALID;
  if (n_frames < 0 || (n_frames > 0 && (!x || !target || !energy))) {
    s->err = "invalid frame-loss arguments";
    return SIM_E_INVALID;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Mesh& m = s->mesh;
  if (s->prec == SIM_FP64)
    launch_frame_loss<double>(static_cast<const double*>(x), static_cast<const double*>(target),
                              m.nv, m.inst_voff, m.inst_nv, m.ninst, n_frames, energy,
                              static_cast<double*>(dl_dx), st);
  else
    launch_frame_loss<float>(static_cast<const float*>(x), static_cast<const float*>(target), m.nv,
                             m.inst_voff, m.inst_nv, m.ninst, n_frames, energy,
                             static_cast<float*>(dl_dx), st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(s, e, "frame loss launch");
  return SIM_OK;
}

sim_status sim_get_vertex_areas(const sim_t* s, double* out) {
  if (!s || !out) return SIM_E_INVALID;
  // internal vertex i is the caller's vertex vold[i] of the same sheet range
  for (int i = 0; i < s->L.nv; ++i) out[s->L.vold[i]] = s->L.varea[i];
  return SIM_OK;
}

sim_status sim_set_timing(sim_t* s, int32_t enable) {
  if (!s) return SIM_E_INVALID;
  s->timing = enable != 0;
  s->ev_used = 0;
  s->stats.solver_ms = 0.0;
  s->stats.solver_launches = 0;
  return SIM_OK;
}

sim_status sim_get_instance_status(const sim_t* s, int32_t* out) {
  if (!s || !out) return SIM_E_INVALID;
  for (int b = 0; b < s->L.ninst; ++b)
    out[b] = b < (int)s->inst_status.size() ? s->inst_status[b] : SIM_OK;
  return SIM_OK;
}

sim_status sim_get_stats(const sim_t* s, sim_stats* out) {
  if (!s || !out) return SIM_E_INVALID;
  *out = s->stats;
  out->graph_captures = s->graph_captures;
  out->graph_replays = s->graph_replays;
  out->device_bytes = (int64_t)s->dev_bytes;
  return SIM_OK;
}

sim_status sim_get_cg_iters(const sim_t* s, int32_t* forward, int32_t* adjoint) {
  if (!s) return SIM_E_INVALID;
  const size_t cnt = (size_t)s->n_steps * s->L.ninst;
  if (cnt == 0) return SIM_OK;
  if (forward && hipMemcpy(forward, s->it_fwd, cnt * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return SIM_E_HIP;
  if (adjoint && hipMemcpy(adjoint, s->it_adj, cnt * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return SIM_E_HIP;
  return SIM_OK;
}

const char* sim_status_string(sim_status st) {
  switch (st) {
    case SIM_OK: return "ok";
    case SIM_E_INVALID: return "invalid argument";
    case SIM_E_MESH: return "invalid mesh";
    case SIM_E_NOMEM: return "out of memory";
    case SIM_E_HIP: return "HIP runtime error";
    case SIM_E_NOT_CONVERGED: return "CG did not converge within cg_max_iter";
    case SIM_E_INDEFINITE: return "CG breakdown (system not positive definite)";
    case SIM_E_NONFINITE: return "non-finite value";
    case SIM_E_STATE: return "call out of order";
  }
  return "unknown status";
}

const char* sim_last_error(const sim_t* s) { return s ? s->err.c_str() : ""; }

void sim_destroy(sim_t* s) {
  if (!s) return;
  if (!s->allocs.empty()) (void)hipDeviceSynchronize();
  graph_release(s->gfwd);
  graph_release(s->gadj);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  for (void* p : s->allocs) (void)hipFree(p);
  delete s;
}

}  // extern "C"

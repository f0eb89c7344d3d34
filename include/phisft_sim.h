/*
 * phisft_sim.h -- C ABI of the differentiable cloth simulator (MI355X / gfx950).
 *
 * What it computes (Kairanda et al., "phi-SfT", CVPR 2022, Sec. 3.1):
 *   * the deformation model S_t = PS(S_{t-1}; phi_{t-1}) (Eq. 1) with
 *     phi = {d, S, B, w, F_t} (Eq. 2): areal density d, stretching stiffness S
 *     and bending stiffness B (scalars k_s, k_b, or strain-dependent anisotropic
 *     tables S in R^24, B in R^15; see sim_material_model), an optional wind
 *     velocity w driving an aerodynamic force (air
 *     density fixed, Sec. 3.4; see sim_rollout) and per-step, per-vertex
 *     corrective forces F_t;
 *   * per step one linearised backward-Euler update (Eq. 4 with the force
 *     linearisation of Eq. 5, df/dv = 0), solved for Delta v by a
 *     preconditioned conjugate gradient (pipelined; three-level additive
 *     preconditioner: 3x3 block Jacobi, the rigid motions of runs of 16
 *     vertices, and a coarse space of the rigid motions of larger aggregates;
 *     block Jacobi alone with coarse_size = 0). A solve is accepted only on a
 *     true residual, ||b - A Delta v||_2 <= cg_tol ||b||_2:
 *         (M + h D + h^2 K_sys(x_{t-1})) Delta v = h (f(x_{t-1}, v_{t-1}) + M g + F_t - h K_sys v_{t-1})
 *         v_t = v_{t-1} + Delta v,   x_t = x_{t-1} + h v_t
 *     with M the lumped mass (density times a third of the incident triangle
 *     areas), f = -dE/dx for E = sum_tri area (k_s/2) |G|_F^2 (Green strain G)
 *     + sum_hinge k_b c_e (theta - theta_rest)^2 (or the anisotropic energy of
 *     sim_material_model), and K_sys the system stiffness (membrane Hessian, see
 *     sim_membrane_system, plus the Gauss-Newton bending Hessian
 *     d^2E/dtheta^2 grad(theta) grad(theta)^T), and
 *     D = -df/dv the velocity Jacobian of the aerodynamic force (zero without
 *     wind);
 *   * the adjoint of that rollout (the paper's backward pass by implicit
 *     differentiation of Eq. 4): gradients of a per-frame loss with respect to
 *     the material (k_s, k_b, d or S, B, d), the wind velocity w, the forces F_t
 *     and the initial state
 *     (x_0, v_0).
 * Collisions (Eq. 6) are not part of this library.
 *
 * Conventions
 *   Layout     Per-vertex device arrays are structure-of-arrays [3][V]
 *              (all x, then all y, then all z), V = total vertices of the handle.
 *              A batch handle concatenates its instances' vertices in order.
 *   dtype      Device state arrays (x0, v0, forces, x_out, dl_dx, dl_dforces,
 *              dl_dx0, dl_dv0) are float for SIM_FP32 and double for SIM_FP64.
 *              Material arrays are always double, [n_instances][n_mat]: with
 *              SIM_MATERIAL_ISOTROPIC n_mat = 3, (k_s [N/m], k_b [N m], d [kg/m^2]);
 *              with SIM_MATERIAL_WANG n_mat = SIM_WANG_PARAMS = 40, the stretch
 *              table S [4][6] [N/m], the bend table B [3][5] [N m], then d.
 *   Units      SI. Gravity defaults to (0, 0, -9.81) m/s^2.
 *   Ownership  sim_create copies mesh, rest positions and pins. The caller owns
 *              every device pointer passed to sim_rollout / sim_adjoint. The
 *              forces and material buffers given to sim_rollout are read again
 *              by the matching sim_adjoint (checkpoint recompute) and must stay
 *              valid and unchanged until it has been enqueued and has run.
 *              The library owns its workspace (trajectory/checkpoints, system
 *              matrix, solver vectors).
 *   Streams    Calls enqueue work on the given hipStream_t (NULL = default
 *              stream) and return without synchronising. One handle must not
 *              be used from two host threads at once.
 *   State      create -> (rollout -> adjoint?)* -> destroy. sim_adjoint refers to
 *              the most recent rollout; otherwise it returns SIM_E_STATE.
 *   Errors     Argument and mesh errors return immediately. Device-side
 *              conditions (non-finite values, CG not converged, CG breakdown
 *              p.Ap <= 0) are sticky: they are recorded on the device and
 *              reported by sim_sync_status. A solve that reaches cg_max_iter
 *              keeps its last iterate and the rollout continues. After an error
 *              outputs are unspecified; the handle stays valid.
 */
#ifndef PHISFT_SIM_H
#define PHISFT_SIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_s sim_t;

typedef enum {
  SIM_OK = 0,
  SIM_E_INVALID = -1,       /* bad argument */
  SIM_E_MESH = -2,          /* degenerate / non-manifold / inconsistently oriented mesh */
  SIM_E_NOMEM = -3,         /* device or host allocation failed */
  SIM_E_HIP = -4,           /* HIP runtime error (text in sim_last_error) */
  SIM_E_NOT_CONVERGED = -5, /* a CG solve stopped at cg_max_iter, or its recurrences kept
                               meeting cg_tol while the true residual did not (16
                               restarts, then a final check of the true residual); the
                               rollout continues with the last iterate */
  SIM_E_INDEFINITE = -6,    /* CG breakdown: p.Ap <= 0 or a singular diagonal block */
  SIM_E_NONFINITE = -7,     /* NaN/Inf in inputs, system or state */
  SIM_E_STATE = -8          /* call out of order (e.g. adjoint without a rollout) */
} sim_status;

typedef enum { SIM_FP32 = 0, SIM_FP64 = 1 } sim_precision;

/* Stress term of the membrane block of the system stiffness K_sys (the
 * Jacobian of Eq. 5, evaluated at the previous state):
 *   SIM_MEMBRANE_EXACT    the true Hessian of the stretching energy (default).
 *                         A = M + h^2 K_sys can become indefinite under
 *                         compression; CG then reports SIM_E_INDEFINITE.
 *   SIM_MEMBRANE_TENSION  only the tension part of the strain enters the stress
 *                         term (compressive principal strains clamped to zero):
 *                         A is SPD in every state, but the clamp is not
 *                         differentiable where a principal strain is zero (for
 *                         instance at the rest state), so gradients taken there
 *                         depend on rounding. */
typedef enum { SIM_MEMBRANE_EXACT = 0, SIM_MEMBRANE_TENSION = 1 } sim_membrane_system;

/* Material model of the internal forces (the paper's S and B, Eq. 2, after Wang et
 * al., whose formulas the paper does not give; sim_options.material_model).
 *   SIM_MATERIAL_ISOTROPIC  E = sum_tri area (k_s/2) |G|_F^2 + sum_hinge k_b c_e
 *                           (theta - theta_rest)^2: scalar stand-ins for S and B.
 *   SIM_MATERIAL_WANG       strain-dependent, anisotropic (S in R^24, B in R^15):
 *     stretch  four measures of the Green strain G in the sheet's material frame (u:
 *              the rest x axis projected into the triangle's plane, the rest y axis
 *              where x is within 0.06 degrees of its normal; v = n x u): s_1 = G_uu
 *              (warp), s_2 = G_vv (weft), s_3 = sqrt(2) G_uv (shear), s_4 = G_uu + G_vv
 *              (area). Measure k has a piecewise-linear stress sigma_k(|s|) whose slope
 *              is S[k][j] on strain segment j (breaks SIM_WANG_STRAIN_BREAKS: 0, 0.25,
 *              0.5, 1, 2, 4 %, the last segment open); the energy is
 *              sum_tri area sum_k psi_k(|s_k|) with psi_k' = sigma_k.
 *     bending  sum_hinge c_e Phi_e(theta - theta_rest), Phi(d) = 2 psi(|d|), psi' the
 *              piecewise-linear moment whose slope on angle segment j (breaks 0, 0.05,
 *              0.1, 0.2, 0.4 rad) is B[0][j], B[1][j], B[2][j] interpolated linearly in
 *              the angle (0, 45, 90 degrees) between the bending direction (in the
 *              plane of the hinge's first triangle, normal to the edge) and that
 *              plane's warp axis.
 *     S[0..2][j] = k_s, S[3][j] = 0 and B[a][j] = k_b give the isotropic model; the
 *     membrane block of K_sys is the exact Hessian (SIM_MEMBRANE_TENSION is refused).
 *     The create-time sim_material (k_s, k_b, d) becomes such isotropic tables. */
typedef enum { SIM_MATERIAL_ISOTROPIC = 0, SIM_MATERIAL_WANG = 1 } sim_material_model;
#define SIM_WANG_STRETCH 24
#define SIM_WANG_BEND 15
#define SIM_WANG_PARAMS 40

/* Where the persistent solver keeps its workgroup's rows of the system matrix during
 * a solve. Every home computes the same products in the same order (bitwise equal
 * results); they differ only in speed.
 *   SIM_MATRIX_AUTO       the library's choice (rule or autotuner).
 *   SIM_MATRIX_STREAMED   read from the assembled matrix in device memory at every
 *                         product.
 *   SIM_MATRIX_LDS        copied once per solve into LDS (only where they fit).
 *   SIM_MATRIX_REGISTERS  copied once per solve into the registers of each row's
 *                         lane (rows of at most 13 blocks, i.e. grid sheets; one
 *                         solver workgroup per CU); in workgroups of at most 128
 *                         rows the blocks may be split over two wavefront teams
 *                         (sim_stats.solver_row_teams).
 * A home that no launch shape can use makes sim_create fail with SIM_E_INVALID. */
typedef enum {
  SIM_MATRIX_AUTO = 0,
  SIM_MATRIX_STREAMED = 1,
  SIM_MATRIX_LDS = 2,
  SIM_MATRIX_REGISTERS = 3
} sim_matrix_home;

/* Host triangle mesh: tris [n_tris][3] vertex ids, counter-clockwise. */
typedef struct {
  int32_t n_verts;
  int32_t n_tris;
  const int32_t* tris;
} sim_mesh;

/* Material of one sheet (Eq. 2: d, and scalar stand-ins for S and B). */
typedef struct {
  double stretch; /* k_s [N/m]   */
  double bend;    /* k_b [N m]   */
  double density; /* d   [kg/m^2] */
} sim_material;

typedef struct {
  int32_t precision;        /* sim_precision of the caller's device arrays; the state
                               trajectory, element arithmetic and solver vectors are
                               always FP64                                              */
  double cg_tol;            /* stop at ||r||_2 <= cg_tol * ||b||_2 (relative residual)  */
  int32_t cg_max_iter;      /* cap per solve                                            */
  int32_t checkpoint_every; /* k > 0: keep every k-th state, recompute in the adjoint;
                               0: keep every state                                      */
  double gravity[3];        /* m/s^2                                                    */
  int32_t max_steps;        /* capacity: longest rollout this handle will run           */
  int32_t rows_per_block;   /* solver rows per workgroup, a multiple of 16 from 64 to
                               256; 0 = the library's choice (rule or autotuner). With
                               a coarse space a workgroup may overlap at most four
                               aggregates (so at most 4 x their size rows), else
                               sim_create fails with SIM_E_INVALID                      */
  int32_t membrane_system;  /* sim_membrane_system                                      */
  int32_t matrix_precision; /* sim_precision of the stored system matrix and its
                               block-Jacobi inverse (default SIM_FP64; SIM_FP32 halves
                               the solver's operand but bounds the solution's relative
                               accuracy near cond(A) * 6e-8)                            */
  int32_t coarse_size;      /* vertices per aggregate of the solver's coarse space
                               (default 64; 0 = block-Jacobi preconditioner only).
                               The preconditioner adds P A_c^-1 P^T, where P holds the
                               six rigid motions of every aggregate of nearby vertices
                               and A_c = P^T A P is inverted per step; a sheet with
                               more than 320 aggregates uses larger ones. The solution
                               still meets cg_tol on the true residual. Each step's
                               operators (FP32 A_c^-1, offsets, 6x6 blocks) are kept
                               for the adjoint: without checkpointing for every step
                               when that fits 16 GB, else not at all (rebuilt in the
                               adjoint); with checkpointing see coarse_keep_all       */
  int32_t autotune;         /* 1: sim_create times every feasible solver launch shape
                               (rows per workgroup; matrix rows in registers, on one or
                               two wavefront teams, in LDS or streamed; rows of the
                               coarse inverse in LDS or streamed; one or two workgroups
                               per CU) on the step system of the rest state and keeps
                               the fastest; 0 (default): fewest co-resident launches,
                               then the matrix homes in the order registers (two teams
                               first), LDS, streamed, then larger workgroups           */
  int32_t graph;            /* 1: sim_rollout and sim_adjoint capture their launches
                               into a HIP graph (on a stream of the handle) and launch
                               it on the caller's stream; a later call with the same
                               pointers, step count and loss frames replays it (the
                               arrays' contents may change). Ignored while solver
                               timing is on. 0 (default): direct launches              */
  int32_t matrix_home;      /* sim_matrix_home (default SIM_MATRIX_AUTO)                */
  double air_density;       /* rho_air [kg/m^3] of the aerodynamic force (default 1, the
                               value the paper fixes, Sec. 3.4); it acts only in
                               rollouts given a wind velocity                           */
  int32_t coarse_keep_all;  /* with checkpointing: 0 (default) keeps the coarse
                               operators of one checkpoint segment (device memory
                               bounded by checkpoint_every; recomputed steps rebuild
                               theirs), 1 keeps every step's when they fit 16 GB (the
                               recompute then reuses the forward's: faster, more memory) */
  int32_t material_model;   /* sim_material_model (default SIM_MATERIAL_ISOTROPIC): sets
                               the material arrays' n_mat (3 or SIM_WANG_PARAMS)        */
} sim_options;

/* Per-handle statistics of the most recent rollout/adjoint (filled by
 * sim_get_stats after sim_sync_status). */
typedef struct {
  int32_t n_steps;
  int32_t n_instances;
  int64_t cg_iters_forward;   /* summed over steps and instances */
  int64_t cg_iters_recompute; /* forward solves repeated by checkpoint recompute */
  int64_t cg_iters_adjoint;
  int32_t cg_iters_max;       /* largest single solve */
  double max_rel_residual;    /* largest final ||r||/||b|| of any solve (the true
                                 residual ||b - A Delta v|| unless a solve stopped at
                                 cg_max_iter: then the recursive estimate) */
  int32_t device_status;      /* sticky device status (sim_status value) */
  int32_t rows_per_block;     /* solver launch shape in use */
  int32_t blocks;             /* solver workgroups per launch */
  int32_t solver_matrix_home; /* sim_matrix_home of the launch shape in use (never AUTO) */
  int32_t solver_launches_per_solve; /* batches split into sets of co-resident sheets */
  int64_t nnz_blocks;         /* non-zero 3x3 blocks of the system matrix */
  int64_t solver_launches;    /* timed solver launches since timing was enabled */
  double solver_ms;           /* their summed duration (HIP events on the call's stream) */
  int32_t coarse_aggregates;  /* aggregates of the coarse space over all sheets (0: none) */
  int32_t coarse_max_dim;     /* largest per-sheet coarse dimension (6 x aggregates) */
  int32_t autotuned;          /* 1: the launch shape was chosen by measurement */
  int32_t autotune_candidates;/* feasible launch shapes */
  double autotune_ms_per_iter;/* measured time per CG iteration of the chosen shape */
  int32_t solver_wg_per_cu;   /* solver variant: 1 or 2 workgroups per CU */
  int32_t coarse_rows_lds;    /* 1: the solver keeps its rows of the coarse inverse in LDS */
  int64_t graph_captures;     /* rollout / adjoint graphs captured (graph option) */
  int64_t graph_replays;      /* calls served by replaying a captured graph */
  int64_t device_bytes;       /* device memory the handle holds (workspace, trajectory or
                                 checkpoints, kept coarse operators, tables) */
  int32_t coarse_store_slots; /* steps whose coarse operators are kept for the adjoint */
  int32_t material_params;    /* n_mat of the material arrays (3 or SIM_WANG_PARAMS) */
  int32_t solver_row_teams;   /* 2: register-resident rows split over two wavefront teams
                                 (workgroups of at most 128 rows), else 1 */
} sim_stats;

/* Fills *opt with the defaults: FP32 arrays, cg_tol 1e-7, cg_max_iter 20000,
 * store every state, gravity (0,0,-9.81), max_steps 1000, tuned rows per block,
 * exact membrane Hessian, FP64 system matrix, aggregates of 64 vertices, air
 * density 1 kg/m^3, coarse operators of one checkpoint segment kept, isotropic
 * material. */
void sim_default_options(sim_options* opt);

/* Creates a handle for one sheet.
 *   mesh      host triangle mesh (fixed topology, Sec. 3.1)
 *   rest_pos  host double [n_verts][3] rest (template) positions S_1
 *   pins      host vertex ids held fixed (v = 0, x = x_0); may be NULL if n_pins = 0
 *   mat       default material (used when sim_rollout gets material = NULL)
 *   dt        time step h [s]
 *   opt       options (NULL = sim_default_options)
 * Computes the rest geometry (per-triangle inverse rest frame and area, lumped
 * vertex areas, hinges with c_e and rest angles), the block sparsity pattern
 * and the element-to-block maps on the host, uploads them and allocates the
 * workspace for opt->max_steps steps. Errors: SIM_E_INVALID (bad argument),
 * SIM_E_MESH (degenerate triangle, vertex id out of range, an edge shared by
 * more than two triangles or used twice in the same direction),
 * SIM_E_NOMEM, SIM_E_HIP. *out is NULL on error. */
sim_status sim_create(const sim_mesh* mesh, const double* rest_pos, const int32_t* pins,
                      int32_t n_pins, const sim_material* mat, double dt, const sim_options* opt,
                      sim_t** out);

/* Creates a handle over n independent sheets run together (one solver launch
 * per step for all of them). Arguments are arrays of length n with the meaning
 * of sim_create's; device arrays of the handle concatenate the instances'
 * vertices in order. Same errors as sim_create. */
sim_status sim_create_batch(int32_t n, const sim_mesh* meshes, const double* const* rest_pos,
                            const int32_t* const* pins, const int32_t* n_pins,
                            const sim_material* mats, double dt, const sim_options* opt,
                            sim_t** out);

/* Rollout of n_steps steps (Eq. 1 applied n_steps times).
 *   x0, v0       device [3][V] initial state; v0 may be NULL (zero). Pinned
 *                vertices keep x0 and zero velocity.
 *   forces       device [n_steps][3][V]: forces[s-1] acts in step s; NULL = none
 *   material     device double [n_instances][n_mat] (see dtype); NULL = the
 *                create-time materials
 *   wind         device double [n_instances][3]: the wind velocity w [m/s] of each
 *                sheet (Eq. 2's w), or NULL for no aerodynamic force. Given a wind,
 *                every triangle t feels rho_air * area_t * |s| s n in the step's
 *                force, n its unit normal at x_{t-1}, area_t its rest area and
 *                s = n . (w - mean velocity of its vertices at t-1), shared equally
 *                by its vertices; its velocity Jacobian enters the step matrix
 *                (Eq. 4-5: A = M - h df/dv + h^2 K_sys; the position Jacobian of
 *                this force is left out of A, so A stays symmetric)
 *   loss_frames  host int32 [n_loss], strictly increasing, each in 1..n_steps
 *   x_out        device [n_loss][3][V]: positions after each loss frame
 *   stream       hipStream_t
 * The forces, material and wind arrays are read again by the matching
 * sim_adjoint. Errors: SIM_E_INVALID (n_steps outside 1..max_steps, bad frames,
 * NULL pointers), SIM_E_HIP. Device-side conditions: see sim_sync_status. */
sim_status sim_rollout(sim_t* sim, int32_t n_steps, const void* x0, const void* v0,
                       const void* forces, const void* material, const void* wind,
                       const int32_t* loss_frames, int32_t n_loss, void* x_out, void* stream);

/* sim_rollout for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same arguments,
 * results and errors as sim_rollout (bitwise the same outputs), and it allocates
 * nothing: the solver's exchange buffers (partial sums, tagged publications, barrier
 * counters, the global copies of the preconditioned vectors; about 136 bytes per
 * vertex plus about 1 KB per solver workgroup) live in a static device array of
 * 8 MiB that each GPU the library runs on holds until the process ends (sheets up to
 * about 60,000 vertices; larger handles get SIM_E_INVALID). Every call on one GPU
 * shares that array, so calls that overlap on one GPU (on different streams or
 * threads) race; the array keeps the last call's contents, and each solver launch
 * clears what must start at zero. Handles created with the graph option are refused
 * (SIM_E_INVALID). A later sim_adjoint works as after sim_rollout. */
sim_status sim_rollout_noalloc(sim_t* sim, int32_t n_steps, const void* x0, const void* v0,
                               const void* forces, const void* material, const void* wind,
                               const int32_t* loss_frames, int32_t n_loss, void* x_out,
                               void* stream);

/* Adjoint of the most recent rollout for a loss with gradient dl_dx
 * (device [n_loss][3][V], one slice per loss frame).
 *   dl_dmaterial  device double [n_instances][n_mat] (dL/dk_s, dL/dk_b, dL/dd, or
 *                 dL/dS, dL/dB, dL/dd) or NULL
 *   dl_dwind      device double [n_instances][3] (dL/dw) or NULL; must be NULL when
 *                 the rollout had no wind
 *   dl_dforces    device [n_steps][3][V] or NULL
 *   dl_dx0        device [3][V] or NULL
 *   dl_dv0        device [3][V] or NULL (zero on pinned vertices)
 * Errors: SIM_E_STATE (no rollout), SIM_E_INVALID, SIM_E_HIP. */
sim_status sim_adjoint(sim_t* sim, const void* dl_dx, void* dl_dmaterial, void* dl_dwind,
                       void* dl_dforces, void* dl_dx0, void* dl_dv0, void* stream);

/* Waits for the handle's last stream and returns the sticky device status
 * (SIM_OK, SIM_E_NOT_CONVERGED, SIM_E_INDEFINITE or SIM_E_NONFINITE) or a HIP
 * error; clears it for the next call. */
sim_status sim_sync_status(sim_t* sim);

/* enable != 0: bracket every solver launch with HIP events on the call's stream
 * and accumulate their durations in sim_stats (solver_launches, solver_ms) at
 * each sim_sync_status; enable = 0 stops timing and clears the totals. */
sim_status sim_set_timing(sim_t* sim, int32_t enable);

/* Copies the statistics of the most recent calls (valid after sim_sync_status). */
sim_status sim_get_stats(const sim_t* sim, sim_stats* out);

/* Per-step CG iteration counts [n_steps][n_instances] of the most recent
 * rollout (forward) and adjoint; either pointer may be NULL. Host memory. */
sim_status sim_get_cg_iters(const sim_t* sim, int32_t* forward, int32_t* adjoint);

/* Sticky device status of each instance (sim_status values) as of the last
 * sim_sync_status; out has n_instances entries. Host memory. */
sim_status sim_get_instance_status(const sim_t* sim, int32_t* out);

/* The outer optimisation of the paper (Sec. 3.3, adaptive temporal window; Sec. 3.4,
 * Adam with learning rate 1e-3) repeats rollout + adjoint over the active frames; these
 * two calls hold its device arithmetic (paper_2203_11938_amd/optimize.py drives them).
 *
 * sim_frame_loss: per frame f < n_frames and sheet b, the energy
 * E[f][b] = sum over the sheet's vertices of |x_f,i - target_f,i|^2 (the 3D stand-in
 * for the per-frame reconstruction energy), summed in FP64 in a fixed order, and its
 * gradient dl_dx = 2 (x - target) (dl_dx may be NULL).
 *   x, target   device [n_frames][3][V] in the handle's precision (caller's order)
 *   energy      device double [n_frames][n_instances]
 * Errors: SIM_E_INVALID, SIM_E_HIP. */
sim_status sim_frame_loss(sim_t* sim, int32_t n_frames, const void* x, const void* target,
                          double* energy, void* dl_dx, void* stream);

/* Lumped vertex areas (a third of the incident rest-triangle areas; the mass is the
 * density times this) in the caller's vertex order: host double [V]. */
sim_status sim_get_vertex_areas(const sim_t* sim, double* out);

/* One Adam step (Kingma and Ba 2015) on n parameters: with theta the optimised variable,
 *   m1 <- b1 m1 + (1 - b1) g,  m2 <- b2 m2 + (1 - b2) g^2,
 *   theta <- theta - lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps),
 * where the stored parameter p is theta itself, exp(theta) (log_space != 0, for
 * positive material parameters) or scale[e % period] * theta (scale != NULL, e.g. a
 * vertex's area share for forces read as loads), and g is dL/dtheta from dL/dp.
 *   param, grad  device [n], FP32 or FP64 (precision); m1, m2 device double [n]
 *   t            step number, from 1
 * Errors: SIM_E_INVALID (bad sizes or hyper-parameters, scale with log_space),
 * SIM_E_HIP. */
sim_status sim_adam_step(void* param, int32_t precision, const void* grad, double* m1, double* m2,
                         int64_t n, const double* scale, int32_t period, int32_t log_space,
                         double lr, double beta1, double beta2, double eps, int32_t t,
                         void* stream);

/* Chamfer distance between two point sets (the paper's evaluation metric, Sec. 4.2,
 * Eq. 10): Ch(G, M) = 1/|G| sum_g min_m |g - m|^2 + 1/|M| sum_m min_g |m - g|^2.
 *   g, m        device float [3][n_g], [3][n_m] points (SoA, like the simulator's state)
 *   ch          device double [1]: the result (NaN if a coordinate is not finite)
 *   d_g, i_g    device float / int32 [n_g] or NULL: each g's smallest squared distance
 *               to M and the index of the first m that attains it (ties: the smallest
 *               index); d_m, i_m the same for M into G
 *   workspace   device memory of at least sim_chamfer_workspace_bytes(n_g, n_m)
 *               bytes, owned by the caller (nothing is allocated)
 * Squared distances are formed coordinate by coordinate in FP32 and the means are
 * summed in FP64 in a fixed order: the result is deterministic. Stream-ordered on
 * `stream`. Errors: SIM_E_INVALID (NULL pointers, n_g or n_m < 1, workspace too
 * small), SIM_E_HIP. */
size_t sim_chamfer_workspace_bytes(int32_t n_g, int32_t n_m);
sim_status sim_chamfer(const float* g, int32_t n_g, const float* m, int32_t n_m, double* ch,
                       float* d_g, int32_t* i_g, float* d_m, int32_t* i_m, void* workspace,
                       size_t workspace_bytes, void* stream);

const char* sim_status_string(sim_status s);
const char* sim_last_error(const sim_t* sim);
void sim_destroy(sim_t* sim);

#ifdef __cplusplus
}
#endif

#endif /* PHISFT_SIM_H */

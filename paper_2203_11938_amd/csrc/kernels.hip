// kernels.hip -- gfx950 kernels of the differentiable cloth step (phi-SfT, Sec. 3.1).
//
// Forward step (Eq. 4 with Eq. 5, df/dv = 0), per step:
//   k_elements      per triangle: deformation gradient F, Green strain G, force and
//                   the nine 3x3 blocks of the system stiffness; per hinge: dihedral
//                   angle, its gradient, force and Gauss-Newton weight.
//   k_assemble      per vertex row (16 lanes each), atomic-free: gathers the row's
//                   blocks in a fixed order into A = M + h^2 K_sys (ELL layout, pins
//                   eliminated), the right-hand side b = h (f + M g + F_t - h K_sys v)
//                   and the inverse of the diagonal block.
//   coarse set-up   aggregate frames, A_c = P^T A P, its inverse by a blocked
//                   symmetric sweep, the FP32 copy; the 6x6 blocks of the middle level.
//   k_pcg           persistent preconditioned pipelined CG: every workgroup owns a
//                   row range, keeps its vectors in FP64 registers (matrix rows in
//                   registers, in LDS or streamed; register rows of small workgroups
//                   split over two wavefront teams that each multiply half of every
//                   row's blocks); per iteration the workgroups of one sheet
//                   exchange their partial sums (tagged words, or a counter barrier
//                   on large sheets) and publish the preconditioned vector as tagged
//                   words that each workgroup polls for its halo only (reductions
//                   are fixed-order, so results are bitwise reproducible).
//   k_update        v_t = v_{t-1} + dv, x_t = x_{t-1} + h v_t, pins held.
// Adjoint step (implicit differentiation of Eq. 4): k_adj_pre, the same assembly and
// solver (A is symmetric), k_adj_elements (element vector-Jacobian products) and
// k_adj_rows; k_material_sum reduces the material gradient.
//
// The state trajectory (x, v), element arithmetic and solver vectors are FP64 in
// every precision mode; T (float or double) is the type of the system matrix, its
// block-Jacobi inverse and the caller's input/output arrays.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "kernels.h"
#include "sim_internal.h"

// Solver exchange buffers of the allocation-free rollout (partial sums, tagged
// publications, barrier counters, the preconditioned vectors' global copies). Host
// code never passes this name to a kernel: it is a host-side stand-in, and kernels
// get the device address that noalloc_scratch looks up per device.
static __device__ __align__(256) unsigned char scratch[phisft::kNoAllocScratchBytes];

namespace phisft {

// ------------------------------------------------------------------ helpers
// Lane exchanges without the LDS crossbar: the partner of lane l differs from l in bit
// O (and, for O = 4, 8, in the lower bits too), which is all a butterfly or a
// recursive halving needs. O = 8, 4: DPP row mirror / half mirror (l <-> 15 - l,
// l <-> 7 - l within each 16 / 8 lanes); O = 2, 1: DPP quad permutations. Steps
// across bits 5 and 4 use the gfx950 permlane swaps directly (swap_sum). Every lane
// of the wavefront must be active.
template <int O>
__device__ __forceinline__ int exch_i(int v, int lane) {
  if constexpr (O == 8) {
    return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);   // row_mirror
  } else if constexpr (O == 4) {
    return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);   // row_half_mirror
  } else if constexpr (O == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);    // quad_perm [2,3,0,1]
  } else {
    static_assert(O == 1, "exchange distance");
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);    // quad_perm [1,0,3,2]
  }
}

template <int O>
__device__ __forceinline__ double exch(double v, int lane) {
  int2 t = *reinterpret_cast<int2*>(&v);
  t.x = exch_i<O>(t.x, lane);
  t.y = exch_i<O>(t.y, lane);
  return *reinterpret_cast<double*>(&t);
}

// One step of a pairwise sum across lane bit O = 32 or 16 with a permlane swap of
// a (kept by the lanes whose bit O is clear) and b (kept by the others): the swap
// leaves, in every lane, its own kept value in one result and its partner's copy of
// the same value in the other, so their sum is the pair's sum with no lane selects
// (the two lanes of a pair add in opposite orders, which rounds identically).
template <int O>
__device__ __forceinline__ double swap_sum(double a, double b) {
  static_assert(O == 32 || O == 16, "permlane swap distance");
  const int2 x = *reinterpret_cast<int2*>(&a), y = *reinterpret_cast<int2*>(&b);
  int2 p, q;
  if constexpr (O == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(x.x, y.x, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(x.y, y.y, false, false);
    p = make_int2(lo[0], hi[0]);
    q = make_int2(lo[1], hi[1]);
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(x.x, y.x, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(x.y, y.y, false, false);
    p = make_int2(lo[0], hi[0]);
    q = make_int2(lo[1], hi[1]);
  }
  return *reinterpret_cast<double*>(&p) + *reinterpret_cast<double*>(&q);
}

__device__ __forceinline__ double wave_sum(double v) {
  // butterfly: every lane ends with the same, order-fixed sum (each step adds two
  // copies in either order, which rounds identically)
  const int lane = threadIdx.x & 63;
  v = swap_sum<32>(v, v);
  v = swap_sum<16>(v, v);
  v += exch<8>(v, lane);
  v += exch<4>(v, lane);
  v += exch<2>(v, lane);
  v += exch<1>(v, lane);
  return v;
}

// Sums of NP values over the 64 lanes of a wavefront by recursive halving: at each
// step a lane keeps one half of its values and adds its partner's copy of that half,
// so lane l ends with the total of value l >> (6 - log2 NP) (fixed order, NP - 1 +
// log2(64 / NP) shuffles instead of 6 NP for one butterfly per value).
template <int H, int O, int NP>
__device__ __forceinline__ void halve_step(double (&v)[NP], int lane) {
  if constexpr (H >= 1) {
    if constexpr (O >= 16) {
      // lanes with bit O clear keep v[k], the others v[k + H]
#pragma unroll
      for (int k = 0; k < H; ++k) v[k] = swap_sum<O>(v[k], v[k + H]);
    } else {
      const bool up = (lane & O) != 0;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const double send = up ? v[k] : v[k + H];
        const double keep = up ? v[k + H] : v[k];
        v[k] = keep + exch<O>(send, lane);
      }
    }
    halve_step<H / 2, O / 2, NP>(v, lane);
  }
}

template <int NP>
__device__ __forceinline__ double wave_sums_scatter(double (&v)[NP], int lane) {
  halve_step<NP / 2, 32, NP>(v, lane);
  double t = v[0];
  if constexpr (32 / NP >= 16) t = swap_sum<16>(t, t);
  if constexpr (32 / NP >= 8) t += exch<8>(t, lane);
  if constexpr (32 / NP >= 4) t += exch<4>(t, lane);
  if constexpr (32 / NP >= 2) t += exch<2>(t, lane);
  if constexpr (32 / NP >= 1) t += exch<1>(t, lane);
  return t;
}


// status[0]: handle-wide word, status[1 + inst]: the instance's word
__device__ __forceinline__ void set_status(int* status, int inst, int bits) {
  __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_or(status + 1 + inst, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool finite3(const double* a) {
  return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]);
}

// forward-mode dual number (value, directional derivative)
struct dual {
  double v, d;
  __device__ dual() : v(0.0), d(0.0) {}
  __device__ dual(double a) : v(a), d(0.0) {}
  __device__ dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ dual operator+(dual a, dual b) { return dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ dual operator-(dual a, dual b) { return dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ dual operator-(dual a) { return dual(-a.v, -a.d); }
__device__ __forceinline__ dual operator*(dual a, dual b) {
  return dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
__device__ __forceinline__ dual operator/(dual a, dual b) {
  double q = a.v / b.v;
  return dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ dual dsqrt(dual a) {
  double s = sqrt(a.v);
  return dual(s, 0.5 * a.d / s);
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }

// ------------------------------------------------------------ element math
// Triangle (a, b, c) with per-vertex weights w_i (F = sum_i x_i w_i^T):
// w_b = first row of B, w_c = second row, w_a = -(w_b + w_c).
struct Tri {
  double F[3][2];
  double G[2][2];
  double w[3][2];
  double area;
};

__device__ __forceinline__ void tri_load(const Mesh& m, const double* __restrict__ x, int t, Tri& s,
                                         int v[3]) {
  const int nt = m.nt, nv = m.nv;
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = m.tri_v[a * nt + t];
  double B00 = m.tri_B[t], B01 = m.tri_B[nt + t], B10 = m.tri_B[2 * nt + t],
         B11 = m.tri_B[3 * nt + t];
  s.w[1][0] = B00;
  s.w[1][1] = B01;
  s.w[2][0] = B10;
  s.w[2][1] = B11;
  s.w[0][0] = -(B00 + B10);
  s.w[0][1] = -(B01 + B11);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double xa = x[r * nv + v[0]];
    double d1 = x[r * nv + v[1]] - xa;
    double d2 = x[r * nv + v[2]] - xa;
    s.F[r][0] = d1 * B00 + d2 * B10;
    s.F[r][1] = d1 * B01 + d2 * B11;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
      s.G[a][b] = 0.5 * (s.F[0][a] * s.F[0][b] + s.F[1][a] * s.F[1][b] + s.F[2][a] * s.F[2][b] -
                         (a == b ? 1.0 : 0.0));
  s.area = m.tri_area[t];
}

// Spectral split of the symmetric strain: eigenvalues l1 >= l2 and the rotation
// (cs, sn) whose first column is the eigenvector of l1.
struct Eig2 {
  double l1, l2, cs, sn;
};
__device__ __forceinline__ Eig2 eig2(const double G[2][2]) {
  double m = 0.5 * (G[0][0] + G[1][1]);
  double hd = 0.5 * (G[0][0] - G[1][1]);
  double b = 0.5 * (G[0][1] + G[1][0]);
  double r = hypot(hd, b);
  double phi = 0.5 * atan2(b, hd);
  Eig2 e;
  e.l1 = m + r;
  e.l2 = m - r;
  e.cs = cos(phi);
  e.sn = sin(phi);
  return e;
}

// X' = R^T X R and X = R X' R^T for the eigenbasis rotation.
__device__ __forceinline__ void to_eig(const Eig2& e, const double X[2][2], double Y[2][2]) {
  double c = e.cs, s = e.sn;
  double a = X[0][0], b = 0.5 * (X[0][1] + X[1][0]), d = X[1][1];
  Y[0][0] = c * c * a + 2.0 * c * s * b + s * s * d;
  Y[1][1] = s * s * a - 2.0 * c * s * b + c * c * d;
  Y[0][1] = Y[1][0] = -c * s * a + (c * c - s * s) * b + c * s * d;
}
__device__ __forceinline__ void from_eig(const Eig2& e, const double Y[2][2], double X[2][2]) {
  double c = e.cs, s = e.sn;
  double a = Y[0][0], b = Y[0][1], d = Y[1][1];
  X[0][0] = c * c * a - 2.0 * c * s * b + s * s * d;
  X[1][1] = s * s * a + 2.0 * c * s * b + c * c * d;
  X[0][1] = X[1][0] = c * s * a + (c * c - s * s) * b - c * s * d;
}

// Tension part G+ (compressive principal strains clamped to zero).
__device__ __forceinline__ void tension(const Eig2& e, double Gp[2][2]) {
  double Y[2][2] = {{e.l1 > 0.0 ? e.l1 : 0.0, 0.0}, {0.0, e.l2 > 0.0 ? e.l2 : 0.0}};
  from_eig(e, Y, Gp);
}

// Directional derivative of G -> G+ along the symmetric S (Daleckii-Krein):
// in the eigenbasis, entry (k,l) is scaled by the divided difference of max(., 0).
__device__ __forceinline__ void tension_deriv(const Eig2& e, const double S[2][2],
                                              double Y[2][2]) {
  double Sp[2][2], Yp[2][2];
  to_eig(e, S, Sp);
  double d1 = e.l1 > 0.0 ? 1.0 : 0.0, d2 = e.l2 > 0.0 ? 1.0 : 0.0;
  double gap = e.l1 - e.l2;
  double f12 = gap > 0.0 ? ((e.l1 > 0.0 ? e.l1 : 0.0) - (e.l2 > 0.0 ? e.l2 : 0.0)) / gap : d1;
  Yp[0][0] = d1 * Sp[0][0];
  Yp[1][1] = d2 * Sp[1][1];
  Yp[0][1] = Yp[1][0] = f12 * Sp[0][1];
  from_eig(e, Yp, Y);
}

// Dihedral angle gradient of hinge (x0, x1 | x2, x3) (Bridson et al. 2003):
// wings -|e| n_k / |n_k|^2, edge vertices by the lever rule along the edge.
template <typename S>
__device__ __forceinline__ void hinge_grad(const S X[4][3], S g[4][3]) {
  S e[3], a[3], d[3], me[3], n1[3], n2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    e[k] = X[1][k] - X[0][k];
    a[k] = X[2][k] - X[0][k];
    me[k] = X[0][k] - X[1][k];
    d[k] = X[3][k] - X[1][k];
  }
  n1[0] = e[1] * a[2] - e[2] * a[1];
  n1[1] = e[2] * a[0] - e[0] * a[2];
  n1[2] = e[0] * a[1] - e[1] * a[0];
  n2[0] = me[1] * d[2] - me[2] * d[1];
  n2[1] = me[2] * d[0] - me[0] * d[2];
  n2[2] = me[0] * d[1] - me[1] * d[0];
  S ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  S le = dsqrt(ee);
  S q1 = n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2];
  S q2 = n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2];
  S t1 = (a[0] * e[0] + a[1] * e[1] + a[2] * e[2]) / ee;
  S t2 = ((X[3][0] - X[0][0]) * e[0] + (X[3][1] - X[0][1]) * e[1] + (X[3][2] - X[0][2]) * e[2]) / ee;
  S s1 = le / q1, s2 = le / q2;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    S w2 = -(s1 * n1[k]);
    S w3 = -(s2 * n2[k]);
    g[2][k] = w2;
    g[3][k] = w3;
    g[0][k] = -((S(1.0) - t1) * w2) - (S(1.0) - t2) * w3;
    g[1][k] = -(t1 * w2) - t2 * w3;
  }
}

__device__ __forceinline__ double hinge_theta(const double X[4][3]) {
  double e[3], a[3], d[3], me[3], n1[3], n2[3], c[3];
  for (int k = 0; k < 3; ++k) {
    e[k] = X[1][k] - X[0][k];
    a[k] = X[2][k] - X[0][k];
    me[k] = X[0][k] - X[1][k];
    d[k] = X[3][k] - X[1][k];
  }
  n1[0] = e[1] * a[2] - e[2] * a[1];
  n1[1] = e[2] * a[0] - e[0] * a[2];
  n1[2] = e[0] * a[1] - e[1] * a[0];
  n2[0] = me[1] * d[2] - me[2] * d[1];
  n2[1] = me[2] * d[0] - me[0] * d[2];
  n2[2] = me[0] * d[1] - me[1] * d[0];
  c[0] = n1[1] * n2[2] - n1[2] * n2[1];
  c[1] = n1[2] * n2[0] - n1[0] * n2[2];
  c[2] = n1[0] * n2[1] - n1[1] * n2[0];
  double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  // atan2 is invariant to the common positive scale |n1| |n2|
  double sn = (c[0] * e[0] + c[1] * e[1] + c[2] * e[2]) / le;
  double cs = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
  return atan2(sn, cs);
}

__device__ __forceinline__ void hinge_load(const Mesh& m, const double* __restrict__ x, int e,
                                           int v[4], double X[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    v[a] = m.hin_v[a * m.nh + e];
#pragma unroll
    for (int k = 0; k < 3; ++k) X[a][k] = x[k * m.nv + v[a]];
  }
}

// Aerodynamic force of a triangle with vertices at xa, xa + e1, xa + e2 for a wind
// relative to its mean vertex velocity rel: unit normal n, s = n . rel, and its
// |N| = 2 x deformed area.
__device__ __forceinline__ void wind_frame(const double e1[3], const double e2[3],
                                           const double rel[3], double n[3], double& sn,
                                           double& ln) {
  const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
  ln = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] = N[k] / ln;
  sn = n[0] * rel[0] + n[1] * rel[1] + n[2] * rel[2];
}

// ------------------------------------------------------ forward: elements
// Threads [0, nt) take triangles, [nt, nt + nh) hinges. With a wind (wind != nullptr,
// the sheets' velocities w), every triangle also gets its aerodynamic force
// rho area |s| s n (n its unit normal at x, s = n . (w - its mean vertex velocity at v),
// area its rest area), a third to each vertex, and the factor c = 2 rho area |s| / 9 of
// its damping blocks: every 3x3 block of its -df/dv is c n n^T.
// ------------------------------------------ anisotropic strain-dependent material
// Piecewise-linear responses: stiffness k_j on segment j of the deformation measure t,
// breaks at 0, 0.25, 0.5, 1, 2, 4 % strain (stretch) and 0, 0.05, 0.1, 0.2, 0.4 rad
// (bending), the last segment open. sigma(t) = sum_j k_j part_j(t), part_j(t) the length
// of [0, t] inside segment j (also d sigma / d k_j); the stiffness at t is k of t's
// segment.
template <bool STRAIN>
__device__ __forceinline__ double wang_break(int j) {
  if constexpr (STRAIN)
    return j == 0 ? 0.0 : j == 1 ? 0.0025 : j == 2 ? 0.005 : j == 3 ? 0.01 : j == 4 ? 0.02 : 0.04;
  else
    return j == 0 ? 0.0 : j == 1 ? 0.05 : j == 2 ? 0.1 : j == 3 ? 0.2 : 0.4;
}

template <int N, bool STRAIN>
__device__ __forceinline__ double seg_part(int j, double t) {
  const double d = t - wang_break<STRAIN>(j);
  if (d <= 0.0) return 0.0;
  return j == N - 1 ? d : fmin(d, wang_break<STRAIN>(j + 1) - wang_break<STRAIN>(j));
}

template <int N, bool STRAIN>
__device__ __forceinline__ int seg_of(double t) {
  int j = 0;
#pragma unroll
  for (int q = 1; q < N; ++q) j = t >= wang_break<STRAIN>(q) ? q : j;
  return j;
}

// N : X for a symmetric measure tensor stored as (N_00, N_01, N_11).
__device__ __forceinline__ double ncon(const double N[3], const double X[2][2]) {
  return N[0] * X[0][0] + N[1] * (X[0][1] + X[1][0]) + N[2] * X[1][1];
}

// Stretch response of a triangle (anisotropic material): the second Piola stress Sg =
// sum_k sgn(s_k) sigma_k(|s_k|) N_k of the strain G, each measure's s_k and segment
// stiffness c_k. Stretch table St [4][6].
__device__ __forceinline__ void wang_stretch(const double N[4][3], const double* St,
                                             const double G[2][2], double Sg[2][2],
                                             double sk[4], double c[4]) {
  Sg[0][0] = Sg[0][1] = Sg[1][0] = Sg[1][1] = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    sk[k] = ncon(N[k], G);
    const double t = fabs(sk[k]);
    double sig = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) sig += St[6 * k + j] * seg_part<6, true>(j, t);
    c[k] = St[6 * k + seg_of<6, true>(t)];
    const double sg = sk[k] < 0.0 ? -sig : sig;
    Sg[0][0] += sg * N[k][0];
    Sg[0][1] += sg * N[k][1];
    Sg[1][0] += sg * N[k][1];
    Sg[1][1] += sg * N[k][2];
  }
}

// Bending response of hinge e at the angle change dth: sc = dE/dtheta, w =
// d^2E/dtheta^2 (isotropic: 2 k_b c_e dth and 2 k_b c_e).
template <bool WANG>
__device__ __forceinline__ void hinge_response(const Mesh& m, const double* mat, int e, double dth,
                                               double& sc, double& w) {
  const int inst = m.hin_inst[e];
  const double ce = m.hin_ce[e];
  if constexpr (!WANG) {
    w = 2.0 * mat[m.matn * inst + 1] * ce;
    sc = w * dth;
    return;
  }
  const double* Bt = mat + m.matn * inst + kWangStretch;
  const double d0 = m.hin_dw[e], d1 = m.hin_dw[m.nh + e], d2 = m.hin_dw[2 * m.nh + e];
  const double t = fabs(dth);
  const int sj = seg_of<5, false>(t);
  double sig = 0.0, kt = 0.0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const double kj = d0 * Bt[j] + d1 * Bt[5 + j] + d2 * Bt[10 + j];
    sig += kj * seg_part<5, false>(j, t);
    kt = j == sj ? kj : kt;
  }
  sc = 2.0 * ce * (dth < 0.0 ? -sig : sig);
  w = 2.0 * ce * kt;
}

__device__ __forceinline__ void load_measures(const Mesh& m, int t, double N[4][3]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int q = 0; q < 3; ++q) N[k][q] = m.tri_N[(3 * k + q) * m.nt + t];
}

template <bool WANG>
__global__ void __launch_bounds__(256) k_elements(Mesh m, Elem el, const double* __restrict__ x,
                                                  const double* __restrict__ vel,
                                                  const double* __restrict__ mat,
                                                  const double* __restrict__ wind, double rho,
                                                  int* status) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < m.nt) {
    const int t = gid, nt = m.nt;
    Tri s;
    int v[3];
    tri_load(m, x, t, s, v);
    const int inst = m.tri_inst[t];
    if constexpr (WANG) {
      // anisotropic stretch: f_i = -A F Sg w_i,
      // K_ij = A [ (w_i^T Sg w_j) I + sum_k c_k (F N_k w_i)(F N_k w_j)^T ]
      double N[4][3], Sg[2][2], sk[4], c[4];
      load_measures(m, t, N);
      wang_stretch(N, mat + m.matn * inst, s.G, Sg, sk, c);
      bool okw = true;
      double FNw[4][3][3];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double n0 = N[k][0] * s.w[i][0] + N[k][1] * s.w[i][1];
          const double n1 = N[k][1] * s.w[i][0] + N[k][2] * s.w[i][1];
#pragma unroll
          for (int r = 0; r < 3; ++r) FNw[k][i][r] = s.F[r][0] * n0 + s.F[r][1] * n1;
        }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double sw0 = Sg[0][0] * s.w[i][0] + Sg[0][1] * s.w[i][1];
        const double sw1 = Sg[1][0] * s.w[i][0] + Sg[1][1] * s.w[i][1];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double f = -s.area * (s.F[r][0] * sw0 + s.F[r][1] * sw1);
          okw = okw && isfinite(f);
          el.tri_f[(i * 3 + r) * nt + t] = f;
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double gij = s.w[i][0] * (Sg[0][0] * s.w[j][0] + Sg[0][1] * s.w[j][1]) +
                             s.w[i][1] * (Sg[1][0] * s.w[j][0] + Sg[1][1] * s.w[j][1]);
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              double k = r == q ? gij : 0.0;
#pragma unroll
              for (int a = 0; a < 4; ++a) k += c[a] * FNw[a][i][r] * FNw[a][j][q];
              el.tri_K[((i * 3 + j) * 9 + r * 3 + q) * nt + t] = s.area * k;
            }
        }
      if (!okw) set_status(status, inst, ST_NONFINITE);
    } else {
      double ak = s.area * mat[m.matn * inst + 0];
      // stress term of the system block: G itself (exact Hessian) or its tension part
      double Gp[2][2];
      if (m.tension) {
        tension(eig2(s.G), Gp);
      } else {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) Gp[p][q] = s.G[p][q];
      }
      double aw[3][3];  // a_i = F w_i
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < 3; ++r) aw[i][r] = s.F[r][0] * s.w[i][0] + s.F[r][1] * s.w[i][1];
      bool ok = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double gw0 = s.G[0][0] * s.w[i][0] + s.G[0][1] * s.w[i][1];
        double gw1 = s.G[1][0] * s.w[i][0] + s.G[1][1] * s.w[i][1];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double f = -ak * (s.F[r][0] * gw0 + s.F[r][1] * gw1);
          ok = ok && isfinite(f);
          el.tri_f[(i * 3 + r) * nt + t] = f;
        }
      }
      double FF[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) FF[r][c] = s.F[r][0] * s.F[c][0] + s.F[r][1] * s.F[c][1];
      // K_ij = area k_s [ (w_i^T G' w_j) I + 1/2 (w_i . w_j) F F^T + 1/2 (F w_j)(F w_i)^T ]
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double gij = s.w[i][0] * (Gp[0][0] * s.w[j][0] + Gp[0][1] * s.w[j][1]) +
                       s.w[i][1] * (Gp[1][0] * s.w[j][0] + Gp[1][1] * s.w[j][1]);
          double cij = s.w[i][0] * s.w[j][0] + s.w[i][1] * s.w[j][1];
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              double k = ak * ((r == c ? gij : 0.0) + 0.5 * cij * FF[r][c] + 0.5 * aw[j][r] * aw[i][c]);
              el.tri_K[((i * 3 + j) * 9 + r * 3 + c) * nt + t] = k;
            }
        }
      if (!ok) set_status(status, inst, ST_NONFINITE);
    }
    bool ok = true;
    if (wind) {
      double e1[3], e2[3], rel[3], n[3], sn, ln;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double xa = x[r * m.nv + v[0]];
        e1[r] = x[r * m.nv + v[1]] - xa;
        e2[r] = x[r * m.nv + v[2]] - xa;
        rel[r] = wind[3 * inst + r] -
                 (vel[r * m.nv + v[0]] + vel[r * m.nv + v[1]] + vel[r * m.nv + v[2]]) / 3.0;
      }
      wind_frame(e1, e2, rel, n, sn, ln);
      const double ra = rho * s.area, mag = ra * fabs(sn) * sn;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        el.tri_fw[r * nt + t] = mag * n[r] / 3.0;
        el.tri_wn[r * nt + t] = n[r];
        ok = ok && isfinite(mag * n[r]);
      }
      el.tri_wn[3 * nt + t] = 2.0 * ra * fabs(sn) / 9.0;
    }
    if (!ok) set_status(status, inst, ST_NONFINITE);
  } else if (gid < m.nt + m.nh) {
    const int e = gid - m.nt, nh = m.nh;
    int v[4];
    double X[4][3], g[4][3];
    hinge_load(m, x, e, v, X);
    double th = hinge_theta(X);
    hinge_grad<double>(X, g);
    double s, w;
    hinge_response<WANG>(m, mat, e, th - m.hin_rest[e], s, w);
    bool ok = isfinite(s);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        el.hin_g[(a * 3 + k) * nh + e] = g[a][k];
        el.hin_f[(a * 3 + k) * nh + e] = -s * g[a][k];
        ok = ok && isfinite(g[a][k]);
      }
    el.hin_w[e] = w;
    if (!ok) set_status(status, m.hin_inst[e], ST_NONFINITE);
  }
}

// ----------------------------------------------------- forward: assembly
// Sum of the stiffness contributions of slot s (fixed order); with wind, also the
// triangles' damping blocks c n n^T in D.
__device__ __forceinline__ void slot_block(const Mesh& m, const Elem& el, int s, bool wind,
                                           double K[9], double D[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) K[q] = D[q] = 0.0;
  const int nt = m.nt, nh = m.nh;
  for (int c = m.slot_ptr[s]; c < m.slot_ptr[s + 1]; ++c) {
    int ref = m.slot_ref[c];
    if (ref >= 0) {
      int t = ref / 9, ab = ref - 9 * (ref / 9);
#pragma unroll
      for (int q = 0; q < 9; ++q) K[q] += el.tri_K[(ab * 9 + q) * nt + t];
      if (wind) {
        const double n[3] = {el.tri_wn[t], el.tri_wn[nt + t], el.tri_wn[2 * nt + t]};
        const double cw = el.tri_wn[3 * nt + t];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q) D[r * 3 + q] += cw * n[r] * n[q];
      }
    } else {
      int r2 = -ref - 1;
      int e = r2 >> 4, a = (r2 >> 2) & 3, b = r2 & 3;
      double w = el.hin_w[e];
      double ga[3], gb[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ga[k] = el.hin_g[(a * 3 + k) * nh + e];
        gb[k] = el.hin_g[(b * 3 + k) * nh + e];
      }
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) K[r * 3 + q] += w * ga[r] * gb[q];
    }
  }
}

__device__ __forceinline__ bool inv3(const double a[9], double o[9]) {
  double c00 = a[4] * a[8] - a[5] * a[7];
  double c01 = a[5] * a[6] - a[3] * a[8];
  double c02 = a[3] * a[7] - a[4] * a[6];
  double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
  double id = 1.0 / det;
  o[0] = c00 * id;
  o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  o[3] = c01 * id;
  o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  o[6] = c02 * id;
  o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  return true;
}

template <typename T, typename TM, int L>
__global__ void __launch_bounds__(256) k_assemble(Mesh m, Elem el, AssembleArgs<T, TM> a) {
  // L lanes per row (4, or 16 on small meshes, which would otherwise occupy few CUs),
  // each taking every L-th matrix slot and every L-th incident element; their partial
  // sums meet through lane exchanges, so every lane stays active up to there (lanes
  // past the last row work on a copy of it and store nothing). L = 4: 16 rows per
  // wavefront, lanes l, l + 16, l + 32, l + 48 share a row (two permlane swaps).
  // L = 16: 4 rows per wavefront, each one 16-lane DPP row (a butterfly within it).
  static_assert(L == 4 || L == 16, "lanes per row");
  constexpr int RW = 64 / L;   // rows per wavefront
  const int lane = threadIdx.x & 63;
  const int g = L == 4 ? lane >> 4 : lane & 15, rw = L == 4 ? lane & 15 : lane >> 4;
  const int i0 = (blockIdx.x * 4 + (int)(threadIdx.x >> 6)) * RW + rw;
  const int nv = m.nv;
  const bool live = i0 < nv;
  const int i = live ? i0 : nv - 1;
  const int inst = m.vert_inst[i];
  const double mass = a.mat[m.matn * inst + m.matn - 1] * m.varea[i];
  const bool pin_i = m.pinned[i] != 0;
  const double h = a.h, h2 = a.h * a.h;
  double kv[3] = {0.0, 0.0, 0.0};
  for (int k = g; k < m.maxnz; k += L) {
    const int s = k * nv + i;
    const int j = m.ell_col[s];
    double Ab[9];
    if (j < 0) {
#pragma unroll
      for (int q = 0; q < 9; ++q) Ab[q] = 0.0;
    } else {
      double K[9], D[9];
      slot_block(m, el, s, a.wind != 0, K, D);
      const bool pin_j = m.pinned[j] != 0;
      if (a.want_rhs && !pin_j) {
        double vj[3] = {a.v[j], a.v[nv + j], a.v[2 * nv + j]};
#pragma unroll
        for (int r = 0; r < 3; ++r) kv[r] += K[r * 3] * vj[0] + K[r * 3 + 1] * vj[1] + K[r * 3 + 2] * vj[2];
      }
      if (pin_i || pin_j) {
#pragma unroll
        for (int q = 0; q < 9; ++q) Ab[q] = (i == j && (q % 4) == 0) ? 1.0 : 0.0;
      } else {
        if (a.wind) {
#pragma unroll
          for (int q = 0; q < 9; ++q) Ab[q] = h2 * K[q] + h * D[q];
        } else {
#pragma unroll
          for (int q = 0; q < 9; ++q) Ab[q] = h2 * K[q];
        }
        if (i == j) {
          Ab[0] += mass;
          Ab[4] += mass;
          Ab[8] += mass;
        }
      }
    }
    if (live) {
#pragma unroll
      for (int q = 0; q < 9; ++q) a.A[(size_t)(k * 9 + q) * nv + i] = (TM)Ab[q];
    }
    if (j == i && live) {
      // block-Jacobi inverse of the stored (rounded) diagonal block
      double dr[9], Ji[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) dr[q] = (double)(TM)Ab[q];
      if (!inv3(dr, Ji)) {
        set_status(a.status, inst, ST_INDEFINITE);
#pragma unroll
        for (int q = 0; q < 9; ++q) Ji[q] = (q % 4) == 0 ? 1.0 : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) a.Jinv[q * nv + i] = (TM)Ji[q];
    }
  }
  if (!a.want_rhs) return;   // uniform
  double f[3] = {0.0, 0.0, 0.0};
  for (int c = m.vinc_ptr[i] + g; c < m.vinc_ptr[i + 1]; c += L) {
    int ref = m.vinc_ref[c];
    if (ref >= 0) {
      int t = ref / 3, va = ref - 3 * (ref / 3);
#pragma unroll
      for (int r = 0; r < 3; ++r) f[r] += el.tri_f[(va * 3 + r) * m.nt + t];
      if (a.wind) {
#pragma unroll
        for (int r = 0; r < 3; ++r) f[r] += el.tri_fw[r * m.nt + t];
      }
    } else {
      int r2 = -ref - 1;
      int e = r2 >> 2, va = r2 & 3;
#pragma unroll
      for (int r = 0; r < 3; ++r) f[r] += el.hin_f[(va * 3 + r) * m.nh + e];
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if constexpr (L == 16) {
      kv[r] += exch<8>(kv[r], lane);
      kv[r] += exch<4>(kv[r], lane);
      kv[r] += exch<2>(kv[r], lane);
      kv[r] += exch<1>(kv[r], lane);
      f[r] += exch<8>(f[r], lane);
      f[r] += exch<4>(f[r], lane);
      f[r] += exch<2>(f[r], lane);
      f[r] += exch<1>(f[r], lane);
    } else {
      kv[r] = swap_sum<16>(kv[r], kv[r]);
      kv[r] = swap_sum<32>(kv[r], kv[r]);
      f[r] = swap_sum<16>(f[r], f[r]);
      f[r] = swap_sum<32>(f[r], f[r]);
    }
  }
  if (g != 0 || !live) return;
  double b[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double fe = a.forces ? (double)a.forces[r * nv + m.vold[i]] : 0.0;
    b[r] = pin_i ? 0.0 : h * (f[r] + mass * a.g[r] + fe - h * kv[r]);
    a.b[r * nv + i] = b[r];
  }
  if (!finite3(b)) set_status(a.status, inst, ST_NONFINITE);
}

// ------------------------------------------------- coarse space (once per step)
// Coarse level of the preconditioner M^-1 = B^-1 + P1 B1^-1 P1^T + P A_c^-1 P^T. Per
// step: the aggregate frames at x_{t-1}, the Galerkin product A_c = P^T A P (dense per
// sheet) and its inverse by a blocked symmetric sweep. The PCG applies A_c^-1 as a
// dense product with the rows of the inverse that its workgroup needs.

// One wavefront per aggregate: centroid of the free vertices at x and the offsets
// x_i - c of its members (zero on pinned members and where rotations are unused).
__global__ void __launch_bounds__(64) k_coarse_frame(Mesh m, Coarse c, const double* __restrict__ x) {
  const int a = blockIdx.x, lane = threadIdx.x, nv = m.nv;
  const int v0 = c.agg_v0[a], v1 = c.agg_v0[a + 1];
  double s[3] = {0.0, 0.0, 0.0}, cnt = 0.0;
  for (int i = v0 + lane; i < v1; i += 64) {
    if (m.pinned[i]) continue;
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] += x[k * nv + i];
    cnt += 1.0;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = wave_sum(s[k]);
  cnt = wave_sum(cnt);
  const bool rot = c.agg_modes[a] == 6;
  for (int i = v0 + lane; i < v1; i += 64) {
    const bool use = rot && !m.pinned[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) c.crel[k * nv + i] = use ? x[k * nv + i] - s[k] / cnt : 0.0;
  }
}

// [r]x, the matrix of v -> r x v (row-major)
__device__ __forceinline__ void skew(const double r[3], double R[9]) {
  R[0] = 0.0;   R[1] = -r[2]; R[2] = r[1];
  R[3] = r[2];  R[4] = 0.0;   R[5] = -r[0];
  R[6] = -r[1]; R[7] = r[0];  R[8] = 0.0;
}

__device__ __forceinline__ void mul33(const double* A, const double* B, double* C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) C[r * 3 + q] = A[r * 3] * B[q] + A[r * 3 + 1] * B[3 + q] + A[r * 3 + 2] * B[6 + q];
}

// One 256-thread workgroup per aggregate pair (a <= b): the 6x6 block sum over its
// matrix slots of P_i^T A_ij P_j with P_i = [I | -[r_i]x], i.e.
//   [[A, -A R_j], [R_i A, -R_i A R_j]];
// written at (a, b) and, transposed, at (b, a). Unused modes give zero rows and
// columns (their unit diagonal is set by k_coarse_dead). The threads take the slots in
// turn (four wavefronts keep more of the dependent gathers in flight); each wavefront
// reduces its 36 sums together by recursive halving, then the wavefronts' sums are
// added in order.
template <typename TM>
__global__ void __launch_bounds__(256) k_coarse_assemble(Mesh m, Coarse c, const TM* __restrict__ A) {
  __shared__ double s_part[4][36];
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nv = m.nv;
  const int a = c.pair_a[p], b = c.pair_b[p];
  double acc[36];
#pragma unroll
  for (int e = 0; e < 36; ++e) acc[e] = 0.0;
  for (int t = c.pair_ptr[p] + tid; t < c.pair_ptr[p + 1]; t += 256) {
    const int s = c.pair_slot[t];
    const int k = s / nv, i = s - k * nv, j = m.ell_col[s];
    double Ab[9], Ri[9], Rj[9], AR[9], RA[9], RAR[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Ab[q] = (double)A[(size_t)(k * 9 + q) * nv + i];
    const double ri[3] = {c.crel[i], c.crel[nv + i], c.crel[2 * nv + i]};
    const double rj[3] = {c.crel[j], c.crel[nv + j], c.crel[2 * nv + j]};
    skew(ri, Ri);
    skew(rj, Rj);
    mul33(Ab, Rj, AR);
    mul33(Ri, Ab, RA);
    mul33(RA, Rj, RAR);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        acc[r * 6 + q] += Ab[r * 3 + q];
        acc[r * 6 + 3 + q] -= AR[r * 3 + q];
        acc[(3 + r) * 6 + q] += RA[r * 3 + q];
        acc[(3 + r) * 6 + 3 + q] -= RAR[r * 3 + q];
      }
  }
  double v[64];
#pragma unroll
  for (int e = 0; e < 64; ++e) v[e] = e < 36 ? acc[e] : 0.0;
  const double t = wave_sums_scatter<64>(v, lane);   // lane l holds sum l
  if (lane < 36) s_part[wave][lane] = t;
  __syncthreads();
  if (tid >= 36) return;
  const int inst = c.agg_inst[a];
  const int np = c.inst_np[inst];
  double* M = c.mat + c.inst_coff[inst];
  const int la = a - c.inst_agg0[inst], lb = b - c.inst_agg0[inst];
  const int ma = c.agg_modes[a], mb = c.agg_modes[b];
  const int r = tid / 6, q = tid % 6;
  const double sum = ((s_part[0][tid] + s_part[1][tid]) + s_part[2][tid]) + s_part[3][tid];
  const double val = (r < ma && q < mb) ? sum : 0.0;
  M[(size_t)(6 * la + r) * np + 6 * lb + q] = val;
  if (a != b) M[(size_t)(6 * lb + q) * np + 6 * la + r] = val;
}

// Middle level, one wavefront per run of kMid vertices: offsets of its members from
// the centroid of its free vertices, its 6x6 diagonal block of P1^T A P1 (the same
// block formula as the coarse operator) and that block's inverse. Unused modes get a
// zero row and column in the inverse; a block that is not positive definite gives a
// zero inverse (the run then adds nothing to the preconditioner).
template <typename TM>
__global__ void __launch_bounds__(64) k_mid_setup(Mesh m, Coarse c, const double* __restrict__ x,
                                                  const TM* __restrict__ A) {
  __shared__ double sr[3][kMid];
  const int a = blockIdx.x, lane = threadIdx.x, nv = m.nv;
  const int v0 = c.mid_v0[a], v1 = c.mid_v0[a + 1], modes = c.mid_modes[a];
  const int i = v0 + lane;
  const bool mem = lane < kMid && i < v1;
  const bool fr = mem && !m.pinned[i];
  double s3[3], cnt = wave_sum(fr ? 1.0 : 0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) s3[k] = wave_sum(fr ? x[k * nv + i] : 0.0);
  if (lane < kMid) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double r = (fr && modes == 6) ? x[k * nv + i] - s3[k] / cnt : 0.0;
      sr[k][lane] = r;
      if (mem) c.mid_crel[k * nv + i] = r;
    }
  }
  __syncthreads();
  double acc[36];
#pragma unroll
  for (int e = 0; e < 36; ++e) acc[e] = 0.0;
  for (int t = c.mid_ptr[a] + lane; t < c.mid_ptr[a + 1]; t += 64) {
    const int sl = c.mid_slot[t];
    const int k = sl / nv, ii = sl - k * nv, j = m.ell_col[sl];
    double Ab[9], Ri[9], Rj[9], AR[9], RA[9], RAR[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Ab[q] = (double)A[(size_t)(k * 9 + q) * nv + ii];
    const double ri[3] = {sr[0][ii - v0], sr[1][ii - v0], sr[2][ii - v0]};
    const double rj[3] = {sr[0][j - v0], sr[1][j - v0], sr[2][j - v0]};
    skew(ri, Ri);
    skew(rj, Rj);
    mul33(Ab, Rj, AR);
    mul33(Ri, Ab, RA);
    mul33(RA, Rj, RAR);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        acc[r * 6 + q] += Ab[r * 3 + q];
        acc[r * 6 + 3 + q] -= AR[r * 3 + q];
        acc[(3 + r) * 6 + q] += RA[r * 3 + q];
        acc[(3 + r) * 6 + 3 + q] -= RAR[r * 3 + q];
      }
  }
  // the 36 sums by recursive halving (lane l holds sum l), gathered for lane 0
  __shared__ double s_acc[36];
  {
    double v[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) v[e] = e < 36 ? acc[e] : 0.0;
    const double t = wave_sums_scatter<64>(v, lane);
    if (lane < 36) s_acc[lane] = t;
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int e = 0; e < 36; ++e) acc[e] = s_acc[e];
    // Gauss-Jordan on the used modes (SPD: no pivoting); unused modes stay zero
    double g[36];
#pragma unroll
    for (int e = 0; e < 36; ++e) g[e] = (e / 6 < modes && e % 6 < modes) ? acc[e] : 0.0;
    bool good = modes > 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      if (p < modes) {
        const double piv = g[p * 6 + p];
        if (!(piv > 0.0) || !isfinite(piv)) good = false;
        const double d = good ? 1.0 / piv : 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) g[p * 6 + j] = j == p ? d : g[p * 6 + j] * d;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          if (r == p || r >= modes) continue;
          const double f = g[r * 6 + p];
#pragma unroll
          for (int j = 0; j < 6; ++j) g[r * 6 + j] = j == p ? -f * d : g[r * 6 + j] - f * g[p * 6 + j];
        }
      }
    }
    double* out = c.mid_inv + (size_t)a * 36;
#pragma unroll
    for (int e = 0; e < 36; ++e) out[e] = good ? g[e] : 0.0;
  }
}

// Unit diagonal for the unused modes of every aggregate and for the padding rows
// of every sheet (threads past the aggregates handle the sheets, and set the sheet's
// success flag); the threads after those clear the sweep's flags.
__global__ void __launch_bounds__(256) k_coarse_dead(Coarse c, int ninst) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < c.nagg) {
    const int inst = c.agg_inst[a], np = c.inst_np[inst], la = a - c.inst_agg0[inst];
    double* M = c.mat + c.inst_coff[inst];
    for (int q = c.agg_modes[a]; q < 6; ++q) M[(size_t)(6 * la + q) * np + 6 * la + q] = 1.0;
  } else if (a < c.nagg + ninst) {
    const int inst = a - c.nagg, np = c.inst_np[inst];
    double* M = c.mat + c.inst_coff[inst];
    for (int r = c.inst_nc[inst]; r < np; ++r) M[(size_t)r * np + r] = 1.0;
    c.ok[inst] = 1;
  } else if (a < c.nagg + ninst + ninst * c.sw_stride) {
    c.sw_sync[a - c.nagg - ninst] = 0;
  }
}

// Reciprocal by Newton-Raphson refinement of the hardware estimate (two steps of
// x <- x + x (1 - a x), each squaring the relative error).
__device__ __forceinline__ double recip_nr(double a) {
  double x = __builtin_amdgcn_rcp(a);
  x = fma(x, fma(-a, x, 1.0), x);
  return fma(x, fma(-a, x, 1.0), x);
}

// In-place symmetric sweep of a 32x32 symmetric positive definite tile on one
// wavefront: for every pivot k in turn, with d = 1 / a_kk,
//   a_ij -= a_ik a_kj d (i, j != k),  a_ik = a_ik d,  a_kj = a_kj d,  a_kk = -d,
// which leaves -A^-1 and keeps every intermediate matrix symmetric. Lane l holds row
// l & 31, columns 16 (l >> 5) .. + 15. Row k of the pivot step is column k (symmetry):
// the lanes holding column k write it to s_col and every lane reads the part of it
// that its columns need (in-order LDS access within the wavefront, no barrier). No
// pivoting: every pivot of an SPD matrix is positive; false if one is not.
__device__ __forceinline__ bool gj_sweep_tile(double (&a)[16], double* s_col, int lane) {
  const int r = lane & 31, h = lane >> 5;
  bool good = true;
#pragma unroll 1
  for (int kh = 0; kh < 2; ++kh) {
#pragma unroll
    for (int kq = 0; kq < 16; ++kq) {
      const int k = 16 * kh + kq;
      if (h == kh) s_col[r] = a[kq];
      asm volatile("" ::: "memory");
      double row[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) row[q] = s_col[16 * h + q];
      const double f = s_col[r], piv = s_col[k];
      asm volatile("" ::: "memory");
      good = good && piv > 0.0 && isfinite(piv);
      const double d = recip_nr(piv);
      // one formula for every entry, s a_ij + g a_kj: off the pivot row s = 1, g = -a_ik d;
      // on it s = 0, g = d (a_kj d formed directly: the scale of the tile never enters as
      // a cancellation); column k becomes -g
      const bool pr = r == k;
      const double g = pr ? d : -f * d, sc = pr ? 0.0 : 1.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double upd = fma(g, row[q], sc * a[q]);
        a[q] = (q == kq && h == kh) ? -g : upd;
      }
      // every entry's update is formed in its own step (the compiler would otherwise
      // defer each to its next use and keep every step's row alive)
#pragma unroll
      for (int q = 0; q < 16; ++q) asm volatile("" : "+v"(a[q]));
    }
  }
  return good;
}

// 32x32 tile product X Y from LDS on the matrix cores (256 threads): wavefront w forms
// the 16x16 block (w / 2, w % 2) with eight FP64 16x16x4 MFMAs (A operand: lane l holds
// row l % 16, column l / 16 of the 16x4 slice; B operand: row l / 16, column l % 16);
// lane l's four results are the entries tile_rc(i) = (16 (w / 2) + l / 16 + 4 i,
// 16 (w % 2) + l % 16), i = 0..3.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void tile_rc(int i, int& r, int& q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  r = 16 * (w >> 1) + (lane >> 4) + 4 * i;
  q = 16 * (w & 1) + (lane & 15);
}

__device__ __forceinline__ void tile_mul_mfma(const double (*X)[kGjTile + 1],
                                              const double (*Y)[kGjTile + 1], double out[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 16 * (w >> 1), c0 = 16 * (w & 1);
  dbl4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < kGjTile; k0 += 4)
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(X[r0 + (lane & 15)][k0 + (lane >> 4)],
                                             Y[k0 + (lane >> 4)][c0 + (lane & 15)], c, 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Polls of the sweep's bounded waits (seconds, far beyond the microseconds a step takes).
constexpr int kGjSpinLimit = 1 << 22;

// Thread 0 waits (bounded) until *flag >= target; every thread returns false once the
// sheet's inversion has failed or the wait timed out (which marks it failed: the step
// then runs without its coarse correction, as after a failed pivot).
__device__ __forceinline__ bool sweep_wait(int* flag, int target, int* ok) {
  __shared__ int s_go;
  __syncthreads();
  if (threadIdx.x == 0) {
    int spins = 0, go = 1;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        go = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kGjSpinLimit) {
        __hip_atomic_store(ok, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        go = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (go && __hip_atomic_load(ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) go = 0;
    s_go = go;
  }
  __syncthreads();
  return s_go != 0;
}

// Releases everything this workgroup wrote: every wavefront's stores are written back
// (an agent-scope release per wavefront: the workgroup barrier alone does not wait for
// the other wavefronts' stores), then thread 0 moves the flag.
__device__ __forceinline__ void sweep_signal(int* flag, int value, bool add) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    if (add) __hip_atomic_fetch_add(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// 32x32 blocks written by other workgroups of the launch into LDS (all loads issued
// before any is stored), each as stored or transposed. Every block the sweep publishes
// has an address of its own, written once per launch and read only after its flag, so
// no cache of the reader can hold an older copy: ordinary (cached) loads are coherent
// here, and the readers of one chiplet share its L2 copy.
template <int NB>
__device__ __forceinline__ void sweep_load(const double* const (&src)[NB],
                                           double (*const (&dst)[NB])[kGjTile + 1],
                                           const bool (&transpose)[NB]) {
  constexpr int T = kGjTile;
  double v[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[b][k] = src[b][threadIdx.x + 256 * k];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = threadIdx.x + 256 * k, r = e / T, q = e % T;
      if (transpose[b]) dst[b][q][r] = v[b][k];
      else dst[b][r][q] = v[b][k];
    }
}

// Blocked symmetric sweep of every sheet's coarse matrix, one launch per step: the
// in-place inverse of an SPD matrix that keeps every intermediate matrix symmetric,
// so only the tiles (i, j), i <= j, are stored and updated. For each pivot tile K with
// P = M_KK^-1:
//   M_ij -= M_iK P M_Kj (i, j != K),  M_iK = M_iK P,  M_Kj = P M_Kj,  M_KK = -P,
// and after the last pivot M = -A_c^-1. Expressed with the column panel D_t = M_tK and
// C_t = D_t P (t != K): M_ij -= C_i D_j^T, M_iK = C_i, M_Kj = C_j^T.
// Each workgroup owns up to c.sw_tpw tiles of one sheet and keeps them in LDS for the
// whole sweep (read from the assembled matrix at the start; at the end A_c^-1 = -M is
// written as the solver's exactly symmetric FP32 copy). Per pivot step K:
//   1. the owner of tile (K+1, K+1) updates it with step K's panels, inverts it on one
//      wavefront (the sweep of the tile gives -P_{K+1} = its value after step K+1 at
//      once) and publishes P_{K+1};
//   2. the owners of the other tiles of row and column K+1 update them, form step
//      K+1's panels from their new values and P_{K+1}, and publish them;
//   3. every other tile is updated as soon as the two panels it needs are published.
// Each workgroup works through its tiles in that order (the longest path first).
// Pivot step 0's inverse and panels come from an initial phase. Every step's panels and
// inverse pivot tile have addresses of their own (nothing is rewritten within a launch,
// so readers need no wait beyond the flag). Sync flags per sheet, each on a cache line
// of its own (zero before the launch): pivot (1 + the last pivot step whose inverse is
// published) and per panel t (1 + the last step whose panel t is published). All waits
// are bounded; a failed pivot or a time-out sets ok = 0 and every workgroup of the
// sheet stops.
__global__ void __launch_bounds__(256) k_gj_sweep(Coarse c, int ninst, int wg0) {
  constexpr int T = kGjTile;
  extern __shared__ __align__(16) unsigned char sw_lds[];
  double (*Mt)[T][T + 1] = reinterpret_cast<double (*)[T][T + 1]>(sw_lds);
  __shared__ double X[T][T + 1], Y[T][T + 1];
  __shared__ double s_col[T];
  const int w = wg0 + blockIdx.x, tid = threadIdx.x, tpw = c.sw_tpw;
  const int inst = c.sw_inst[w];
  const int np = c.inst_np[inst], nb = np / T;
  // flags, kSwFlag ints apart: pivot, then one per panel t
  int* sync = c.sw_sync + (size_t)inst * c.sw_stride;
  int* const piv_flag = sync;
  auto panel_flag = [&](int t) { return sync + kSwFlag * (1 + t); };
  int* ok = c.ok + inst;
  const double* M = c.mat + c.inst_coff[inst];
  // step K's panels C_t, D_t at gj_c / gj_r + coff + (K nb + t) T^2, its inverse pivot
  // tile at gj_pinv + boff + K T^2
  const long long coff = c.inst_coff[inst], boff = c.inst_boff[inst];
  // the workgroup's tiles (uniform; slots past nt hold -1)
  __shared__ int ti[kSwMaxTiles], tj[kSwMaxTiles];
  if (tid < kSwMaxTiles) {
    const int ij = tid < tpw ? c.sw_ij[(size_t)w * tpw + tid] : -1;
    ti[tid] = ij < 0 ? -1 : ij >> 16;
    tj[tid] = ij < 0 ? -1 : ij & 0xffff;
  }
  __syncthreads();
  int nt = 0;
  for (int s = 0; s < kSwMaxTiles; ++s)
    if (ti[s] >= 0) nt = s + 1;
#pragma unroll 1
  for (int s = 0; s < nt; ++s) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + 256 * k, r = e / T, q = e % T;
      Mt[s][r][q] = M[(size_t)(ti[s] * T + r) * np + tj[s] * T + q];
    }
  }
  __syncthreads();

  // pivot tile K (held in slot s): sweep it in place (-P_K), publish P_K
  auto invert = [&](int s, int K) {
    __syncthreads();   // the tile's last update is complete
    if (tid < 64) {
      // the step waits for this wavefront: it goes first on its SIMD
      __builtin_amdgcn_s_setprio(3);
      double a[16];
      const int r = tid & 31, h = tid >> 5;
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = Mt[s][r][16 * h + q];
      const bool good = gj_sweep_tile(a, s_col, tid);
      double* P = c.gj_pinv + boff + (size_t)K * T * T;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        Mt[s][r][16 * h + q] = a[q];
        P[r * T + 16 * h + q] = -a[q];
      }
      if (!good && tid == 0) __hip_atomic_store(ok, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_setprio(0);
    }
    sweep_signal(piv_flag, K + 1, false);
  };
  // panel t of step K from the tile in slot s (row / column K): D_t = M_tK oriented as
  // rows of t, C_t = D_t P_K; false when the sheet's inversion stopped
  auto panel = [&](int s, int t, int K) -> bool {
    if (!sweep_wait(piv_flag, K + 1, ok)) return false;
    const bool tr = ti[s] == K;   // tile (K, t): D_t is its transpose
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + 256 * k, r = e / T, q = e % T;
      if (tr) X[q][r] = Mt[s][r][q];
      else X[r][q] = Mt[s][r][q];
    }
    {
      const double* const src[1] = {c.gj_pinv + boff + (size_t)K * T * T};
      double (*const dst[1])[T + 1] = {Y};
      const bool tr1[1] = {false};
      sweep_load<1>(src, dst, tr1);
    }
    __syncthreads();
    double o[4];
    tile_mul_mfma(X, Y, o);
    double* C = c.gj_c + coff + ((size_t)K * nb + t) * T * T;
    double* D = c.gj_r + coff + ((size_t)K * nb + t) * T * T;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int r, q;
      tile_rc(k, r, q);
      C[r * T + q] = o[k];
      const int e = tid + 256 * k;
      D[e] = X[e / T][e % T];
    }
    sweep_signal(panel_flag(t), K + 1, false);
    return true;
  };
  // step K's update of the tile in slot s
  auto update = [&](int s, int K) -> bool {
    const int i = ti[s], j = tj[s];
    const double* Cb = c.gj_c + coff + (size_t)K * nb * T * T;
    const double* Db = c.gj_r + coff + (size_t)K * nb * T * T;
    if (j == K || i == K) {   // M_iK = C_i, or M_Kj = C_j^T
      const int t = j == K ? i : j;
      if (!sweep_wait(panel_flag(t), K + 1, ok)) return false;
      const double* const src[1] = {Cb + (size_t)t * T * T};
      double (*const dst[1])[T + 1] = {Mt[s]};
      const bool tr1[1] = {i == K};
      sweep_load<1>(src, dst, tr1);
      return true;
    }
    if (!sweep_wait(panel_flag(i), K + 1, ok)) return false;
    if (j != i && !sweep_wait(panel_flag(j), K + 1, ok)) return false;
    {
      const double* const src[2] = {Cb + (size_t)i * T * T, Db + (size_t)j * T * T};
      double (*const dst[2])[T + 1] = {X, Y};
      const bool tr2[2] = {false, true};   // Y = D_j^T
      sweep_load<2>(src, dst, tr2);
    }
    __syncthreads();
    double o[4];
    tile_mul_mfma(X, Y, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int r, q;
      tile_rc(k, r, q);
      Mt[s][r][q] -= o[k];
    }
    return true;
  };

  bool go = true;
  // initial phase: pivot 0 and the panels of step 0
#pragma unroll 1
  for (int s = 0; s < nt; ++s)
    if (ti[s] == 0 && tj[s] == 0) invert(s, 0);
#pragma unroll 1
  for (int s = 0; s < nt; ++s)
    if (go && ti[s] == 0 && tj[s] > 0) go = panel(s, tj[s], 0);
  for (int K = 0; K < nb && go; ++K) {
    const int K1 = K + 1;
    // the longest path of the step first: the next pivot tile, then the tiles of its row
    // and column with step K + 1's panels, then the other tiles
    int ps = -1;
    for (int s = 0; s < nt; ++s)
      if (K1 < nb && ti[s] == K1 && tj[s] == K1) ps = s;
    if (ps >= 0) {
      go = update(ps, K);
      if (go) invert(ps, K1);
    }
#pragma unroll 1
    for (int s = 0; s < nt; ++s) {
      if (!go || K1 >= nb) break;
      if (s == ps || (ti[s] != K1 && tj[s] != K1)) continue;
      go = update(s, K);
      if (go) go = panel(s, ti[s] == K1 ? tj[s] : ti[s], K1);
    }
#pragma unroll 1
    for (int s = 0; s < nt; ++s) {
      if (!go) break;
      if (s == ps || (ti[s] == K && tj[s] == K) || (K1 < nb && (ti[s] == K1 || tj[s] == K1)))
        continue;
      go = update(s, K);
    }
  }
  // this workgroup's tiles are final: A_c^-1 = -M as the solver's FP32 copy (tiles below
  // the diagonal as transposes, diagonal tiles averaged with their transpose). A sheet
  // whose inversion stopped (ok = 0, possibly set by another workgroup meanwhile) runs
  // its solves without the copy, so a partial write is never read.
  __syncthreads();
  if (!go || __hip_atomic_load(ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  float* Xo = c.xinv + c.inst_coff[inst];
#pragma unroll 1
  for (int s = 0; s < nt; ++s) {
    const int I = ti[s], J = tj[s];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = tid + 256 * k, r = e / T, q = e % T;
      if (I == J) {
        Xo[(size_t)(I * T + r) * np + J * T + q] = (float)(-0.5 * (Mt[s][r][q] + Mt[s][q][r]));
      } else {
        Xo[(size_t)(I * T + r) * np + J * T + q] = (float)(-Mt[s][r][q]);
        Xo[(size_t)(J * T + r) * np + I * T + q] = (float)(-Mt[s][q][r]);
      }
    }
  }
}

// ------------------------------------------------------- persistent PCG
constexpr int kSpinLimit = 1 << 25;
// Cluster barrier of the workgroups of one sheet. Counters live in 128-byte slots
// of w.barrier: slot inst is the sheet's root counter; a sheet with more than
// kBarrierGroup workgroups also has per-group arrival counters and release flags
// (slots from plan.inst_grp0). Arrival is counted per group; the last arriver of a
// group adds the group to the root, waits for all groups, then releases its group.
// Every wait is bounded: a timeout sets the abort flag, which ends all waits.
struct Barrier {
  int* root;
  int* gctr;   // nullptr: flat barrier
  int* gflag;
  int ngroups;
  int gsize;   // members of this workgroup's group (flat: workgroups of the sheet)
  int epoch;
  bool released;   // thread 0: this workgroup completed its group's arrival and released it
  bool ok;         // thread 0: no time-out or abort in the arrival half
};

// Polls with relaxed agent-scope loads (they read the coherent value without cache
// maintenance). Everything another workgroup of the same launch wrote and this one
// reads after a wait (partial sums, restriction partials, halo rows) is read with
// agent-scope atomic loads as well, which are coherent on their own; so no agent
// acquire (an invalidation of this XCD's L2, which would also evict the matrix and
// coarse rows that the other workgroups on the XCD are reading) is needed, only the
// ordering of those loads after the poll: a workgroup-scope acquire (a wait for the
// poll, and a compiler barrier). The writers release with an agent-scope release
// (their stores are written back before the flag or counter moves).
__device__ __forceinline__ bool bounded_wait_ge(int* addr, int target, int* abort_flag) {
  int spins = 0;
  while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit ||
        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      return false;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return true;
}

__device__ __forceinline__ Barrier make_barrier(const SolverPlan& plan, const SolverWork& w, int inst,
                                                int wg, int iw0, int nwg) {
  Barrier b;
  b.root = w.barrier + (size_t)inst * kBarrierSlot;
  b.epoch = 0;
  if (nwg <= kBarrierGroup) {
    b.gctr = b.gflag = nullptr;
    b.ngroups = 1;
    b.gsize = nwg;
  } else {
    const int gi = (wg - iw0) / kBarrierGroup;
    b.ngroups = (nwg + kBarrierGroup - 1) / kBarrierGroup;
    b.gsize = min(kBarrierGroup, nwg - gi * kBarrierGroup);
    const int slot = plan.inst_grp0[inst] + 2 * gi;
    b.gctr = w.barrier + (size_t)slot * kBarrierSlot;
    b.gflag = w.barrier + (size_t)(slot + 1) * kBarrierSlot;
  }
  return b;
}

// Arrival half: thread 0 counts the workgroup in (a release of everything the workgroup
// wrote before it). The last arriver of a group completes the group's arrival at the
// root, waits for every group and releases its own, so the sheet's release never waits
// for work placed between the halves; every other workgroup may do work that needs
// nothing from the others before cluster_wait.
__device__ __forceinline__ void cluster_arrive(Barrier& b, int* abort_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    b.epoch += 1;
    const int e = b.epoch;
    b.released = false;
    b.ok = true;
    if (b.gctr == nullptr) {
      __hip_atomic_fetch_add(b.root, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const int old = __hip_atomic_fetch_add(b.gctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (old == e * b.gsize - 1) {  // last arriver of the group
        // acquire what the group's members released, then release it to the root
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_fetch_add(b.root, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        b.ok = bounded_wait_ge(b.root, e * b.ngroups, abort_flag);
        __hip_atomic_store(b.gflag, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        b.released = true;
      }
    }
  }
}

// Waiting half: true when every workgroup of the sheet has arrived (false on a time-out
// or an abort, after setting the abort flag and the sheet's status).
__device__ __forceinline__ bool cluster_wait(Barrier& b, int* abort_flag, int* status, int inst) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    const int e = b.epoch;
    bool ok = b.ok;
    if (b.gctr == nullptr) ok = bounded_wait_ge(b.root, e * b.gsize, abort_flag);
    else if (!b.released) ok = bounded_wait_ge(b.gflag, e, abort_flag);
    if (!ok) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      set_status(status, inst, ST_TIMEOUT);
    }
    s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ bool cluster_barrier(Barrier& b, int* abort_flag, int* status,
                                                int inst) {
  cluster_arrive(b, abort_flag);
  return cluster_wait(b, abort_flag, status, inst);
}

// Sheets with at most this many solver workgroups exchange their per-iteration partial
// sums as tagged words instead of through a cluster barrier (measured: 32 and 157
// workgroups gain). The collection reads one workgroup's partials per thread, so a
// sheet also has at most as many workgroups as a block has threads; split register
// rows collect on wavefront 0 only (at most kTagWgMaxSplit).
constexpr int kTagWgMax = 256;
constexpr int kTagWgMaxSplit = 64;

// Tagged publication of a vertex's three doubles of a row vector as four 64-bit words
// (word-major, [4][nv]: each store instruction of a wavefront fills whole cache lines),
// each holding a 16-bit tag (from the publication's number,
// the same in every workgroup of a sheet, never 0) above 48 of the 192 value bits. A
// 64-bit store is single-copy atomic, so a reader that sees the expected tag in all
// four words has the values published with it: no flag, no fence, no separate round
// trip. Words are written and read with coherent agent-scope atomics; the buffer is
// zeroed before each launch. Publications alternate between two buffers by iteration
// parity, and a workgroup cannot rewrite a word two publications later before its
// readers are done with it: in between it needs their partial sums of the next
// iteration, which they publish only after they have read (restarts pass full cluster
// barriers). So a word a reader sees is from this publication or from the one two
// before (tag 2 lower modulo 65535), which the 16-bit tag tells apart.
__device__ __forceinline__ unsigned long long vtag(unsigned pub) {
  return (unsigned long long)((pub - 1u) % 65535u + 1u) << 48;
}

constexpr unsigned long long kLow48 = (1ull << 48) - 1;

__device__ __forceinline__ void publish_tagged(unsigned long long* tb, int i, int nv,
                                               const double v[3], unsigned pub) {
  const unsigned long long t = vtag(pub);
  const unsigned long long a = (unsigned long long)__double_as_longlong(v[0]);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v[1]);
  const unsigned long long c = (unsigned long long)__double_as_longlong(v[2]);
  unsigned long long* p = tb + i;
  const size_t s = (size_t)nv;
  __hip_atomic_store(p, t | (a & kLow48), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + s, t | (a >> 48) | ((b & 0xffffffffull) << 16), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 2 * s, t | (b >> 32) | ((c & 0xffffull) << 32), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 3 * s, t | (c >> 16), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The three doubles of four words published together (tags already checked).
__device__ __forceinline__ void unpack_tagged(const unsigned long long (&w)[4], double v[3]) {
  v[0] = __longlong_as_double((long long)((w[0] & kLow48) | ((w[1] & 0xffffull) << 48)));
  v[1] = __longlong_as_double((long long)(((w[1] >> 16) & 0xffffffffull) | ((w[2] & 0xffffffffull) << 32)));
  v[2] = __longlong_as_double((long long)(((w[2] >> 32) & 0xffffull) | ((w[3] & kLow48) << 16)));
}

__device__ __forceinline__ void store_tagged(unsigned long long* p, unsigned tag, double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const unsigned long long t = (unsigned long long)tag << 32;
  __hip_atomic_store(p, t | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, t | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool tag_ok(unsigned long long w0, unsigned long long w1, unsigned tag) {
  return (unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag;
}

__device__ __forceinline__ double tag_value(unsigned long long w0, unsigned long long w1) {
  return __longlong_as_double((long long)((w1 << 32) | (w0 & 0xffffffffull)));
}

// Re-reads one tagged entry until it carries `tag` (bounded); false on a time-out or
// an abort.
__device__ __forceinline__ bool poll_tagged(const unsigned long long* p, unsigned tag,
                                            int* abort_flag, unsigned long long& w0,
                                            unsigned long long& w1) {
  unsigned long long* q = const_cast<unsigned long long*>(p);
  int spins = 0;
  while (!tag_ok(w0, w1, tag)) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit ||
        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      return false;
    w0 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    w1 = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

__device__ __forceinline__ void load_tagged(const unsigned long long* p, unsigned long long& w0,
                                            unsigned long long& w1) {
  unsigned long long* q = const_cast<unsigned long long*>(p);
  w0 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  w1 = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Halo of a tagged vector into vl[c][R + h]: every halo vertex's four words are polled
// until all carry the publication's tag (bounded like the barrier's waits). A thread's
// vertices are read kHaloBatch at a time (one with SPREAD), all loads issued before any
// is checked (one round trip per batch, not per vertex). False (every thread) on a time-out or an
// abort; the caller then stops.
constexpr int kHaloBatch = 4;
// SPREAD: vertices past the end re-read the thread's own first vertex instead of the
// last one (no single address that every thread of the sheet reads), and one vertex
// per thread per pass (a split workgroup's 256 threads cover its halo in one); kept
// for split register rows, where it measured faster
template <bool SPREAD>
__device__ __forceinline__ bool halo_load_tagged(const unsigned long long* tb, int nv,
                                                 const int* __restrict__ hidx, int nh,
                                                 double* __restrict__ vl, int R, int RH,
                                                 unsigned pub, int* abort_flag) {
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  bool ok = true;
  const unsigned long long t = vtag(pub);
  constexpr int HB = SPREAD ? 1 : kHaloBatch;
  const int nb = blockDim.x;
  for (int h0 = threadIdx.x; h0 < nh && ok; h0 += HB * nb) {
    unsigned long long w[HB][4];
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      // vertices past the end re-read another (no branches around the loads)
      const int hu = h0 + u * nb;
      unsigned long long* p = const_cast<unsigned long long*>(tb) +
                              hidx[SPREAD ? (hu < nh ? hu : h0) : min(hu, nh - 1)];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[u][k] = __hip_atomic_load(p + (size_t)k * nv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      const int h = h0 + u * nb;
      if (h >= nh) break;
      unsigned long long* p = const_cast<unsigned long long*>(tb) + hidx[h];
      int spins = 0;
      while (ok && ((w[u][0] ^ t) >> 48 | (w[u][1] ^ t) >> 48 | (w[u][2] ^ t) >> 48 |
                    (w[u][3] ^ t) >> 48) != 0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit ||
            __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          ok = false;
          break;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
          w[u][k] = __hip_atomic_load(p + (size_t)k * nv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (ok) {
        double v[3];
        unpack_tagged(w[u], v);
#pragma unroll
        for (int c = 0; c < 3; ++c) vl[c * RH + R + h] = v[c];
      }
    }
  }
  if (!ok) s_bad = 1;
  __syncthreads();
  return s_bad == 0;
}

// Fixed-order workgroup sum of three values; thread 0 stores them at dst.
__device__ __forceinline__ void publish3(const double a[3], double* dst) {
  __shared__ double s_part[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  double v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = wave_sum(a[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) s_part[k][wave] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double t = 0.0;
      for (int q = 0; q < nwaves; ++q) t += s_part[k][q];
      dst[k] = t;
    }
  }
}

// After a cluster barrier: fixed-order sum of the cluster's partials (wave 0),
// left in s_out; the caller synchronises the workgroup before reading it. Each lane
// loads up to four workgroups' partials per pass, so clusters of up to 256
// workgroups need one round trip.
__device__ __forceinline__ void collect3(const double* red_slot, int iw0, int nwg, double* s_out) {
  const int lane = threadIdx.x & 63;
  if ((threadIdx.x >> 6) != 0) return;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q0 = lane; q0 < nwg; q0 += 4 * 64) {
    double v[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double* src = red_slot + (size_t)(iw0 + min(q0 + 64 * u, nwg - 1)) * 3;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        v[u][k] = __hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k) t[k] += q0 + 64 * u < nwg ? v[u][k] : 0.0;
  }
  const double s = wave_sums_scatter<4>(t, lane);   // lane l holds sum l >> 4
  if ((lane & 15) == 0 && (lane >> 4) < 3) s_out[lane >> 4] = s;
}

#ifndef SCHED_BARRIER
#define SCHED_BARRIER 1
#endif
#ifndef GATHER_CHUNK
#define GATHER_CHUNK 8
#endif
// neighbours gathered per batch: LDS matrix (kChunk) and streamed matrix (kStreamChunk,
// whose 9 x kStreamChunk matrix loads are issued back to back before any of them is used)
constexpr int kChunk = GATHER_CHUNK;
#ifndef STREAM_CHUNK
#define STREAM_CHUNK 7
#endif
constexpr int kStreamChunk = STREAM_CHUNK;

// Gather CH of the row's neighbour values, starting at slot k0, from the workgroup's
// LDS copy vl [3][RH] of the vector: own rows at their local index, the halo
// (neighbour rows of other workgroups, loaded after the barrier) behind them. Cl holds
// those local indices. Slots past maxnz read the last one; with ZERO they contribute
// zero (the streamed product reads those slots' blocks without branches).
template <int CH, bool ZERO>
__device__ __forceinline__ void loadnb(const int* __restrict__ Cl, int R, int tid, int k0,
                                       int maxnz, const double* __restrict__ vl, int RH,
                                       double g[3][CH]) {
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int j = Cl[min(k0 + k, maxnz - 1) * R + tid];
    const bool in = !ZERO || k0 + k < maxnz;
    g[0][k] = in ? vl[j] : 0.0;
    g[1][k] = in ? vl[RH + j] : 0.0;
    g[2][k] = in ? vl[2 * RH + j] : 0.0;
  }
}

// Halo of the vector vg ([3][nv] in global memory, written by other workgroups of
// this launch; coherent agent-scope loads) into vl[c][R + h].
__device__ __forceinline__ void halo_load(const double* vg, int nv,
                                          const int* __restrict__ hidx, int nh,
                                          double* __restrict__ vl, int R, int RH) {
  for (int e = threadIdx.x; e < 3 * nh; e += blockDim.x) {
    const int c = e / nh, h = e - c * nh;
    vl[c * RH + R + h] = __hip_atomic_load(const_cast<double*>(vg) + (size_t)c * nv + hidx[h],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// y += (blocks k0..k0+CH-1 of the row) * g. The matrix is read at
// A[((k * 9 + e) * stride) + idx]: the LDS copy (stride R, idx = thread) or the
// assembled ELL array in global memory (stride nv, idx = row).
// LDS matrix (SB): scheduling barriers keep each block's LDS loads next to their use
// instead of hoisting them all into registers; slots past maxnz are skipped.
// Streamed matrix: all 9 x CH loads first (slots past maxnz re-read the last block,
// whose g is zero), then a scheduling barrier, then the products, so one round trip
// to memory serves the whole chunk whatever the register allocator does elsewhere.
template <typename TM, bool SB, int CH>
__device__ __forceinline__ void applynb(const TM* __restrict__ Am, int stride, int idx, int k0,
                                        int maxnz, const double g[3][CH], double y[3]) {
  if (SB) {
#pragma unroll
    for (int k = 0; k < CH; ++k) {
#if SCHED_BARRIER
      __builtin_amdgcn_sched_barrier(0);
#endif
      if (k0 + k < maxnz) {
        const TM* blk = Am + (size_t)(k0 + k) * 9 * stride + idx;
#pragma unroll
        for (int r = 0; r < 3; ++r)
          y[r] += (double)blk[(size_t)(r * 3) * stride] * g[0][k] +
                  (double)blk[(size_t)(r * 3 + 1) * stride] * g[1][k] +
                  (double)blk[(size_t)(r * 3 + 2) * stride] * g[2][k];
      }
    }
  } else {
    TM a[CH][9];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const TM* blk = Am + (size_t)min(k0 + k, maxnz - 1) * 9 * stride + idx;
#pragma unroll
      for (int e = 0; e < 9; ++e) a[k][e] = blk[(size_t)e * stride];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < CH; ++k)
#pragma unroll
      for (int r = 0; r < 3; ++r)
        y[r] += (double)a[k][r * 3] * g[0][k] + (double)a[k][r * 3 + 1] * g[1][k] +
                (double)a[k][r * 3 + 2] * g[2][k];
  }
}

// y = (slots kb..ke-1 of this thread's row) v, v from the workgroup's LDS copy (own
// rows + halo). CH: slots per batch of a streamed matrix (fewer when registers are
// scarce).
template <typename TM, bool SB, int SCH>
__device__ __forceinline__ void spmv_range(const TM* __restrict__ Am, int stride, int idx,
                                           const int* __restrict__ Cl, int R, int tid, int kb,
                                           int ke, const double* __restrict__ vl, int RH,
                                           double y[3]) {
  constexpr int CH = SB ? kChunk : SCH;
  y[0] = y[1] = y[2] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += CH) {
    double g[3][CH];
    loadnb<CH, !SB>(Cl, R, tid, k0, ke, vl, RH, g);
    applynb<TM, SB, CH>(Am, stride, idx, k0, ke, g, y);
  }
}

// y = A v for this thread's row: slots [0, kSpmvSplit) and [kSpmvSplit, maxnz)
// summed apart, then added.
template <typename TM, bool SB, int SCH = kStreamChunk>
__device__ __forceinline__ void spmv_row(const TM* __restrict__ Am, int stride, int idx,
                                         const int* __restrict__ Cl, int R, int tid, int maxnz,
                                         const double* __restrict__ vl, int RH, double y[3]) {
  double y2[3];
  spmv_range<TM, SB, SCH>(Am, stride, idx, Cl, R, tid, 0, min(kSpmvSplit, maxnz), vl, RH, y);
  spmv_range<TM, SB, SCH>(Am, stride, idx, Cl, R, tid, kSpmvSplit, maxnz, vl, RH, y2);
#pragma unroll
  for (int r = 0; r < 3; ++r) y[r] += y2[r];
}

// y = sum over held blocks k0..k1-1 of Ar[k] g[.][k], in slot order (the same
// operations in the same order as the streamed and LDS products).
template <typename TM, int NB>
__device__ __forceinline__ void reg_products(const TM (&Ar)[NB][9], const double g[3][NB],
                                             int k0, int k1, double y[3]) {
  y[0] = y[1] = y[2] = 0.0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k < k0 || k >= k1) continue;   // k0, k1 are compile-time after unrolling
#pragma unroll
    for (int r = 0; r < 3; ++r)
      y[r] += (double)Ar[k][r * 3] * g[0][k] + (double)Ar[k][r * 3 + 1] * g[1][k] +
              (double)Ar[k][r * 3 + 2] * g[2][k];
  }
}

// y = (slots kb..kb+NB-1 of this thread's row) v with those blocks held in registers
// (copied once per launch; slots past maxnz hold zero blocks): all NB neighbour values
// are read from LDS first (local columns Cl as for the other products; slots at or
// past ke contribute zero), then the products.
template <typename TM, int NB>
__device__ __forceinline__ void spmv_reg_range(const TM (&Ar)[NB][9], const int* __restrict__ Cl,
                                               int R, int tid, int kb, int ke,
                                               const double* __restrict__ vl, int RH,
                                               double y[3]) {
  double g[3][NB];
  loadnb<NB, true>(Cl, R, tid, kb, ke, vl, RH, g);
  reg_products<TM, NB>(Ar, g, 0, NB, y);
}

// y = A v with the whole row in registers: one gather of all its neighbour values,
// then the two slot ranges' sums, added.
template <typename TM>
__device__ __forceinline__ void spmv_reg(const TM (&Ar)[kRegRowBlocks][9],
                                         const int* __restrict__ Cl, int R, int tid, int maxnz,
                                         const double* __restrict__ vl, int RH, double y[3]) {
  double g[3][kRegRowBlocks], y2[3];
  loadnb<kRegRowBlocks, true>(Cl, R, tid, 0, maxnz, vl, RH, g);
  reg_products<TM, kRegRowBlocks>(Ar, g, 0, kSpmvSplit, y);
  reg_products<TM, kRegRowBlocks>(Ar, g, kSpmvSplit, kRegRowBlocks, y2);
#pragma unroll
  for (int r = 0; r < 3; ++r) y[r] += y2[r];
}

// Restarts from the true residual per solve; one more verifies the final iterate.
constexpr int kMaxRestarts = 16;

// Preconditioned pipelined CG (Ghysels & Vanroose 2014) from x = 0: one global
// reduction per iteration, (r,u), (w,u), (r,r), exchanged with the coarse restriction
// (tagged words, or a cluster barrier on large sheets and without a coarse space);
// then m = M^-1 w is published (tagged) for the iteration's single SpMV n = A m,
// each workgroup reading only its halo. The local part of m (block Jacobi and middle
// level) is formed while the partial sums travel, between their publication and the
// wait for the other workgroups' (the arrival and waiting halves of the barrier on
// large sheets). Vectors per row:
// x, r, u = M^-1 r, w = A u, z, q, s, p (recurrences of the method), all FP64.
// The recursively updated residual drifts from b - A x (rounding), so
// convergence is accepted only on a true residual: when the recursive residual
// meets the tolerance the recurrences restart from b - A x and the test is
// repeated. A step denominator <= 0 also triggers a restart; at a fresh start
// the denominator is u^T A u, so a non-positive value there is reported as an
// indefinite system.
// LDS: two copies of m [parity][3][rows + halo] (own rows written directly, the halo
// loaded after each publication), the rows' local columns [slot][row], the halo row
// list, and, with the matrix at home in LDS, the workgroup's matrix rows
// [slot][entry][row] (held in registers, or streamed from the assembled array in
// global memory at every product, in the other two variants); with a
// coarse space also the coarse residual, reduction scratch, the middle level's 6x6
// inverses and, when they fit, the workgroup's FP32 rows of the coarse inverse.
#ifdef PHISFT_PHASES
// per-workgroup accumulated wall-clock ticks of the solver phases (tuning builds only)
__device__ unsigned long long g_phase[512][8];
#define PHASE_T(v) const unsigned long long v = wall_clock64()
#define PHASE_ADD(k, d) ph[k] += (d)
#else
#define PHASE_T(v)
#define PHASE_ADD(k, d)
#endif

// Coarse restriction of this thread's row vector y: per-aggregate sums of
// (y, r_i x y) = P_i^T y over the workgroup's rows, published as
// part[wg][k][0..5] (k: aggregate minus the workgroup's first aggregate). Fixed
// order: a butterfly per wavefront, then the wavefronts in order.
__device__ __forceinline__ void coarse_restrict(double* __restrict__ part, int wg, int wna,
                                                int kf, int kl, int kloc, bool live,
                                                const double r[3], const double y[3]) {
  __shared__ double s_wp[4][kMaxWgAgg][6];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  for (int e = tid; e < 4 * kMaxWgAgg * 6; e += blockDim.x) (&s_wp[0][0][0])[e] = 0.0;
  double v[6];
  v[0] = y[0];
  v[1] = y[1];
  v[2] = y[2];
  v[3] = r[1] * y[2] - r[2] * y[1];
  v[4] = r[2] * y[0] - r[0] * y[2];
  v[5] = r[0] * y[1] - r[1] * y[0];
  __syncthreads();
  for (int k = kf; k <= kl; ++k) {   // this wavefront's aggregates (empty if it has no rows)
    const bool mine = live && kloc == k;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double t = wave_sum(mine ? v[q] : 0.0);
      if (lane == 0) s_wp[wave][k][q] = t;
    }
  }
  __syncthreads();
  for (int e = tid; e < wna * 6; e += blockDim.x) {
    const int k = e / 6, q = e % 6;
    double t = 0.0;
    for (int w = 0; w < nwaves; ++w) t += s_wp[w][k][q];
    part[((size_t)wg * kMaxWgAgg + k) * 6 + q] = t;
  }
}

// The iteration's publication in one pass: the coarse restriction of y (as
// coarse_restrict) and the workgroup's three dot-product partials (as publish3),
// either as tagged words that the other workgroups of the sheet poll (no barrier) or
// into the plain arrays that a cluster barrier releases. A
// wavefront whose rows lie in one aggregate (the usual case: aggregates are runs of
// whole 16-row groups) reduces its nine values together by recursive halving; one
// that spans several aggregates falls back to a butterfly per aggregate and value.
// One workgroup barrier in all.
__device__ __forceinline__ void publish_restrict_dots(bool tagged, unsigned long long* trw,
                                                      unsigned tag, double* __restrict__ part,
                                                      double* dst, int wg, int wna, int kf,
                                                      int kl, int kloc, bool live,
                                                      const double r[3], const double y[3],
                                                      const double loc[3]) {
  __shared__ double s_wp[4][kMaxWgAgg][6];
  __shared__ double s_pd[4][3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  double v[6];
  v[0] = live ? y[0] : 0.0;
  v[1] = live ? y[1] : 0.0;
  v[2] = live ? y[2] : 0.0;
  v[3] = live ? r[1] * y[2] - r[2] * y[1] : 0.0;
  v[4] = live ? r[2] * y[0] - r[0] * y[2] : 0.0;
  v[5] = live ? r[0] * y[1] - r[1] * y[0] : 0.0;
  if (kl <= kf) {   // uniform per wavefront; kl < kf: a wavefront without rows (all zero)
    const int ka = kl < kf ? 0 : kf;
    double a[16];
#pragma unroll
    for (int q = 0; q < 6; ++q) a[q] = v[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) a[6 + q] = loc[q];
#pragma unroll
    for (int q = 9; q < 16; ++q) a[q] = 0.0;
    const double t = wave_sums_scatter<16>(a, lane);   // lane l holds value l >> 2
    const int idx = lane >> 2;
    if ((lane & 3) == 0) {
      if (idx < 6) s_wp[wave][ka][idx] = t;
      else if (idx < 9) s_pd[wave][idx - 6] = t;
    }
    for (int e = lane; e < wna * 6; e += 64)
      if (e / 6 != ka) s_wp[wave][e / 6][e % 6] = 0.0;
  } else {
    for (int k = 0; k < wna; ++k) {
      const bool mine = kloc == k;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double t = wave_sum(mine ? v[q] : 0.0);
        if (lane == 0) s_wp[wave][k][q] = t;
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double t = wave_sum(loc[q]);
      if (lane == 0) s_pd[wave][q] = t;
    }
  }
  __syncthreads();
  // tagged: this workgroup's slots (the dot partials, then 6 per aggregate); else the
  // plain partial arrays read after a barrier
  if (tid < wna * 6) {
    const int k = tid / 6, q = tid % 6;
    double t = 0.0;
    for (int w = 0; w < nwaves; ++w) t += s_wp[w][k][q];
    if (tagged) store_tagged(trw + (size_t)(3 + tid) * 2, tag, t);
    else part[((size_t)wg * kMaxWgAgg + k) * 6 + q] = t;
  } else if (tid >= 32 && tid < 35) {
    double t = 0.0;
    for (int w = 0; w < nwaves; ++w) t += s_pd[w][tid - 32];
    if (tagged) store_tagged(trw + (size_t)(tid - 32) * 2, tag, t);
    else dst[tid - 32] = t;
  }
}

// Per-launch constants of a workgroup's coarse correction.
struct CoarseRow {
  const float* X;        // rows of A_c^-1 of the workgroup's aggregates (global, stride np)
  const float* XL;       // the same rows in LDS (stride nc), or nullptr
  const double* part;    // restriction partial sums
  int nc, np, nrow, ok;
  int nwm;               // most partial slots (workgroups) of any aggregate of the sheet
};

// e_q = sum_c X[q][c] w_c for the NR rows of this workgroup: the wavefronts that hold
// rows (the first of TEAMS equal teams: the partition, and so the rounding, does not
// depend on helper wavefronts) take 64-column tiles in turn, every lane accumulates
// all NR rows of its columns (NR x TU independent loads per pass), then one
// recursive-halving reduction per wavefront and a fixed-order sum over the wavefronts
// leave e in s_e[0..NR).
template <int NR, bool XLDS, int TEAMS>
__device__ __forceinline__ void coarse_rows(const float* __restrict__ X, int ld, int nc,
                                            const double* s_wc, double* s_red, double* s_e) {
  constexpr int NP = NR <= 8 ? 8 : (NR <= 16 ? 16 : 32);
  constexpr int TU = NR <= 6 ? 4 : (NR <= 12 ? 3 : 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = (int)(blockDim.x >> 6) / TEAMS;
  const bool rows = TEAMS == 1 || wave < nwaves;
  const int ntile = (nc + 63) >> 6;
  double acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = 0.0;
  for (int t0 = rows ? wave : ntile; t0 < ntile; t0 += TU * nwaves) {
    float xv[TU][NR];
    double wcv[TU];
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      // tiles past the end read the last column with weight zero (no branches)
      const int col = (t0 + u * nwaves) * 64 + lane;
      const int colc = min(col, nc - 1);
      wcv[u] = col < nc ? s_wc[colc] : 0.0;
#pragma unroll
      for (int q = 0; q < NR; ++q) xv[u][q] = X[(size_t)q * ld + colc];
    }
#pragma unroll
    for (int u = 0; u < TU; ++u)
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] += (double)xv[u][q] * wcv[u];
  }
  const double t = wave_sums_scatter<NP>(acc, lane);
  constexpr int SH = (NP == 8 ? 3 : (NP == 16 ? 2 : 1));   // 6 - log2 NP
  const int idx = lane >> SH;
  if ((lane & ((1 << SH) - 1)) == 0 && idx < NR && rows) s_red[wave * 24 + idx] = t;
  __syncthreads();
  if (tid < NR) {
    double e = 0.0;
    for (int w = 0; w < nwaves; ++w) e += s_red[w * 24 + tid];
    s_e[tid] = e;
  }
  __syncthreads();
}

template <int NR, int TEAMS>
__device__ __forceinline__ void coarse_rows_at(const CoarseRow& cr_, const double* s_wc,
                                               double* s_red, double* s_e) {
  if (cr_.XL) coarse_rows<NR, true, TEAMS>(cr_.XL, cr_.nc, cr_.nc, s_wc, s_red, s_e);
  else coarse_rows<NR, false, TEAMS>(cr_.X, cr_.np, cr_.nc, s_wc, s_red, s_e);
}

// After the partial sums are published: the sheet's coarse residual w_c into LDS.
// Every column sums its aggregate's partials in slot order, reading the NW slots an
// aggregate can have (NW: the most workgroups any aggregate of the sheet spans, a
// compile-time count so that one pass issues its loads together; slot -1 reads entry 0
// with weight 0, no branches around the loads). The caller synchronises the workgroup
// before w_c is read. Skipped when the step's inversion failed.
template <int NW>
__device__ __forceinline__ void coarse_gather_n(const CoarseRow& cr_, const int* s_pidx,
                                                double* s_wc) {
  const int tid = threadIdx.x;
  const int nc = cr_.nc;
  constexpr int CU = 8;
  for (int col0 = tid; col0 < nc; col0 += CU * blockDim.x) {
    double wc[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int col = min(col0 + u * (int)blockDim.x, nc - 1);
      const int t = col / 6, q = col - 6 * t;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int pi = s_pidx[t * kMaxAggWg + k];
        const double v = __hip_atomic_load(const_cast<double*>(cr_.part) + (size_t)max(pi, 0) * 6 + q,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc += pi >= 0 ? v : 0.0;
      }
      wc[u] = acc;
    }
#pragma unroll
    for (int u = 0; u < CU; ++u)
      if (col0 + u * (int)blockDim.x < nc) s_wc[col0 + u * blockDim.x] = wc[u];
  }
}

__device__ __forceinline__ void coarse_gather(const CoarseRow& cr_, const int* s_pidx,
                                              double* s_wc) {
  if (!cr_.ok) return;
  switch (cr_.nwm) {   // uniform
    case 1: coarse_gather_n<1>(cr_, s_pidx, s_wc); break;
    case 2: coarse_gather_n<2>(cr_, s_pidx, s_wc); break;
    case 3: coarse_gather_n<3>(cr_, s_pidx, s_wc); break;
    default: coarse_gather_n<kMaxAggWg>(cr_, s_pidx, s_wc); break;
  }
}

// Tagged counterparts of coarse_gather and collect3, reading the partials of the
// iteration's tagged publication (slot base trp = [nwg][kTagSlots][2] words): loads are
// issued together, then each entry is re-read until it carries `tag`. False on a
// time-out or an abort (per thread; the caller combines).
template <int NW, bool SPREAD>
__device__ __forceinline__ bool coarse_gather_tagged_n(const CoarseRow& cr_, const int* s_pidx,
                                                       double* s_wc,
                                                       const unsigned long long* trp,
                                                       unsigned tag, int* abort_flag) {
  const int tid = threadIdx.x;
  const int nc = cr_.nc;
  constexpr int CU = SPREAD ? 2 : 4;   // batches of blockDim columns per pass
  bool ok = true;
  for (int col0 = tid; col0 < nc; col0 += CU * blockDim.x) {
    unsigned long long w0[CU][NW], w1[CU][NW];
    const unsigned long long* adr[CU][NW];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      // columns past the end re-read another (SPREAD: the thread's first one, as for
      // halo_load_tagged)
      const int cu = col0 + u * (int)blockDim.x;
      const int col = SPREAD ? (cu < nc ? cu : col0) : min(cu, nc - 1);
      const int t = col / 6, q = col - 6 * t;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int pi = max(s_pidx[t * kMaxAggWg + k], 0);
        adr[u][k] = trp + ((size_t)(pi / kMaxWgAgg) * kTagSlots + 3 + (pi % kMaxWgAgg) * 6 + q) * 2;
        load_tagged(adr[u][k], w0[u][k], w1[u][k]);
      }
    }
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int col = col0 + u * (int)blockDim.x;
      if (col >= nc) continue;
      const int t = col / 6;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        if (s_pidx[t * kMaxAggWg + k] < 0) continue;
        ok = ok && poll_tagged(adr[u][k], tag, abort_flag, w0[u][k], w1[u][k]);
        acc += tag_value(w0[u][k], w1[u][k]);
      }
      s_wc[col] = acc;
    }
  }
  return ok;
}

template <bool SPREAD>
__device__ __forceinline__ bool coarse_gather_tagged(const CoarseRow& cr_, const int* s_pidx,
                                                     double* s_wc,
                                                     const unsigned long long* trp,
                                                     unsigned tag, int* abort_flag) {
  if (!cr_.ok) return true;
  switch (cr_.nwm) {   // uniform
    case 1: return coarse_gather_tagged_n<1, SPREAD>(cr_, s_pidx, s_wc, trp, tag, abort_flag);
    case 2: return coarse_gather_tagged_n<2, SPREAD>(cr_, s_pidx, s_wc, trp, tag, abort_flag);
    case 3: return coarse_gather_tagged_n<3, SPREAD>(cr_, s_pidx, s_wc, trp, tag, abort_flag);
    default:
      return coarse_gather_tagged_n<kMaxAggWg, SPREAD>(cr_, s_pidx, s_wc, trp, tag, abort_flag);
  }
}

// The dot partials of a tagged sheet spread over the wavefronts: wavefront w reads
// workgroup 64 w + lane (a tagged sheet has at most one workgroup per thread of the
// block), and its three sums (fixed-order lane reduction) go to s_wd[3 w + k]. After
// the caller's barrier the readers add the wavefronts' sums in order; with at most 64
// workgroups that is wavefront 0's sum alone, the same value as collect3_finish.
__device__ __forceinline__ bool collect3_waves(const unsigned long long* trp, int iw0, int nwg,
                                               double* s_wd, unsigned tag, int* abort_flag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave * 64 >= nwg) return true;   // uniform per wavefront
  const int q = wave * 64 + lane;
  unsigned long long w0[3], w1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    load_tagged(trp + ((size_t)(iw0 + min(q, nwg - 1)) * kTagSlots + k) * 2, w0[k], w1[k]);
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  bool ok = true;
  if (q < nwg) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ok = ok && poll_tagged(trp + ((size_t)(iw0 + q) * kTagSlots + k) * 2, tag, abort_flag,
                             w0[k], w1[k]);
      t[k] += tag_value(w0[k], w1[k]);
    }
  }
  const double sm = wave_sums_scatter<4>(t, lane);   // lane l holds sum l >> 4
  if ((lane & 15) == 0 && (lane >> 4) < 3) s_wd[3 * wave + (lane >> 4)] = sm;
  return ok;
}

// Wavefront 0's part of collect3_waves in two halves for split register rows
// (registers to spare; their tagged sheets have at most kTagWgMaxSplit <= 64
// workgroups): the loads are issued first (collect3_issue, so that they travel while
// the coarse columns are polled), then each is re-read until it carries the tag and
// the three sums go to s_out (collect3_finish).
static_assert(kTagWgMaxSplit <= 64, "one workgroup per lane");
__device__ __forceinline__ void collect3_issue(const unsigned long long* trp, int iw0, int nwg,
                                               unsigned long long w0[3], unsigned long long w1[3]) {
  const int q = min((int)(threadIdx.x & 63), nwg - 1);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    load_tagged(trp + ((size_t)(iw0 + q) * kTagSlots + k) * 2, w0[k], w1[k]);
}

__device__ __forceinline__ bool collect3_finish(const unsigned long long* trp, int iw0, int nwg,
                                                double* s_out, unsigned tag, int* abort_flag,
                                                unsigned long long w0[3],
                                                unsigned long long w1[3]) {
  const int lane = threadIdx.x & 63;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  bool ok = true;
  if (lane < nwg) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ok = ok && poll_tagged(trp + ((size_t)(iw0 + lane) * kTagSlots + k) * 2, tag, abort_flag,
                             w0[k], w1[k]);
      t[k] += tag_value(w0[k], w1[k]);
    }
  }
  const double s = wave_sums_scatter<4>(t, lane);   // lane l holds sum l >> 4
  if ((lane & 15) == 0 && (lane >> 4) < 3) s_out[lane >> 4] = s;
  return ok;
}

// e = the rows of A_c^-1 belonging to this workgroup's aggregates times w_c (already
// in LDS), then y += P_i e on this thread's row. Fixed summation order throughout.
// Skipped when the step's inversion failed. TEAMS: as for coarse_rows.
template <int TEAMS>
__device__ __forceinline__ void coarse_apply(const CoarseRow& cr_, int kloc, bool live,
                                             const double r[3], double y[3], const double* s_wc,
                                             double* s_red, double* s_e) {
  if (!cr_.ok) return;
  switch (cr_.nrow) {   // 6 x the workgroup's aggregates (uniform)
    case 6: coarse_rows_at<6, TEAMS>(cr_, s_wc, s_red, s_e); break;
    case 12: coarse_rows_at<12, TEAMS>(cr_, s_wc, s_red, s_e); break;
    case 18: coarse_rows_at<18, TEAMS>(cr_, s_wc, s_red, s_e); break;
    case 24: coarse_rows_at<24, TEAMS>(cr_, s_wc, s_red, s_e); break;
    default: break;
  }
  if (live) {
    const double* e = s_e + 6 * kloc;
    y[0] += e[0] + (e[4] * r[2] - e[5] * r[1]);
    y[1] += e[1] + (e[5] * r[0] - e[3] * r[2]);
    y[2] += e[2] + (e[3] * r[1] - e[4] * r[0]);
  }
}

// The whole coarse correction after the barrier that publishes the partial sums.
template <int TEAMS>
__device__ __forceinline__ void coarse_correct(const CoarseRow& cr_, int kloc, bool live,
                                               const double r[3], double y[3],
                                               const int* s_pidx, double* s_wc, double* s_red,
                                               double* s_e) {
  if (!cr_.ok) return;
  coarse_gather(cr_, s_pidx, s_wc);
  __syncthreads();
  coarse_apply<TEAMS>(cr_, kloc, live, r, y, s_wc, s_red, s_e);
}

// y += P1_i B1^-1 P1^T v on this thread's row: the middle-level correction. The run
// of kMid rows occupies one aligned group of kMid lanes, so P1^T v is a butterfly
// within the group; Bm is the run's 6x6 inverse (LDS). No barrier, no global access.
__device__ __forceinline__ void mid_apply(const double* __restrict__ Bm, bool live, const double r[3],
                                          const double v[3], double y[3]) {
  double t[6];
  t[0] = live ? v[0] : 0.0;
  t[1] = live ? v[1] : 0.0;
  t[2] = live ? v[2] : 0.0;
  t[3] = live ? r[1] * v[2] - r[2] * v[1] : 0.0;
  t[4] = live ? r[2] * v[0] - r[0] * v[2] : 0.0;
  t[5] = live ? r[0] * v[1] - r[1] * v[0] : 0.0;
  // sums over the run's 16 lanes (one DPP row), in every lane of the row
  static_assert(kMid == 16, "a run is one DPP row");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    t[q] += exch<1>(t[q], lane);
    t[q] += exch<2>(t[q], lane);
    t[q] += exch<4>(t[q], lane);
    t[q] += exch<8>(t[q], lane);
  }
  double e[6];
#pragma unroll
  for (int q = 0; q < 6; ++q)
    e[q] = Bm[q * 6] * t[0] + Bm[q * 6 + 1] * t[1] + Bm[q * 6 + 2] * t[2] + Bm[q * 6 + 3] * t[3] +
           Bm[q * 6 + 4] * t[4] + Bm[q * 6 + 5] * t[5];
  if (live) {
    y[0] += e[0] + (e[4] * r[2] - e[5] * r[1]);
    y[1] += e[1] + (e[5] * r[0] - e[3] * r[2]);
    y[2] += e[2] + (e[3] * r[1] - e[4] * r[0]);
  }
}

// Kernel-only matrix home: register-resident rows split over two wavefront teams.
constexpr int kMatRegHalf = 3;

template <typename TM, int MM, bool COARSE, int OCC>
__global__ void __launch_bounds__(256, OCC) k_pcg(Mesh m, SolverPlan plan, SolverWork w, Coarse cs,
                                             PcgArgs<TM> a) {
  // SPLIT (rows of at most kSplitRows): the block is twice the row threads; threads
  // PB + t hold slots [kSpmvSplit, maxnz) of row t in registers and compute that part
  // of every product A v, and take part in everything else as rows that do not exist
  constexpr bool SPLIT = MM == kMatRegHalf;
  constexpr int TEAMS = SPLIT ? 2 : 1;
  constexpr bool LDS_MATRIX = MM == kMatLds, REG_MATRIX = MM == kMatReg || SPLIT;
  static_assert(!REG_MATRIX || OCC == 1, "register-resident rows need the whole register file");
#ifdef PHISFT_PHASES
  unsigned long long ph[7] = {0, 0, 0, 0, 0, 0, 0};
#endif
  // two workgroups per CU leave 256 registers per lane: smaller streamed batches
  constexpr int SCH = OCC >= 2 ? 4 : kStreamChunk;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double s_out[3];
  __shared__ double s_wd[3 * 4];   // tagged dot partials per wavefront (unsplit blocks)
  const int wg = plan.wg_base + blockIdx.x;
  const int inst = plan.wg_inst[wg];
  const int row0 = plan.wg_row0[wg];
  const int nrows = plan.wg_nrows[wg];
  const int iw0 = plan.inst_wg0[inst], nwg = plan.inst_nwg[inst];
  // R rows per workgroup (the LDS stride); the block has R rounded up to whole
  // wavefronts so every lane of every wave exists for the cross-lane reductions.
  // RH: R plus the largest halo, rounded up to 8 (the stride of the vector copies)
  const int tid = threadIdx.x, R = plan.rows, RH = R + (plan.max_halo + 7) / 8 * 8;
  const int nv = m.nv, maxnz = m.maxnz;
  const int PB = SPLIT ? (int)blockDim.x / 2 : (int)blockDim.x;   // threads with rows
  const bool helper = SPLIT && tid >= PB;
  const int lrow = helper ? tid - PB : tid;   // the row whose blocks this thread holds
  const bool act = tid < nrows;               // helpers: tid >= PB >= nrows
  const bool hact = helper && lrow < nrows;
  const int i = row0 + (act ? tid : 0);
  Barrier bar = make_barrier(plan, w, inst, wg, iw0, nwg);
  const int h0 = plan.halo_ptr[wg], nh = plan.halo_ptr[wg + 1] - h0;
  int nep = 0, pep = 0;   // tagged publications of m and of the partials
  const bool tagp =
      COARSE && nwg <= (SPLIT ? kTagWgMaxSplit : min(kTagWgMax, (int)blockDim.x));

  double* mL = reinterpret_cast<double*>(lds_raw);                 // [2][3][RH]
  int* Cl = reinterpret_cast<int*>(mL + 6 * (size_t)RH);           // [maxnz][R] local columns
  int* s_hidx = Cl + (size_t)maxnz * R;                            // [RH - R] halo rows
  TM* Al = reinterpret_cast<TM*>(s_hidx + (RH - R));               // [maxnz][9][R] (LDS mode)
  // coarse: w_c [max nc], row sums [waves][24], e [24], partial-sum indices
  // [aggregates][kMaxAggWg]
  double* s_wc = reinterpret_cast<double*>(Al + (LDS_MATRIX ? (size_t)maxnz * 9 * R : 0));
  double* s_red = s_wc + cs.max_nc;
  double* s_e = s_red + 4 * 6 * kMaxWgAgg;
  double* s_mid = s_e + 6 * kMaxWgAgg;                             // [PB / kMid][36]
  int* s_pidx = reinterpret_cast<int*>(s_mid + (PB / kMid) * 36);
  float* s_x = reinterpret_cast<float*>(s_pidx + (cs.max_nc / 6) * kMaxAggWg);  // [nrow][nc]
  // matrix operand: LDS copy, or the assembled ELL array read in place
  const TM* Am = LDS_MATRIX ? Al : a.A;
  const int As = LDS_MATRIX ? R : nv;
  const int Ai = LDS_MATRIX ? tid : i;
  // REG_MATRIX: the row's blocks (SPLIT: one of its two slot ranges, from slot kr0),
  // in registers for the launch
  constexpr int NREG = SPLIT ? kSpmvSplit : (REG_MATRIX ? kRegRowBlocks : 1);
  static_assert(!SPLIT || 2 * kSpmvSplit >= kRegRowBlocks, "two ranges hold a row");
  TM Ar[NREG][9];
  if (REG_MATRIX) {
    const int kr0 = helper ? kSpmvSplit : 0, ir = row0 + lrow;
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
      const bool in = (act || hact) && kr0 + k < maxnz;
      const int j = in ? m.ell_col[(kr0 + k) * nv + ir] : -1;
#pragma unroll
      for (int q = 0; q < 9; ++q)
        Ar[k][q] = j < 0 ? TM(0) : a.A[(size_t)((kr0 + k) * 9 + q) * nv + ir];
    }
  }
  // y = A v for this thread's row; y is left unchanged on threads without a row. Every
  // thread of the workgroup calls it (SPLIT: the second range's sums reach the row's
  // thread through LDS, two buffers in turn: a helper rewrites one only after the
  // next call's barrier, which every reader of the previous one has passed).
  __shared__ double s_half[SPLIT ? 2 * 3 * kSplitRows : 1];
  int nspmv = 0;
  auto spmv = [&](const double* vl, double y[3]) {
    if constexpr (SPLIT) {
      double t[3] = {0.0, 0.0, 0.0};
      const int kb = helper ? kSpmvSplit : 0, ke = helper ? maxnz : min(kSpmvSplit, maxnz);
      if (act || hact) spmv_reg_range<TM, kSpmvSplit>(Ar, Cl, R, lrow, kb, ke, vl, RH, t);
      double* hb = s_half + (nspmv++ & 1) * 3 * kSplitRows;
      if (hact) {
#pragma unroll
        for (int c = 0; c < 3; ++c) hb[c * kSplitRows + lrow] = t[c];
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) y[c] = t[c] + hb[c * kSplitRows + tid];
      }
    } else if (act) {
      if constexpr (REG_MATRIX) spmv_reg<TM>(Ar, Cl, R, tid, maxnz, vl, RH, y);
      else spmv_row<TM, LDS_MATRIX, SCH>(Am, As, Ai, Cl, R, tid, maxnz, vl, RH, y);
    }
  };
  if (act) {
    for (int k = 0; k < maxnz; ++k) {
      Cl[k * R + tid] = plan.lcol[k * nv + i];
      if (LDS_MATRIX) {
        const int j = m.ell_col[k * nv + i];
#pragma unroll
        for (int q = 0; q < 9; ++q)
          Al[(k * 9 + q) * R + tid] = j < 0 ? TM(0) : a.A[(size_t)(k * 9 + q) * nv + i];
      }
    }
  }
  for (int h = tid; h < nh; h += blockDim.x) s_hidx[h] = plan.halo_idx[h0 + h];
  // coarse-space data of this row (cr: offset in its aggregate, cr1: in its run)
  int wa0 = 0, wna = 0, kloc = 0, kf = 0, kl = -1;
  CoarseRow crow{};
  bool live = false;
  double cr[3] = {0.0, 0.0, 0.0}, cr1[3] = {0.0, 0.0, 0.0};
  if (COARSE) {
    wa0 = cs.wg_agg0[wg];
    wna = cs.wg_nagg[wg];
    // partial-sum indices of every aggregate of the sheet (fixed for the launch)
    const int ag0 = cs.inst_agg0[inst], nag = cs.inst_nagg[inst];
    for (int e = tid; e < nag * kMaxAggWg; e += blockDim.x) {
      const int t = e / kMaxAggWg, k = e - t * kMaxAggWg, a = ag0 + t;
      int pi = -1;
      if (k < cs.agg_nwg[a]) {
        const int w2 = cs.agg_wg0[a] + k;
        pi = w2 * kMaxWgAgg + (a - cs.wg_agg0[w2]);
      }
      s_pidx[e] = pi;
    }
    // most workgroups any aggregate of the sheet spans (the gathers read no more
    // partial slots per aggregate): every wavefront reduces the whole list
    {
      int nm = 1;
      for (int t = tid & 63; t < nag; t += 64) nm = max(nm, cs.agg_nwg[ag0 + t]);
      for (int o = 32; o > 0; o >>= 1) nm = max(nm, __shfl_xor(nm, o));
      crow.nwm = min(nm, kMaxAggWg);
    }
    const int np = cs.inst_np[inst];
    crow.X = cs.xinv + cs.inst_coff[inst] + (size_t)6 * (wa0 - ag0) * np;
    crow.XL = nullptr;
    crow.part = cs.part;
    crow.nc = cs.inst_nc[inst];
    crow.np = np;
    crow.nrow = 6 * wna;
    crow.ok = cs.ok[inst];
    if (plan.xl_floats > 0) {
      // the rows are fixed for the launch: one copy into LDS
      const int nc = crow.nc;
      for (int q = 0; q < crow.nrow; ++q)
        for (int c = tid; c < nc; c += blockDim.x) s_x[q * nc + c] = crow.X[(size_t)q * np + c];
      crow.XL = s_x;
    }
    const int f = (tid >> 6) * 64;
    if (f < nrows) {
      kf = cs.vert_agg[row0 + f] - wa0;
      kl = cs.vert_agg[row0 + min(nrows, f + 64) - 1] - wa0;
    }
    if (act) {
      kloc = cs.vert_agg[i] - wa0;
      live = m.pinned[i] == 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cr[c] = cs.crel[c * nv + i];
        cr1[c] = cs.mid_crel[c * nv + i];
      }
    }
    // the middle level's 6x6 inverses of this workgroup's runs (rows start on a run)
    const int m0 = cs.vert_mid[row0], nmw = (nrows + kMid - 1) / kMid;
    for (int e = tid; e < nmw * 36; e += blockDim.x) s_mid[e] = cs.mid_inv[(size_t)m0 * 36 + e];
  }
  __syncthreads();
  const double* Bm = s_mid + (lrow / kMid) * 36;

  double J[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) J[q] = act ? (double)a.Jinv[q * nv + i] : 0.0;
  double x[3] = {0.0, 0.0, 0.0}, r[3] = {0.0, 0.0, 0.0}, u[3], wv[3] = {0.0, 0.0, 0.0};
  double mm[3], nn[3], z[3] = {0.0, 0.0, 0.0}, q3[3] = {0.0, 0.0, 0.0};
  double sv[3] = {0.0, 0.0, 0.0}, p[3] = {0.0, 0.0, 0.0};
  if (act) {
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = a.rhs[c * nv + i];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) u[c] = J[3 * c] * r[0] + J[3 * c + 1] * r[1] + J[3 * c + 2] * r[2];
  bool ok = true;
  if (COARSE) {
    mid_apply(Bm, live, cr1, r, u);
    coarse_restrict(cs.part, wg, wna, kf, kl, kloc, live, cr, r);
    ok = cluster_barrier(bar, w.abort_flag, a.status, inst);
    if (ok) coarse_correct<TEAMS>(crow, kloc, live, cr, u, s_pidx, s_wc, s_red, s_e);
  }
  // w_0 = A u_0 needs the neighbours' u_0 (LDS copy of parity 1; the loop starts at 0)
  double* ub = w.zbuf;
  {
    double* ul = mL + 3 * (size_t)RH;
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ub[c * nv + i] = u[c];
        ul[c * RH + tid] = u[c];
      }
    }
    // every wavefront wrote rows: each releases its own stores before the barrier
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (ok) ok = cluster_barrier(bar, w.abort_flag, a.status, inst);
    if (ok) {
      halo_load(ub, nv, s_hidx, nh, ul, R, RH);
      __syncthreads();
      spmv(ul, wv);
    }
  }

  double bnorm = 0.0, rr = 0.0, gamma_prev = 1.0, alpha_prev = 1.0;
  int it = 0, flag = 0, fresh = 1, restarts = 0;
  bool restart = false;
  while (ok) {
    if (restart) {
      // Restart the recurrences from the true residual r = b - A x (x published
      // through the pbuf slot and the LDS copy that no workgroup reads in this phase).
      restart = false;
      double* xb = w.pbuf + (size_t)((it + 1) & 1) * 3 * nv;
      double* xl = mL + (size_t)((it + 1) & 1) * 3 * RH;
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xb[c * nv + i] = x[c];
          xl[c * RH + tid] = x[c];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (!(ok = cluster_barrier(bar, w.abort_flag, a.status, inst))) break;
      halo_load(xb, nv, s_hidx, nh, xl, R, RH);
      __syncthreads();
      double ax[3] = {0.0, 0.0, 0.0};
      spmv(xl, ax);
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = a.rhs[c * nv + i] - ax[c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
        u[c] = J[3 * c] * r[0] + J[3 * c + 1] * r[1] + J[3 * c + 2] * r[2];
      if (COARSE) {
        mid_apply(Bm, live, cr1, r, u);
        coarse_restrict(cs.part, wg, wna, kf, kl, kloc, live, cr, r);
        if (!(ok = cluster_barrier(bar, w.abort_flag, a.status, inst))) break;
        coarse_correct<TEAMS>(crow, kloc, live, cr, u, s_pidx, s_wc, s_red, s_e);
      }
      __syncthreads();  // every thread is done reading xl before it is overwritten
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ub[c * nv + i] = u[c];
          xl[c * RH + tid] = u[c];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (!(ok = cluster_barrier(bar, w.abort_flag, a.status, inst))) break;
      halo_load(ub, nv, s_hidx, nh, xl, R, RH);
      __syncthreads();
      spmv(xl, wv);
#pragma unroll
      for (int c = 0; c < 3; ++c) z[c] = q3[c] = sv[c] = p[c] = 0.0;
      fresh = 1;
      ++restarts;
    }
    const int par = it & 1;
    double* mb = w.pbuf + (size_t)par * 3 * nv;
    double* ml = mL + (size_t)par * 3 * RH;
    // m = M^-1 w: block Jacobi and middle level here (block Jacobi only: published
    // before the barrier, whose halo read needs it), with the coarse space after the
    // partials have left (the local part needs nothing from other workgroups)
    auto m_local = [&]() {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        mm[c] = J[3 * c] * wv[0] + J[3 * c + 1] * wv[1] + J[3 * c + 2] * wv[2];
      if (COARSE) mid_apply(Bm, live, cr1, wv, mm);
    };
    if (!COARSE) {
      m_local();
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          mb[c * nv + i] = mm[c];
          ml[c * RH + tid] = mm[c];
        }
      }
    }
    const double loc[3] = {r[0] * u[0] + r[1] * u[1] + r[2] * u[2],
                           wv[0] * u[0] + wv[1] * u[1] + wv[2] * u[2],
                           r[0] * r[0] + r[1] * r[1] + r[2] * r[2]};
    double* red_slot = w.red + (size_t)par * plan.nwg * 3;
    // Coarse space on a sheet of at most kTagWgMax (split rows: kTagWgMaxSplit)
    // workgroups: the partials go out as tagged words that every workgroup of the sheet
    // polls (no barrier). Larger sheets and block-Jacobi only: plain partials released
    // by a cluster barrier.
    const unsigned long long* trp = w.tred + (size_t)par * plan.nwg * kTagSlots * 2;
    PHASE_T(t0);
    if (COARSE) {
      ++pep;
      publish_restrict_dots(tagp, const_cast<unsigned long long*>(trp) + (size_t)wg * kTagSlots * 2,
                            (unsigned)pep, cs.part, red_slot + (size_t)wg * 3, wg, wna, kf, kl,
                            kloc, live, cr, wv, loc);
    } else {
      publish3(loc, red_slot + (size_t)wg * 3);
    }
    PHASE_T(t1);
    if (!tagp) cluster_arrive(bar, w.abort_flag);
    if (COARSE) m_local();
    if (!tagp && !(ok = cluster_wait(bar, w.abort_flag, a.status, inst))) break;
    PHASE_T(t2);
    if (tagp) {
      // the coarse residual and the dot partials are polled together; with split rows
      // wavefront 0 issues the partials' loads first, so both round trips overlap;
      // without, every wavefront collects up to 64 workgroups' partials
      __shared__ int s_late;
      unsigned long long d0[3], d1[3];
      if (SPLIT && tid < 64) collect3_issue(trp, iw0, nwg, d0, d1);
      if (tid == 0) s_late = 0;
      __syncthreads();
      bool got =
          coarse_gather_tagged<SPLIT>(crow, s_pidx, s_wc, trp, (unsigned)pep, w.abort_flag);
      if constexpr (SPLIT) {
        if (tid < 64)
          got = collect3_finish(trp, iw0, nwg, s_out, (unsigned)pep, w.abort_flag, d0, d1) && got;
      } else {
        got = collect3_waves(trp, iw0, nwg, s_wd, (unsigned)pep, w.abort_flag) && got;
      }
      if (!got) s_late = 1;
      __syncthreads();
      if (s_late) {
        if (tid == 0) {
          __hip_atomic_store(w.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          set_status(a.status, inst, ST_TIMEOUT);
        }
        ok = false;
        break;
      }
    } else {
      // the halo of m (block-Jacobi only) or the coarse residual, and the partial sums
      if (!COARSE) halo_load(mb, nv, s_hidx, nh, ml, R, RH);
      if (COARSE) coarse_gather(crow, s_pidx, s_wc);
      collect3(red_slot, iw0, nwg, s_out);
      __syncthreads();
    }
    double gamma = s_out[0], delta = s_out[1];
    rr = s_out[2];
    if (!SPLIT && tagp) {
      gamma = delta = rr = 0.0;
      for (int q = 0; q * 64 < nwg; ++q) {
        gamma += s_wd[3 * q];
        delta += s_wd[3 * q + 1];
        rr += s_wd[3 * q + 2];
      }
    }
    __syncthreads();  // s_out and s_wd are rewritten by the next collection
    PHASE_T(t3);
    if (it == 0) bnorm = sqrt(rr);
    if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rr)) {
      flag = ST_NONFINITE;
      break;
    }
    if (bnorm == 0.0) break;
    if (sqrt(rr) <= a.tol * bnorm) {
      // accept only a true residual: right after a (re)start r = b - A x exactly
      if (fresh) break;
      restart = true;
      continue;
    }
    if (fresh && restarts > kMaxRestarts) {
      // the restart after the last allowed one verified x and found it short of the
      // tolerance (the recurrences kept meeting it while the true residual did not):
      // stop, reporting that true residual
      flag = ST_NOT_CONVERGED;
      break;
    }
    if (it >= a.max_iter) {
      flag = ST_NOT_CONVERGED;
      break;
    }
    PHASE_T(t5);
    if (COARSE) {
      // m = M^-1 w needs the coarse correction before it is published for the SpMV
      coarse_apply<TEAMS>(crow, kloc, live, cr, mm, s_wc, s_red, s_e);
      PHASE_ADD(6, wall_clock64() - t5);
      unsigned long long* tb = w.tbuf + (size_t)par * 4 * nv;
      ++nep;
      if (act) {
        publish_tagged(tb, i, nv, mm, (unsigned)nep);
#pragma unroll
        for (int c = 0; c < 3; ++c) ml[c * RH + tid] = mm[c];
      }
      PHASE_ADD(4, wall_clock64() - t5);
      if (!halo_load_tagged<SPLIT>(tb, nv, s_hidx, nh, ml, R, RH, (unsigned)nep, w.abort_flag)) {
        if (tid == 0) {
          __hip_atomic_store(w.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          set_status(a.status, inst, ST_TIMEOUT);
        }
        ok = false;
        break;
      }
      PHASE_ADD(5, wall_clock64() - t5);
    }
    nn[0] = nn[1] = nn[2] = 0.0;
    spmv(ml, nn);
    PHASE_T(t4);
    PHASE_ADD(0, t1 - t0);
    PHASE_ADD(1, t2 - t1);
    PHASE_ADD(2, t3 - t2);
    PHASE_ADD(3, t4 - t3);
    const double beta = fresh ? 0.0 : gamma / gamma_prev;
    const double denom = fresh ? delta : delta - beta * gamma / alpha_prev;
    if (!(denom > 0.0)) {
      // Right after a (re)start denom = u^T A u: A is not positive definite. Later, the
      // recurrences have drifted (rounding): restart them from the true residual (past
      // the restart cap, that restart ends the solve unless it meets the tolerance).
      if (fresh) {
        flag = ST_INDEFINITE;
        break;
      }
      restart = true;
      continue;
    }
    fresh = 0;
    const double alpha = gamma / denom;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[c] = nn[c] + beta * z[c];
      q3[c] = mm[c] + beta * q3[c];
      sv[c] = wv[c] + beta * sv[c];
      p[c] = u[c] + beta * p[c];
      x[c] += alpha * p[c];
      r[c] -= alpha * sv[c];
      u[c] -= alpha * q3[c];
      wv[c] -= alpha * z[c];
    }
    gamma_prev = gamma;
    alpha_prev = alpha;
    ++it;
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.sol[c * nv + i] = x[c];
  }
#ifdef PHISFT_PHASES
  if (tid == 0 && wg < 512) {
    for (int k = 0; k < 7; ++k) g_phase[wg][k] += ph[k];
    g_phase[wg][7] += it;
  }
#endif
  if (wg == iw0 && tid == 0) {
    if (flag) set_status(a.status, inst, flag);
    if (a.iters) a.iters[inst] = it;
    if (a.resid) a.resid[inst] = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
  }
}

// ---------------------------------------------------------- forward: update
template <typename T>
__global__ void __launch_bounds__(256) k_update(int nv, const int* __restrict__ pinned,
                                                const int* __restrict__ vert_inst,
                                                const int* __restrict__ vold,
                                                const double* __restrict__ xp,
                                                const double* __restrict__ vp,
                                                const double* __restrict__ dv, double h,
                                                double* __restrict__ xn, double* __restrict__ vn,
                                                T* __restrict__ xout, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const bool pin = pinned[i] != 0;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = pin ? 0.0 : vp[c * nv + i] + dv[c * nv + i];
    double xx = xp[c * nv + i] + h * v;
    ok = ok && isfinite(xx) && isfinite(v);
    vn[c * nv + i] = v;
    xn[c * nv + i] = xx;
    if (xout) xout[c * nv + vold[i]] = (T)xx;
  }
  if (!ok) set_status(status, vert_inst[i], ST_NONFINITE);
}

template <typename T>
__global__ void __launch_bounds__(256) k_init_state(int nv, const int* __restrict__ pinned,
                                                    const int* __restrict__ vert_inst,
                                                    const int* __restrict__ vold,
                                                    const T* __restrict__ x0,
                                                    const T* __restrict__ v0,
                                                    double* __restrict__ xs,
                                                    double* __restrict__ vs, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const int o = vold[i];
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double xx = (double)x0[c * nv + o];
    double v = (v0 && !pinned[i]) ? (double)v0[c * nv + o] : 0.0;
    ok = ok && isfinite(xx) && isfinite(v);
    xs[c * nv + i] = xx;
    vs[c * nv + i] = v;
  }
  if (!ok) set_status(status, vert_inst[i], ST_NONFINITE);
}

// ---------------------------------------------------------------- adjoint
// gx += dL/dx_s (if s is a loss frame); u = mask(gv + h gx)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_pre(int nv, const int* __restrict__ pinned,
                                                 const int* __restrict__ vert_inst,
                                                 const int* __restrict__ vold,
                                                 const T* __restrict__ dl, double h,
                                                 double* __restrict__ gx,
                                                 const double* __restrict__ gv,
                                                 double* __restrict__ u, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double g = gx[c * nv + i];
    if (dl) {
      double d = (double)dl[c * nv + vold[i]];
      ok = ok && isfinite(d);
      g += d;
      gx[c * nv + i] = g;
    }
    u[c * nv + i] = pinned[i] ? 0.0 : gv[c * nv + i] + h * g;
  }
  if (!ok) set_status(status, vert_inst[i], ST_NONFINITE);
}

// Element vector-Jacobian products of one adjoint step at x_{s-1}, with the
// adjoint solution mu and the new velocity v_s:
//   ag = -h K_exact mu - h^2 grad_x(mu^T K_sys(x) v_s)   (state gradient)
//   ak = K_sys mu                                         (velocity gradient)
//   acc_ks += mu . (h f_m/k_s - h^2 (K_sys,m/k_s) v_s), acc_kb likewise.
template <typename T, bool WANG>
__global__ void __launch_bounds__(256) k_adj_elements(Mesh m, Elem el, AdjArgs<T> a) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nv = m.nv;
  const double h = a.h, h2 = a.h * a.h;
  if (gid < m.nt) {
    const int t = gid, nt = m.nt;
    Tri s;
    int v[3];
    tri_load(m, a.x, t, s, v);
    const double ks = a.mat[m.matn * m.tri_inst[t] + 0];
    double mu[3][3], vv[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mu[i][c] = a.mu[c * nv + v[i]];
        vv[i][c] = a.vs[c * nv + v[i]];
      }
    double dFm[3][2], dFv[3][2];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        dFm[r][c] = mu[0][r] * s.w[0][c] + mu[1][r] * s.w[1][c] + mu[2][r] * s.w[2][c];
        dFv[r][c] = vv[0][r] * s.w[0][c] + vv[1][r] * s.w[1][c] + vv[2][r] * s.w[2][c];
      }
    // S3 = sym(F^T dF_mu), S2 = sym(F^T dF_v), S1 = sym(dF_mu^T dF_v)
    double S1[2][2], S2[2][2], S3[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double fm = 0, mf = 0, fv = 0, vf = 0, mv = 0, vm = 0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          fm += s.F[r][p] * dFm[r][q];
          mf += dFm[r][p] * s.F[r][q];
          fv += s.F[r][p] * dFv[r][q];
          vf += dFv[r][p] * s.F[r][q];
          mv += dFm[r][p] * dFv[r][q];
          vm += dFv[r][p] * dFm[r][q];
        }
        S3[p][q] = 0.5 * (fm + mf);
        S2[p][q] = 0.5 * (fv + vf);
        S1[p][q] = 0.5 * (mv + vm);
      }
    if constexpr (WANG) {
      // anisotropic stretch (exact membrane block, measure stiffnesses c_k constant on
      // their segments): with C : X = sum_k c_k (N_k : X) N_k,
      //   K mu at vertex i = A (dF_mu Sg + F (C : S3)) w_i,
      //   grad_x (mu^T K v) at vertex i = A (F (C : S1) + dF_mu (C : S2) + dF_v (C : S3)) w_i,
      // and for the table entry (k, j): d Sg / dS[k][j] = sgn(s_k) part_j(|s_k|) N_k,
      // d c_k / dS[k][j] = [j is s_k's segment].
      const int inst = m.tri_inst[t];
      double N[4][3], Sg[2][2], sk[4], c[4];
      load_measures(m, t, N);
      wang_stretch(N, a.mat + m.matn * inst, s.G, Sg, sk, c);
      double CS1[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, CS2[2][2] = {{0.0, 0.0}, {0.0, 0.0}},
             CS3[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
      double n1[4], n2[4], n3[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        n1[k] = ncon(N[k], S1);
        n2[k] = ncon(N[k], S2);
        n3[k] = ncon(N[k], S3);
        const double m1 = c[k] * n1[k], m2 = c[k] * n2[k], m3 = c[k] * n3[k];
        const double Nm[2][2] = {{N[k][0], N[k][1]}, {N[k][1], N[k][2]}};
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            CS1[p][q] += m1 * Nm[p][q];
            CS2[p][q] += m2 * Nm[p][q];
            CS3[p][q] += m3 * Nm[p][q];
          }
      }
      const double A = s.area;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double qe = 0.0, qt = 0.0;
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2) {
            const double e2 = dFm[r][0] * Sg[0][c2] + dFm[r][1] * Sg[1][c2] +
                              s.F[r][0] * CS3[0][c2] + s.F[r][1] * CS3[1][c2];
            const double t2 = s.F[r][0] * CS1[0][c2] + s.F[r][1] * CS1[1][c2] +
                              dFm[r][0] * CS2[0][c2] + dFm[r][1] * CS2[1][c2] +
                              dFv[r][0] * CS3[0][c2] + dFv[r][1] * CS3[1][c2];
            qe += e2 * s.w[i][c2];
            qt += t2 * s.w[i][c2];
          }
          el.tri_ag[(i * 3 + r) * nt + t] = -h * A * qe - h2 * A * qt;
          el.tri_ak[(i * 3 + r) * nt + t] = A * qe;
        }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double tk = fabs(sk[k]), sg = sk[k] < 0.0 ? -1.0 : 1.0;
        const int sj = seg_of<6, true>(tk);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          const double dp = sg * seg_part<6, true>(j, tk);
          el.acc_ws[(6 * k + j) * nt + t] +=
              -h * A * dp * n3[k] - h2 * A * (dp * n1[k] + (j == sj ? n3[k] * n2[k] : 0.0));
        }
      }
    } else {
      // stress term of K_sys and its derivative along S1
      double Gp[2][2], Y[2][2];
      if (m.tension) {
        Eig2 eg = eig2(s.G);
        tension(eg, Gp);
        tension_deriv(eg, S1, Y);
      } else {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            Gp[p][q] = s.G[p][q];
            Y[p][q] = S1[p][q];
          }
      }
      // 3x2 matrices, all without the area * k_s factor
      double Qe[3][2], Qs[3][2], Qt[3][2], Pf[3][2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          double fs3 = s.F[r][0] * S3[0][c] + s.F[r][1] * S3[1][c];
          Qe[r][c] = dFm[r][0] * s.G[0][c] + dFm[r][1] * s.G[1][c] + fs3;
          Qs[r][c] = dFm[r][0] * Gp[0][c] + dFm[r][1] * Gp[1][c] + fs3;
          Qt[r][c] = s.F[r][0] * Y[0][c] + s.F[r][1] * Y[1][c] + dFm[r][0] * S2[0][c] +
                     dFm[r][1] * S2[1][c] + dFv[r][0] * S3[0][c] + dFv[r][1] * S3[1][c];
          Pf[r][c] = s.F[r][0] * s.G[0][c] + s.F[r][1] * s.G[1][c];
        }
      const double A = s.area, ak = s.area * ks;
      double part = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double qe = Qe[r][0] * s.w[i][0] + Qe[r][1] * s.w[i][1];
          double qs = Qs[r][0] * s.w[i][0] + Qs[r][1] * s.w[i][1];
          double qt = Qt[r][0] * s.w[i][0] + Qt[r][1] * s.w[i][1];
          double pf = Pf[r][0] * s.w[i][0] + Pf[r][1] * s.w[i][1];
          el.tri_ag[(i * 3 + r) * nt + t] = -h * ak * qe - h2 * ak * qt;
          el.tri_ak[(i * 3 + r) * nt + t] = ak * qs;
          // unit-stiffness force -A pf, unit-stiffness K_sys mu = A qs (symmetric: v.K mu)
          part += mu[i][r] * (-h * A * pf) - h2 * vv[i][r] * (A * qs);
        }
      el.acc_ks[t] += part;
    }
    if (a.wind) {
      // The wind's share of the step: h f_w in b and h D in A, so the adjoint takes the
      // gradient of Phi = h (mu . f_w - mu^T D dv) over the triangle's positions,
      // velocities v_{s-1} and the wind w. With mean vertex values mb (of mu) and db (of
      // dv = v_s - v_{s-1}), s = n . (w - mean v_{s-1}), a = n . mb, b = n . db and
      // ra = rho area: Phi = h ra |s| a (s - 2 b), so
      //   dPhi/ds = 2 h ra a (|s| - sgn(s) b)      (n held fixed)
      //   dPhi/dn = dPhi/ds (w - mean v) + h ra |s| ((s - 2 b) mb - 2 a db),
      // through n = N / |N| and N = (x_b - x_a) x (x_c - x_a) to the positions; s gives
      // dPhi/dw = dPhi/ds n and dPhi/dv_j = -dPhi/ds n / 3 for each vertex j.
      const double* wv = a.wind + 3 * m.tri_inst[t];
      double e1[3], e2[3], rel[3], mb[3], db[3], n[3], sn, ln;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double xa = a.x[r * nv + v[0]];
        e1[r] = a.x[r * nv + v[1]] - xa;
        e2[r] = a.x[r * nv + v[2]] - xa;
        const double p0 = a.vp[r * nv + v[0]], p1 = a.vp[r * nv + v[1]], p2 = a.vp[r * nv + v[2]];
        rel[r] = wv[r] - (p0 + p1 + p2) / 3.0;
        mb[r] = (mu[0][r] + mu[1][r] + mu[2][r]) / 3.0;
        db[r] = ((vv[0][r] - p0) + (vv[1][r] - p1) + (vv[2][r] - p2)) / 3.0;
      }
      wind_frame(e1, e2, rel, n, sn, ln);
      const double ra = a.rho * s.area, as = fabs(sn), sg = sn >= 0.0 ? 1.0 : -1.0;
      const double an = n[0] * mb[0] + n[1] * mb[1] + n[2] * mb[2];
      const double bn = n[0] * db[0] + n[1] * db[1] + n[2] * db[2];
      const double dps = 2.0 * h * ra * an * (as - sg * bn);
      double gn[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        gn[r] = dps * rel[r] + h * ra * as * ((sn - 2.0 * bn) * mb[r] - 2.0 * an * db[r]);
      const double ng = n[0] * gn[0] + n[1] * gn[1] + n[2] * gn[2];
      double gN[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) gN[r] = (gn[r] - n[r] * ng) / ln;
      const double gb[3] = {e2[1] * gN[2] - e2[2] * gN[1], e2[2] * gN[0] - e2[0] * gN[2],
                            e2[0] * gN[1] - e2[1] * gN[0]};
      const double gc[3] = {gN[1] * e1[2] - gN[2] * e1[1], gN[2] * e1[0] - gN[0] * e1[2],
                            gN[0] * e1[1] - gN[1] * e1[0]};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        el.tri_ag[r * nt + t] -= gb[r] + gc[r];
        el.tri_ag[(3 + r) * nt + t] += gb[r];
        el.tri_ag[(6 + r) * nt + t] += gc[r];
        el.tri_wv[r * nt + t] = -dps * n[r] / 3.0;
        el.acc_w[r * nt + t] += dps * n[r];
      }
    }
  } else if (gid < m.nt + m.nh) {
    const int e = gid - m.nt, nh = m.nh;
    int v[4];
    double X[4][3], g[4][3], mu[4][3], vv[4][3];
    hinge_load(m, a.x, e, v, X);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mu[i][c] = a.mu[c * nv + v[i]];
        vv[i][c] = a.vs[c * nv + v[i]];
      }
    const double th = hinge_theta(X);
    hinge_grad<double>(X, g);
    const double ce = m.hin_ce[e];
    const double dth = th - m.hin_rest[e];
    double sc, wgt;   // dE/dtheta, d^2E/dtheta^2
    hinge_response<WANG>(m, a.mat, e, dth, sc, wgt);
    double gm = 0.0, gv = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gm += g[i][c] * mu[i][c];
        gv += g[i][c] * vv[i][c];
      }
    // y = (h sc + h^2 wgt gv) mu + h^2 wgt gm v; Hess(theta) y by one dual pass of
    // grad(theta)
    const double cm = h * sc + h2 * wgt * gv, cv = h2 * wgt * gm;
    dual Xd[4][3], gd[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) Xd[i][c] = dual(X[i][c], cm * mu[i][c] + cv * vv[i][c]);
    hinge_grad<dual>(Xd, gd);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        el.hin_ag[(i * 3 + c) * nh + e] = -(wgt * h * gm * g[i][c] + gd[i][c].d);
        el.hin_ak[(i * 3 + c) * nh + e] = wgt * gm * g[i][c];
      }
    if constexpr (!WANG) {
      el.acc_kb[e] += -2.0 * ce * gm * (h * dth + h2 * gv);
    } else {
      // table entry (a, j): d sc = 2 c_e d_a sgn part_j(|dth|), d wgt = 2 c_e d_a [j is the
      // segment]
      const double t = fabs(dth), sg = dth < 0.0 ? -1.0 : 1.0;
      const int sj = seg_of<5, false>(t);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double db = 2.0 * ce * m.hin_dw[b * nh + e];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const double dsc = db * sg * seg_part<5, false>(j, t), dw = j == sj ? db : 0.0;
          el.acc_wb[(5 * b + j) * nh + e] += -h * gm * dsc - h2 * gm * gv * dw;
        }
      }
    }
  }
}

// Per-vertex completion of one adjoint step: gather the element products,
// gx -= ..., gv = mask(u - h^2 K_sys mu), dL/dF_{s-1} = h mu, density partial.
// Sixteen lanes per vertex (one 16-lane DPP row), each taking every sixteenth incident
// element; a butterfly within the row sums them and lane 0 of the row finishes.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_rows(Mesh m, Elem el, AdjArgs<T> a) {
  const int lane = threadIdx.x & 63, g = lane & 15;
  const int i0 = blockIdx.x * 16 + (int)(threadIdx.x >> 4);
  const int nv = m.nv;
  if (blockIdx.x * 16 + (int)((threadIdx.x >> 6) << 2) >= nv) return;   // a wavefront past the rows
  const bool live = i0 < nv;   // lanes past the last row work on a copy of it
  const int i = live ? i0 : nv - 1;
  const double h = a.h, h2 = a.h * a.h;
  double ag[3] = {0.0, 0.0, 0.0}, ak[3] = {0.0, 0.0, 0.0}, aw[3] = {0.0, 0.0, 0.0};
  for (int c = m.vinc_ptr[i] + g; c < m.vinc_ptr[i + 1]; c += 16) {
    int ref = m.vinc_ref[c];
    if (ref >= 0) {
      int t = ref / 3, va = ref - 3 * (ref / 3);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        ag[r] += el.tri_ag[(va * 3 + r) * m.nt + t];
        ak[r] += el.tri_ak[(va * 3 + r) * m.nt + t];
      }
      if (a.wind) {
#pragma unroll
        for (int r = 0; r < 3; ++r) aw[r] += el.tri_wv[r * m.nt + t];
      }
    } else {
      int r2 = -ref - 1;
      int e = r2 >> 2, va = r2 & 3;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        ag[r] += el.hin_ag[(va * 3 + r) * m.nh + e];
        ak[r] += el.hin_ak[(va * 3 + r) * m.nh + e];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    ag[r] += exch<8>(ag[r], lane);
    ag[r] += exch<4>(ag[r], lane);
    ag[r] += exch<2>(ag[r], lane);
    ag[r] += exch<1>(ag[r], lane);
    ak[r] += exch<8>(ak[r], lane);
    ak[r] += exch<4>(ak[r], lane);
    ak[r] += exch<2>(ak[r], lane);
    ak[r] += exch<1>(ak[r], lane);
    aw[r] += exch<8>(aw[r], lane);
    aw[r] += exch<4>(aw[r], lane);
    aw[r] += exch<2>(aw[r], lane);
    aw[r] += exch<1>(aw[r], lane);
  }
  if (g != 0 || !live) return;
  const bool pin = m.pinned[i] != 0;
  const double varea = m.varea[i];
  double dpart = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double mu = a.mu[r * nv + i];
    a.gx[r * nv + i] += ag[r];
    a.gv[r * nv + i] = pin ? 0.0 : (a.wind ? a.u[r * nv + i] - h2 * ak[r] + aw[r]
                                           : a.u[r * nv + i] - h2 * ak[r]);
    if (a.dl_dF) a.dl_dF[r * nv + m.vold[i]] = (T)(h * mu);
    const double dv = pin ? 0.0 : a.vs[r * nv + i] - a.vp[r * nv + i];
    dpart += mu * (h * varea * a.g[r] - varea * dv);
  }
  el.acc_d[i] += dpart;
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_final(int nv, const int* __restrict__ vold,
                                                   const double* __restrict__ gx,
                                                   const double* __restrict__ gv,
                                                   T* __restrict__ dx0, T* __restrict__ dv0) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * nv) return;
  const int c = k / nv, i = k - c * nv;
  const int o = c * nv + vold[i];
  if (dx0) dx0[o] = (T)gx[k];
  if (dv0) dv0[o] = (T)gv[k];
}

// One workgroup per sheet: fixed-order sums of the per-element partials (the material
// gradient into out, and with out_wind the wind gradient).
__global__ void __launch_bounds__(256) k_material_sum(Mesh m, Elem el, double* __restrict__ out,
                                                      double* __restrict__ out_wind) {
  __shared__ double s_part[3][4];
  const int inst = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  const int toff = m.inst_toff[inst], nt = m.inst_nt[inst];
  const int hoff = m.inst_hoff[inst], nh = m.inst_nh[inst];
  const int voff = m.inst_voff[inst], nv = m.inst_nv[inst];
  if (m.wang) {
    // 24 stretch and 15 bend table entries, then the density: one fixed-order sum each
    const int nwaves = (blockDim.x + 63) >> 6;
    for (int q = 0; q < kWangParams; ++q) {
      double v = 0.0;
      if (q < kWangStretch)
        for (int k = threadIdx.x; k < nt; k += blockDim.x) v += el.acc_ws[(size_t)q * m.nt + toff + k];
      else if (q < kWangStretch + kWangBend)
        for (int k = threadIdx.x; k < nh; k += blockDim.x)
          v += el.acc_wb[(size_t)(q - kWangStretch) * m.nh + hoff + k];
      else
        for (int k = threadIdx.x; k < nv; k += blockDim.x) v += el.acc_d[voff + k];
      v = wave_sum(v);
      __syncthreads();   // the previous entry's partials have been read
      if (lane == 0) s_part[0][wave] = v;
      __syncthreads();
      if (threadIdx.x == 0 && out) {
        double r = 0.0;
        for (int w = 0; w < nwaves; ++w) r += s_part[0][w];
        out[kWangParams * inst + q] = r;
      }
    }
  } else {
    for (int k = threadIdx.x; k < nt; k += blockDim.x) t0 += el.acc_ks[toff + k];
    for (int k = threadIdx.x; k < nh; k += blockDim.x) t1 += el.acc_kb[hoff + k];
    for (int k = threadIdx.x; k < nv; k += blockDim.x) t2 += el.acc_d[voff + k];
    t0 = wave_sum(t0);
    t1 = wave_sum(t1);
    t2 = wave_sum(t2);
    if (lane == 0) {
      s_part[0][wave] = t0;
      s_part[1][wave] = t1;
      s_part[2][wave] = t2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nwaves = (blockDim.x + 63) >> 6;
      double r0 = 0.0, r1 = 0.0, r2 = 0.0;
      for (int q = 0; q < nwaves; ++q) {
        r0 += s_part[0][q];
        r1 += s_part[1][q];
        r2 += s_part[2][q];
      }
      if (out) {
        out[3 * inst + 0] = r0;
        out[3 * inst + 1] = r1;
        out[3 * inst + 2] = r2;
      }
    }
  }
  if (!out_wind) return;   // uniform
  double w3[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nt; k += blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) w3[c] += el.acc_w[c * m.nt + toff + k];
  __syncthreads();   // s_part is reused
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w3[c] = wave_sum(w3[c]);
    if (lane == 0) s_part[c][wave] = w3[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double r = 0.0;
      for (int q = 0; q < nwaves; ++q) r += s_part[c][q];
      out_wind[3 * inst + c] = r;
    }
  }
}

__global__ void k_fill_int(int* p, int n, int v) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// Zeroes up to four int ranges in one launch (grid-stride; the solver's counters,
// abort flag and tagged buffers before each launch).
struct ZeroRanges {
  int* p[4];
  int n[4];
};

__global__ void __launch_bounds__(256) k_zero_ranges(ZeroRanges z) {
  const int stride = gridDim.x * blockDim.x;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < z.n[r]; k += stride) z.p[r][k] = 0;
}

__global__ void k_fill_double(double* p, long n, double v) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// --------------------------------------------------------------- launchers
static inline int blocks_for(long n, int bs) { return (int)((n + bs - 1) / bs); }

// Each GPU holds its own copy of the scratch array at its own address: resolved once
// per device, with that device current, and kept.
hipError_t noalloc_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

void launch_fill_int(int* p, int n, int v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}
void launch_fill_double(double* p, long n, double v, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_fill_double, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_elements(const Mesh& m, const Elem& el, const double* x, const double* v,
                     const double* mat, const double* wind, double rho, int* status,
                     hipStream_t st) {
  long n = (long)m.nt + m.nh;
  if (m.wang)
    hipLaunchKernelGGL(k_elements<true>, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, el, x, v,
                       mat, wind, rho, status);
  else
    hipLaunchKernelGGL(k_elements<false>, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, el, x, v,
                       mat, wind, rho, status);
}

template <typename T, typename TM>
void launch_assemble(const Mesh& m, const Elem& el, const AssembleArgs<T, TM>& a, hipStream_t st) {
  // sixteen lanes per row for every mesh size: the same summation order whatever the
  // handle holds, so a sheet in a batch assembles bit for bit as on its own
  hipLaunchKernelGGL((k_assemble<T, TM, 16>), dim3(blocks_for(m.nv, 16)), dim3(256), 0, st, m, el, a);
}

template <typename TM>
size_t pcg_lds_bytes(int maxnz, int rows, int mat_home, int coarse_nc, int max_halo,
                     int xl_floats) {
  const size_t rh = rows + (size_t)(max_halo + 7) / 8 * 8;
  return (size_t)maxnz * rows * ((mat_home == kMatLds ? 9 * sizeof(TM) : 0) + sizeof(int)) +
         6 * sizeof(double) * rh + sizeof(int) * (rh - rows) +
         (coarse_nc > 0 ? sizeof(double) * ((size_t)coarse_nc + 5 * 6 * kMaxWgAgg +
                                            (size_t)pcg_threads(rows) / kMid * 36) +
                              sizeof(int) * (size_t)(coarse_nc / 6) * kMaxAggWg +
                              sizeof(float) * (size_t)xl_floats
                        : 0);
}

// Kernel variants: matrix streamed, in LDS or in registers (MatrixHome), coarse space
// or not, one or two workgroups of 256 threads per CU (the latter caps registers at
// 256 per lane; register-resident rows only with one).
template <typename TM, int OCC>
static const void* pcg_entry_occ(int mat_home, bool coarse) {
  if (coarse) {
    if (mat_home == kMatLds) return reinterpret_cast<const void*>(&k_pcg<TM, kMatLds, true, OCC>);
    return reinterpret_cast<const void*>(&k_pcg<TM, kMatStream, true, OCC>);
  }
  if (mat_home == kMatLds) return reinterpret_cast<const void*>(&k_pcg<TM, kMatLds, false, OCC>);
  return reinterpret_cast<const void*>(&k_pcg<TM, kMatStream, false, OCC>);
}

// split: register-resident rows over two wavefront teams (pcg_split)
template <typename TM>
static const void* pcg_entry(int mat_home, bool coarse, int occ, bool split) {
  if (mat_home == kMatReg && split)
    return coarse ? reinterpret_cast<const void*>(&k_pcg<TM, kMatRegHalf, true, 1>)
                  : reinterpret_cast<const void*>(&k_pcg<TM, kMatRegHalf, false, 1>);
  if (mat_home == kMatReg)
    return coarse ? reinterpret_cast<const void*>(&k_pcg<TM, kMatReg, true, 1>)
                  : reinterpret_cast<const void*>(&k_pcg<TM, kMatReg, false, 1>);
  return occ >= 2 ? pcg_entry_occ<TM, 2>(mat_home, coarse)
                  : pcg_entry_occ<TM, 1>(mat_home, coarse);
}

// Rejects shapes no variant handles: rows of more than kMaxRowBlocks blocks, and
// register-resident rows of more than kRegRowBlocks or with two workgroups per CU.
static bool pcg_shape_ok(int maxnz, int mat_home, int occ) {
  if (maxnz > kMaxRowBlocks) return false;
  if (mat_home == kMatReg && (maxnz > kRegRowBlocks || occ != 1)) return false;
  return mat_home >= kMatStream && mat_home <= kMatReg;
}

template <typename TM>
hipError_t pcg_prepare(size_t lds, int maxnz, int mat_home, bool coarse, int occ) {
  if (!pcg_shape_ok(maxnz, mat_home, occ)) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(pcg_entry<TM>(mat_home, coarse, occ, false),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess && mat_home == kMatReg)
    e = hipFuncSetAttribute(pcg_entry<TM>(mat_home, coarse, occ, true),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e;
}

template <typename TM>
hipError_t pcg_occupancy(int rows, size_t lds, int maxnz, int mat_home, bool coarse, int occ,
                         bool split, int* blocks_per_cu) {
  if (!pcg_shape_ok(maxnz, mat_home, occ)) return hipErrorInvalidValue;
  if (split && !pcg_can_split(rows, mat_home)) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, pcg_entry<TM>(mat_home, coarse, occ, split), pcg_block(rows, split), lds);
}

template <typename TM, int L, bool C, int O>
static void launch_pcg_v(dim3 grid, dim3 block, size_t lds, hipStream_t st, const Mesh& m,
                         const SolverPlan& pg, const SolverWork& w, const Coarse& cs,
                         const PcgArgs<TM>& a) {
  hipLaunchKernelGGL((k_pcg<TM, L, C, O>), grid, block, lds, st, m, pg, w, cs, a);
}

template <typename TM>
void launch_pcg(const Mesh& m, const SolverPlan& plan, const SolverWork& w, const Coarse& cs,
                const PcgArgs<TM>& a, hipStream_t st) {
  const bool coarse = cs.nagg > 0;
  size_t lds = pcg_lds_bytes<TM>(m.maxnz, plan.rows, plan.mat_home, coarse ? cs.max_nc : 0,
                                 plan.max_halo, coarse ? plan.xl_floats : 0);
  ZeroRanges z{};
  z.p[0] = w.barrier;
  z.n[0] = w.barrier_ints;
  z.p[1] = w.abort_flag;
  z.n[1] = 1;
  if (coarse) {
    z.p[2] = reinterpret_cast<int*>(w.tbuf);
    z.n[2] = 16 * m.nv;   // [2][4][nv] 64-bit words
    z.p[3] = reinterpret_cast<int*>(w.tred);
    z.n[3] = w.tred_ints;
  }
  const int most = std::max(std::max(z.n[0], z.n[2]), z.n[3]);
  hipLaunchKernelGGL(k_zero_ranges, dim3(std::min(blocks_for(most, 256), 1024)), dim3(256), 0,
                     st, z);
  // one launch per solver group (a set of whole sheets whose workgroups are co-resident)
  for (int g = 0; g < plan.ngroups; ++g) {
    SolverPlan pg = plan;
    pg.wg_base = plan.group_wg0_host[g];
    const dim3 grid(plan.group_wg0_host[g + 1] - pg.wg_base),
        block(pcg_block(plan.rows, plan.split != 0));
    if (plan.split) {
      if (coarse) launch_pcg_v<TM, kMatRegHalf, true, 1>(grid, block, lds, st, m, pg, w, cs, a);
      else launch_pcg_v<TM, kMatRegHalf, false, 1>(grid, block, lds, st, m, pg, w, cs, a);
      continue;
    }
    if (plan.mat_home == kMatReg) {
      // one workgroup per CU only (pcg_prepare rejects the rest)
      if (coarse) launch_pcg_v<TM, kMatReg, true, 1>(grid, block, lds, st, m, pg, w, cs, a);
      else launch_pcg_v<TM, kMatReg, false, 1>(grid, block, lds, st, m, pg, w, cs, a);
      continue;
    }
    const int sel = (plan.mat_home == kMatLds ? 4 : 0) + (coarse ? 2 : 0) + (plan.occ >= 2 ? 1 : 0);
    switch (sel) {
      case 0: launch_pcg_v<TM, kMatStream, false, 1>(grid, block, lds, st, m, pg, w, cs, a); break;
      case 1: launch_pcg_v<TM, kMatStream, false, 2>(grid, block, lds, st, m, pg, w, cs, a); break;
      case 2: launch_pcg_v<TM, kMatStream, true, 1>(grid, block, lds, st, m, pg, w, cs, a); break;
      case 3: launch_pcg_v<TM, kMatStream, true, 2>(grid, block, lds, st, m, pg, w, cs, a); break;
      case 4: launch_pcg_v<TM, kMatLds, false, 1>(grid, block, lds, st, m, pg, w, cs, a); break;
      case 5: launch_pcg_v<TM, kMatLds, false, 2>(grid, block, lds, st, m, pg, w, cs, a); break;
      case 6: launch_pcg_v<TM, kMatLds, true, 1>(grid, block, lds, st, m, pg, w, cs, a); break;
      default: launch_pcg_v<TM, kMatLds, true, 2>(grid, block, lds, st, m, pg, w, cs, a); break;
    }
  }
}

template <typename TM>
void launch_coarse_setup(const Mesh& m, const Coarse& c, const double* x, const TM* A,
                         long long coarse_doubles, const std::vector<int>& sweep_groups,
                         hipStream_t st) {
  if (c.nagg == 0) return;
  hipLaunchKernelGGL(k_coarse_frame, dim3(c.nagg), dim3(64), 0, st, m, c, x);
  launch_fill_double(c.mat, coarse_doubles, 0.0, st);
  if (c.npair > 0)
    hipLaunchKernelGGL((k_coarse_assemble<TM>), dim3(c.npair), dim3(256), 0, st, m, c, A);
  if (c.nmid > 0) hipLaunchKernelGGL((k_mid_setup<TM>), dim3(c.nmid), dim3(64), 0, st, m, c, x, A);
  hipLaunchKernelGGL(k_coarse_dead, dim3(blocks_for(c.nagg + m.ninst + m.ninst * c.sw_stride, 256)),
                     dim3(256), 0, st, c, m.ninst);
  // one launch per group of whole sheets whose workgroups are co-resident
  const size_t lds = gj_sweep_lds(c.sw_tpw);
  for (size_t g = 0; g + 1 < sweep_groups.size(); ++g) {
    const int n = sweep_groups[g + 1] - sweep_groups[g];
    if (n > 0)
      hipLaunchKernelGGL(k_gj_sweep, dim3(n), dim3(256), lds, st, c, m.ninst, sweep_groups[g]);
  }
}

size_t gj_sweep_lds(int tiles_per_wg) {
  return (size_t)tiles_per_wg * kGjTile * (kGjTile + 1) * sizeof(double);
}

hipError_t gj_sweep_occupancy(int tiles_per_wg, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, reinterpret_cast<const void*>(&k_gj_sweep), 256, gj_sweep_lds(tiles_per_wg));
}

template <typename T>
void launch_update(const Mesh& m, const double* xp, const double* vp, const double* dv, double h,
                   double* xn, double* vn, T* xout, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_update<T>, dim3(blocks_for(m.nv, 256)), dim3(256), 0, st, m.nv, m.pinned,
                     m.vert_inst, m.vold, xp, vp, dv, h, xn, vn, xout, status);
}

template <typename T>
void launch_init_state(const Mesh& m, const T* x0, const T* v0, double* xs, double* vs,
                       int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_init_state<T>, dim3(blocks_for(m.nv, 256)), dim3(256), 0, st, m.nv,
                     m.pinned, m.vert_inst, m.vold, x0, v0, xs, vs, status);
}

template <typename T>
void launch_adj_pre(const Mesh& m, const T* dl, double h, double* gx, const double* gv, double* u,
                    int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_pre<T>, dim3(blocks_for(m.nv, 256)), dim3(256), 0, st, m.nv, m.pinned,
                     m.vert_inst, m.vold, dl, h, gx, gv, u, status);
}

template <typename T>
void launch_adj_elements(const Mesh& m, const Elem& el, const AdjArgs<T>& a, hipStream_t st) {
  long n = (long)m.nt + m.nh;
  if (m.wang)
    hipLaunchKernelGGL((k_adj_elements<T, true>), dim3(blocks_for(n, 256)), dim3(256), 0, st, m, el, a);
  else
    hipLaunchKernelGGL((k_adj_elements<T, false>), dim3(blocks_for(n, 256)), dim3(256), 0, st, m, el,
                       a);
}

template <typename T>
void launch_adj_rows(const Mesh& m, const Elem& el, const AdjArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_rows<T>, dim3(blocks_for(m.nv, 16)), dim3(256), 0, st, m, el, a);
}

template <typename T>
void launch_adj_final(const Mesh& m, const double* gx, const double* gv, T* dx0, T* dv0,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_adj_final<T>, dim3(blocks_for(3L * m.nv, 256)), dim3(256), 0, st, m.nv,
                     m.vold, gx, gv, dx0, dv0);
}

void launch_material_sum(const Mesh& m, const Elem& el, double* out_mat, double* out_wind,
                         hipStream_t st) {
  if (!out_mat && !out_wind) return;
  hipLaunchKernelGGL(k_material_sum, dim3(m.ninst), dim3(256), 0, st, m, el, out_mat, out_wind);
}

#define PHISFT_INSTANTIATE_ASM(T, TM)                                                             \
  template void launch_assemble<T, TM>(const Mesh&, const Elem&, const AssembleArgs<T, TM>&,     \
                                       hipStream_t);
PHISFT_INSTANTIATE_ASM(float, float)
PHISFT_INSTANTIATE_ASM(float, double)
PHISFT_INSTANTIATE_ASM(double, float)
PHISFT_INSTANTIATE_ASM(double, double)

#define PHISFT_INSTANTIATE(T)                                                                    \
  template size_t pcg_lds_bytes<T>(int, int, int, int, int, int);                                \
  template hipError_t pcg_prepare<T>(size_t, int, int, bool, int);                               \
  template hipError_t pcg_occupancy<T>(int, size_t, int, int, bool, int, bool, int*);            \
  template void launch_pcg<T>(const Mesh&, const SolverPlan&, const SolverWork&, const Coarse&, \
                              const PcgArgs<T>&, hipStream_t);                                   \
  template void launch_coarse_setup<T>(const Mesh&, const Coarse&, const double*, const T*,      \
                                       long long, const std::vector<int>&, hipStream_t);         \
  template void launch_update<T>(const Mesh&, const double*, const double*, const double*,        \
                                 double, double*, double*, T*, int*, hipStream_t);               \
  template void launch_init_state<T>(const Mesh&, const T*, const T*, double*, double*, int*,    \
                                     hipStream_t);                                               \
  template void launch_adj_pre<T>(const Mesh&, const T*, double, double*, const double*,         \
                                  double*, int*, hipStream_t);                                   \
  template void launch_adj_elements<T>(const Mesh&, const Elem&, const AdjArgs<T>&,              \
                                       hipStream_t);                                             \
  template void launch_adj_rows<T>(const Mesh&, const Elem&, const AdjArgs<T>&, hipStream_t);   \
  template void launch_adj_final<T>(const Mesh&, const double*, const double*, T*, T*,       \
                                    hipStream_t);

PHISFT_INSTANTIATE(float)
PHISFT_INSTANTIATE(double)

}  // namespace phisft

#ifdef PHISFT_PHASES
extern "C" int phisft_read_phases(unsigned long long* out, int reset) {
  if (hipMemcpyFromSymbol(out, HIP_SYMBOL(phisft::g_phase), sizeof(phisft::g_phase)) != hipSuccess)
    return -1;
  if (reset) {
    static unsigned long long zero[512][8];
    if (hipMemcpyToSymbol(HIP_SYMBOL(phisft::g_phase), zero, sizeof(zero)) != hipSuccess) return -1;
  }
  return 0;
}
#endif

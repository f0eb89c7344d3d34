// phisft_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded FP64 CPU reference of the differentiable
// cloth simulator at the core of phi-SfT (Kairanda et al., "phi-SfT:
// Shape-from-Template with a Physics-Based Deformation Model", CVPR 2022):
//   * the deformation model S_t = PS(S_{t-1}; phi_{t-1})           (Sec. 3.1, Eq. 1-2)
//   * internal forces from stretching, bending and density          (Sec. 3.1, Eq. 3)
//   * one linearised backward-Euler step per frame, Delta v solved  (Sec. 3.1, Eq. 4-5)
//   * the adjoint of that step by implicit differentiation           (Sec. 3.1, backward pass)
//
// The paper defers the material model and the gradient formulas to cited work;
// the readings taken here are:
//   R1  h = dt (the paper writes h = 1), SI units.
//   R2  the unknown of the solve is Delta v, started from 0.
//   R3  df/dv = 0 (no damping, state-independent external forces).
//   R4  the corrective forces F_t enter the step's right-hand side as forces.
//   R6  lumped vertex mass m_i = d * sum_{t contains i} area_t / 3.
//   R7  stretching: isotropic St.Venant-Kirchhoff with lambda = 0,
//       E_m = area * (k_s / 2) * ||G||_F^2, G = (F^T F - I) / 2.
//   R8  bending: hinge energy E_b = k_b * c_e * (theta - theta_rest)^2 with
//       c_e = 3 |e_rest|^2 / (area_1 + area_2).
//   R9  the Jacobians are evaluated at the state of time t-1. The system
//       matrix uses K_sys = exact membrane Hessian + Gauss-Newton bending
//       Hessian 2 k_b c_e grad(theta) grad(theta)^T. Under compression the
//       exact membrane block can make A = M + h^2 K_sys indefinite; the solver
//       then reports a breakdown. A recorded variant keeps only the tension
//       part G+ of the strain in the membrane's stress term (compressive
//       principal strains clamped to zero), which makes A SPD in every state
//       but is not differentiable where a principal strain is zero; a
//       Gauss-Newton variant (no stress term) exists for the test showing that
//       it lets tensioned sheets gain energy. All three are selected through
//       orc_set_membrane_system. The adjoint uses the true Hessian K_exact
//       wherever the force itself is differentiated and the derivative of
//       K_sys in the state-derivative term.
//   R11 pinned vertices keep v = 0 and x = x_0 (Dirichlet rows/columns).
//   R20 stretch, anisotropic model (orc_set_material, model 1; the paper's S in R^24,
//       from Wang et al., whose formulas it does not give): four measures of the Green
//       strain in the sheet's material frame (u: the rest x axis projected into the
//       triangle's plane, the rest y axis where x is nearly normal to it; v = n x u):
//       s_1 = G_uu (warp), s_2 = G_vv (weft), s_3 = sqrt(2) G_uv (shear), s_4 = G_uu +
//       G_vv (area). Each has a piecewise-linear stress sigma_k(|s|) whose slope is
//       S[k][j] [N/m] on strain segment j (breaks 0, 0.25, 0.5, 1, 2, 4 %); the energy
//       density is sum_k psi_k(|s_k|) with psi' = sigma (even in s). S[k][j] = k_s for
//       k = 1..3 and S[4][j] = 0 give R7.
//   R21 bending, anisotropic model (the paper's B in R^15): the hinge energy
//       c_e Phi(theta - theta_rest), Phi(d) = 2 psi(|d|) with a piecewise-linear
//       sigma(|d|) whose slope on angle segment j (breaks 0, 0.05, 0.1, 0.2, 0.4 rad)
//       interpolates B[0][j], B[1][j], B[2][j] linearly in the angle between the
//       bending direction (in-plane, normal to the rest edge) and the warp axis u of
//       the hinge's first triangle, at 0, 45 and 90 degrees. B = k_b gives R8.
//   R19 wind (Eq. 2's w, a velocity; air density fixed, Sec. 3.4): every triangle
//       feels F_t = rho_air * area_t * |s| s n, n its unit normal at x_{t-1},
//       area_t its rest area, s = n . (w - mean of its vertices' v_{t-1}); each
//       vertex takes F_t / 3. Its velocity Jacobian enters the step matrix as
//       -h df/dv (Eq. 4-5); its position Jacobian is left out of the matrix (it is
//       not symmetric) and acts through the right-hand side only. The adjoint
//       differentiates exactly this step.
//
// Independence: nothing here is shared with the GPU library. Element stiffness
// blocks are obtained by probing the Hessian-vector product with unit vectors,
// third-derivative contractions by forward-mode dual numbers, and the linear
// solve is a textbook block-Jacobi preconditioned CG at a tight tolerance.
//
// Only the test suite, the package smoke check and the benchmark's CPU
// baseline load this library.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

// ---------------------------------------------------------------- status codes
enum {
  ORC_OK = 0,
  ORC_E_INVALID = -1,
  ORC_E_MESH = -2,
  ORC_E_NOT_CONVERGED = -5,
  ORC_E_INDEFINITE = -6,
  ORC_E_NONFINITE = -7,
};

// --------------------------------------------------- forward-mode dual numbers
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: implicit promotion is intended
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline Dual atan2(Dual y, Dual x) {
  double r2 = x.v * x.v + y.v * y.v;
  return Dual(std::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2);
}
inline double value_of(double a) { return a; }
inline double value_of(const Dual& a) { return a.v; }
inline double deriv_of(const Dual& a) { return a.d; }

// Hyper-dual numbers f(x + a e1 + b e2 + ab e1 e2) with e1^2 = e2^2 = 0: the ab part
// carries the exact mixed second derivative (used for the wind force's terms in the
// adjoint, where the velocity Jacobian is differentiated once more).
struct HDual {
  double v, a, b, ab;
  HDual() : v(0.0), a(0.0), b(0.0), ab(0.0) {}
  HDual(double x) : v(x), a(0.0), b(0.0), ab(0.0) {}  // NOLINT: implicit promotion is intended
  HDual(double x, double da, double db, double dab) : v(x), a(da), b(db), ab(dab) {}
};
inline HDual operator+(HDual p, HDual q) { return HDual(p.v + q.v, p.a + q.a, p.b + q.b, p.ab + q.ab); }
inline HDual operator-(HDual p, HDual q) { return HDual(p.v - q.v, p.a - q.a, p.b - q.b, p.ab - q.ab); }
inline HDual operator-(HDual p) { return HDual(-p.v, -p.a, -p.b, -p.ab); }
inline HDual operator*(HDual p, HDual q) {
  return HDual(p.v * q.v, p.a * q.v + p.v * q.a, p.b * q.v + p.v * q.b,
               p.ab * q.v + p.a * q.b + p.b * q.a + p.v * q.ab);
}
inline HDual recip(HDual q) {
  // 1/q: f = 1/v, f' = -1/v^2, f'' = 2/v^3
  const double f = 1.0 / q.v, f1 = -f * f, f2 = 2.0 * f * f * f;
  return HDual(f, f1 * q.a, f1 * q.b, f1 * q.ab + f2 * q.a * q.b);
}
inline HDual operator/(HDual p, HDual q) { return p * recip(q); }
inline HDual sqrt(HDual q) {
  const double f = std::sqrt(q.v), f1 = 0.5 / f, f2 = -0.25 / (f * q.v);
  return HDual(f, f1 * q.a, f1 * q.b, f1 * q.ab + f2 * q.a * q.b);
}
inline double value_of(const HDual& a) { return a.v; }
template <class S> inline S absval(const S& a) { return value_of(a) >= 0.0 ? a : -a; }
using std::atan2;
using std::sqrt;

// ------------------------------------------------------------- 3-vector tools
template <class S> inline void sub3(const S* a, const S* b, S* o) {
  for (int k = 0; k < 3; ++k) o[k] = a[k] - b[k];
}
template <class S> inline S dot3(const S* a, const S* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <class S> inline void cross3(const S* a, const S* b, S* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// ------------------------------------------------------------ membrane (R7)
// Deformation gradient F = [x_b - x_a, x_c - x_a] * B with B = D_m^{-1}
// (B stored row-major as B00 B01 B10 B11).
template <class S>
void deformation_gradient(const S* xa, const S* xb, const S* xc, const double* B, S F[3][2]) {
  S d1[3], d2[3];
  sub3(xb, xa, d1);
  sub3(xc, xa, d2);
  for (int r = 0; r < 3; ++r) {
    F[r][0] = d1[r] * B[0] + d2[r] * B[2];
    F[r][1] = d1[r] * B[1] + d2[r] * B[3];
  }
}

// Green strain G = (F^T F - I) / 2.
template <class S> void green_strain(S F[3][2], S G[2][2]) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      S s = F[0][a] * F[0][b] + F[1][a] * F[1][b] + F[2][a] * F[2][b];
      G[a][b] = 0.5 * (s - (a == b ? 1.0 : 0.0));
    }
}

// A 3x2 matrix Q = dPhi/dD_s is mapped to per-vertex gradients through
// D_s = [x_b - x_a, x_c - x_a]:  g_b = Q B^T e_0, g_c = Q B^T e_1, g_a = -(g_b + g_c).
template <class S> void scatter_ds(S Q[3][2], const double* B, S* ga, S* gb, S* gc) {
  for (int r = 0; r < 3; ++r) {
    gb[r] = Q[r][0] * B[0] + Q[r][1] * B[1];
    gc[r] = Q[r][0] * B[2] + Q[r][1] * B[3];
    ga[r] = -(gb[r] + gc[r]);
  }
}

template <class S>
S membrane_energy(const S* xa, const S* xb, const S* xc, const double* B, double area, double ks) {
  S F[3][2], G[2][2];
  deformation_gradient(xa, xb, xc, B, F);
  green_strain(F, G);
  S n2 = G[0][0] * G[0][0] + G[0][1] * G[0][1] + G[1][0] * G[1][0] + G[1][1] * G[1][1];
  return (area * ks * 0.5) * n2;
}

// dE_m/dx for the three vertices: first Piola stress P = k_s F G, dE/dD_s = area P B^T.
template <class S>
void membrane_gradient(const S* xa, const S* xb, const S* xc, const double* B, double area,
                       double ks, S* ga, S* gb, S* gc) {
  S F[3][2], G[2][2], Q[3][2];
  deformation_gradient(xa, xb, xc, B, F);
  green_strain(F, G);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 2; ++c) Q[r][c] = (area * ks) * (F[r][0] * G[0][c] + F[r][1] * G[1][c]);
  scatter_ds(Q, B, ga, gb, gc);
}

// Tension part of a symmetric 2x2 strain: G+ = sum_k max(lambda_k, 0) e_k e_k^T.
// Written as G+ = A I + B (G - m I) with m the mean eigenvalue, r the half gap,
// A = (s(l1) + s(l2)) / 2 and B = (s(l1) - s(l2)) / (l1 - l2) for s = max(., 0);
// at r = 0, B = s'(m) (taken as 0 at m = 0). This form stays finite for dual
// numbers at repeated eigenvalues.
template <class S> void tension_part(S G[2][2], S Gp[2][2]) {
  S a = G[0][0], b = 0.5 * (G[0][1] + G[1][0]), c = G[1][1];
  S m = 0.5 * (a + c), hd = 0.5 * (a - c);
  S q = hd * hd + b * b;
  S A, B;
  if (value_of(q) > 0.0) {
    S r = sqrt(q);
    S l1 = m + r, l2 = m - r;
    S s1 = value_of(l1) > 0.0 ? l1 : S(0.0);
    S s2 = value_of(l2) > 0.0 ? l2 : S(0.0);
    A = 0.5 * (s1 + s2);
    B = (s1 - s2) / (2.0 * r);
  } else {
    A = value_of(m) > 0.0 ? m : S(0.0);
    B = S(value_of(m) > 0.0 ? 1.0 : 0.0);
  }
  Gp[0][0] = A + B * hd;
  Gp[1][1] = A - B * hd;
  Gp[0][1] = B * b;
  Gp[1][0] = B * b;
}

// Stress term of the membrane Hessian (the dF G part of dP):
enum { GEO_NONE = 0, GEO_EXACT = 1, GEO_TENSION = 2 };

// Hessian-vector product of E_m along u:
// dP = k_s (dF G' + F sym(F^T dF)), (H u) = area dP B^T scattered, where G' is
// G itself (GEO_EXACT: the true Hessian), its tension part G+ (GEO_TENSION: the
// system-matrix block, positive semi-definite because both terms are), or 0
// (GEO_NONE: Gauss-Newton).
template <class S>
void membrane_hvp(const S* xa, const S* xb, const S* xc, const S* ua, const S* ub, const S* uc,
                  const double* B, double area, double ks, int geo, S* oa, S* ob, S* oc) {
  S F[3][2], G[2][2], Gs[2][2], dF[3][2], dG[2][2], Q[3][2];
  deformation_gradient(xa, xb, xc, B, F);
  green_strain(F, G);
  if (geo == GEO_TENSION) {
    tension_part(G, Gs);
  } else {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) Gs[a][b] = geo == GEO_EXACT ? G[a][b] : S(0.0);
  }
  deformation_gradient(ua, ub, uc, B, dF);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      S s1 = F[0][a] * dF[0][b] + F[1][a] * dF[1][b] + F[2][a] * dF[2][b];
      S s2 = dF[0][a] * F[0][b] + dF[1][a] * F[1][b] + dF[2][a] * F[2][b];
      dG[a][b] = 0.5 * (s1 + s2);
    }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 2; ++c)
      Q[r][c] = (area * ks) * (dF[r][0] * Gs[0][c] + dF[r][1] * Gs[1][c] + F[r][0] * dG[0][c] +
                               F[r][1] * dG[1][c]);
  scatter_ds(Q, B, oa, ob, oc);
}

// ------------------------------------------- anisotropic material (R20, R21)
constexpr int kWangStretch = 24, kWangBend = 15, kWangParams = 40;
const double kStrainBreaks[6] = {0.0, 0.0025, 0.005, 0.01, 0.02, 0.04};
const double kBendBreaks[5] = {0.0, 0.05, 0.1, 0.2, 0.4};

// Piecewise-linear response of a deformation measure t >= 0 whose stiffness is k[j] on
// [b_j, b_{j+1}) (the last segment unbounded): sigma(t) = integral of the stiffness
// from 0 to t, psi(t) = integral of sigma from 0 to t, kt = the stiffness at t.
template <class S>
void pw_response(const S& t, const double* k, const double* b, int n, S& sigma, S& psi,
                 double& kt) {
  double sig = 0.0, ps = 0.0;
  int j = 0;
  while (j + 1 < n && value_of(t) >= b[j + 1]) {
    const double len = b[j + 1] - b[j];
    ps += sig * len + 0.5 * k[j] * len * len;
    sig += k[j] * len;
    ++j;
  }
  S r = t - b[j];
  psi = ps + sig * r + 0.5 * k[j] * r * r;
  sigma = sig + k[j] * r;
  kt = k[j];
}

// N : G for a symmetric 2x2 N stored as (N_00, N_01, N_11).
template <class S> S ncontract(const double* N, S G[2][2]) {
  return N[0] * G[0][0] + N[1] * (G[0][1] + G[1][0]) + N[2] * G[1][1];
}

// R20 energy density W(G) of a triangle whose four measure tensors (local frame) are
// N[0..11]; also the second Piola stress dW/dG and each measure's segment stiffness.
template <class S>
S wang_stress(S G[2][2], const double* N, const double* Sp, S S2[2][2], double c[4]) {
  S W(0.0);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) S2[a][b] = S(0.0);
  for (int k = 0; k < 4; ++k) {
    const double* Nk = &N[3 * k];
    S sk = ncontract(Nk, G);
    const bool neg = value_of(sk) < 0.0;
    S t = neg ? -sk : sk;
    S sig, psi;
    pw_response(t, &Sp[6 * k], kStrainBreaks, 6, sig, psi, c[k]);
    S sg = neg ? -sig : sig;
    S2[0][0] = S2[0][0] + sg * Nk[0];
    S2[0][1] = S2[0][1] + sg * Nk[1];
    S2[1][0] = S2[1][0] + sg * Nk[1];
    S2[1][1] = S2[1][1] + sg * Nk[2];
    W = W + psi;
  }
  return W;
}

template <class S>
S wang_membrane_energy(const S* xa, const S* xb, const S* xc, const double* B, double area,
                       const double* N, const double* Sp) {
  S F[3][2], G[2][2], S2[2][2];
  double c[4];
  deformation_gradient(xa, xb, xc, B, F);
  green_strain(F, G);
  return area * wang_stress(G, N, Sp, S2, c);
}

// dE/dx: dE/dD_s = area F S2 B^T.
template <class S>
void wang_membrane_gradient(const S* xa, const S* xb, const S* xc, const double* B, double area,
                            const double* N, const double* Sp, S* ga, S* gb, S* gc) {
  S F[3][2], G[2][2], S2[2][2], Q[3][2];
  double c[4];
  deformation_gradient(xa, xb, xc, B, F);
  green_strain(F, G);
  wang_stress(G, N, Sp, S2, c);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 2; ++k) Q[r][k] = area * (F[r][0] * S2[0][k] + F[r][1] * S2[1][k]);
  scatter_ds(Q, B, ga, gb, gc);
}

// Hessian-vector product along u: dP = dF S2' + F dS2, dS2 = sum_k c_k (N_k : dG) N_k
// (the stiffness of each measure is constant on its segment); S2' = S2 (GEO_EXACT) or 0
// (GEO_NONE).
template <class S>
void wang_membrane_hvp(const S* xa, const S* xb, const S* xc, const S* ua, const S* ub,
                       const S* uc, const double* B, double area, const double* N,
                       const double* Sp, int geo, S* oa, S* ob, S* oc) {
  S F[3][2], G[2][2], S2[2][2], dF[3][2], dG[2][2], dS[2][2], Q[3][2];
  double c[4];
  deformation_gradient(xa, xb, xc, B, F);
  green_strain(F, G);
  wang_stress(G, N, Sp, S2, c);
  deformation_gradient(ua, ub, uc, B, dF);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      S s1 = F[0][a] * dF[0][b] + F[1][a] * dF[1][b] + F[2][a] * dF[2][b];
      S s2 = dF[0][a] * F[0][b] + dF[1][a] * F[1][b] + dF[2][a] * F[2][b];
      dG[a][b] = 0.5 * (s1 + s2);
      dS[a][b] = S(0.0);
    }
  for (int k = 0; k < 4; ++k) {
    const double* Nk = &N[3 * k];
    S m = c[k] * ncontract(Nk, dG);
    dS[0][0] = dS[0][0] + m * Nk[0];
    dS[0][1] = dS[0][1] + m * Nk[1];
    dS[1][0] = dS[1][0] + m * Nk[1];
    dS[1][1] = dS[1][1] + m * Nk[2];
  }
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 2; ++k) {
      S t = F[r][0] * dS[0][k] + F[r][1] * dS[1][k];
      if (geo == GEO_EXACT) t = t + dF[r][0] * S2[0][k] + dF[r][1] * S2[1][k];
      Q[r][k] = area * t;
    }
  scatter_ds(Q, B, oa, ob, oc);
}

// ------------------------------------------------------------- bending (R8)
// Hinge (x0, x1 | x2, x3): edge x0 -> x1, triangle (x0, x1, x2) and the
// neighbour (x1, x0, x3). theta = atan2((n1 x n2) . e, n1 . n2) with unit normals.
template <class S> S hinge_theta(const S* x0, const S* x1, const S* x2, const S* x3) {
  S e[3], a[3], b[3], n1[3], n2[3], c[3];
  sub3(x1, x0, e);
  sub3(x2, x0, a);
  cross3(e, a, n1);  // (x1 - x0) x (x2 - x0)
  S me[3], d[3];
  sub3(x0, x1, me);
  sub3(x3, x1, d);
  cross3(me, d, n2);  // (x0 - x1) x (x3 - x1)
  S l1 = sqrt(dot3(n1, n1)), l2 = sqrt(dot3(n2, n2)), le = sqrt(dot3(e, e));
  for (int k = 0; k < 3; ++k) {
    n1[k] = n1[k] / l1;
    n2[k] = n2[k] / l2;
    b[k] = e[k] / le;
  }
  cross3(n1, n2, c);
  return atan2(dot3(c, b), dot3(n1, n2));
}

// Closed-form gradient of theta (Bridson et al. 2003; Grinspun et al. 2003):
// wings get -|e| n_k / |n_k|^2, edge vertices the lever-rule combination
// that makes the gradient translation- and rotation-free.
template <class S>
void hinge_theta_grad(const S* x0, const S* x1, const S* x2, const S* x3, S* g0, S* g1, S* g2,
                      S* g3) {
  S e[3], a[3], n1[3], n2[3], me[3], d[3];
  sub3(x1, x0, e);
  sub3(x2, x0, a);
  cross3(e, a, n1);
  sub3(x0, x1, me);
  sub3(x3, x1, d);
  cross3(me, d, n2);
  S ee = dot3(e, e), le = sqrt(ee);
  S q1 = dot3(n1, n1), q2 = dot3(n2, n2);
  S w2[3], w3[3];
  S t1 = dot3(a, e) / ee;
  S x3m0[3];
  sub3(x3, x0, x3m0);
  S t2 = dot3(x3m0, e) / ee;
  for (int k = 0; k < 3; ++k) {
    w2[k] = -le * n1[k] / q1;
    w3[k] = -le * n2[k] / q2;
  }
  for (int k = 0; k < 3; ++k) {
    g2[k] = w2[k];
    g3[k] = w3[k];
    g0[k] = -(1.0 - t1) * w2[k] - (1.0 - t2) * w3[k];
    g1[k] = -t1 * w2[k] - t2 * w3[k];
  }
}

// ------------------------------------------------- aerodynamic force (R19)
// Total force of the wind on one triangle (each vertex takes a third):
// rho_area * |s| s n with n = N / |N|, N = (x_b - x_a) x (x_c - x_a), and
// s = n . (w - (v_a + v_b + v_c) / 3).
template <class S>
void aero_force(const S* xa, const S* xb, const S* xc, const S* va, const S* vb, const S* vc,
                const S* w, double rho_area, S* F) {
  S e1[3], e2[3], N[3], n[3], rel[3];
  sub3(xb, xa, e1);
  sub3(xc, xa, e2);
  cross3(e1, e2, N);
  S ln = sqrt(dot3(N, N));
  for (int k = 0; k < 3; ++k) {
    n[k] = N[k] / ln;
    rel[k] = w[k] - (va[k] + vb[k] + vc[k]) / 3.0;
  }
  S sn = dot3(n, rel);
  S mag = absval(sn) * sn * rho_area;
  for (int k = 0; k < 3; ++k) F[k] = mag * n[k];
}

// ------------------------------------------------------------------ problem
struct Problem {
  int nv = 0, nt = 0, nh = 0;
  std::vector<int> tri;        // nt*3
  std::vector<double> rest;    // nv*3
  std::vector<char> pinned;    // nv
  std::vector<double> Bm;      // nt*4
  std::vector<double> area;    // nt
  std::vector<double> varea;   // nv
  std::vector<int> hv;         // nh*4
  std::vector<double> hce;     // nh
  std::vector<double> hrest;   // nh
  double ks = 0, kb = 0, dens = 0, h = 0.01;
  double grav[3] = {0, 0, -9.81};
  double cg_tol = 1e-12;
  int cg_max_iter = 100000;
  // Stress term of the system matrix's membrane block: GEO_EXACT (default, the
  // true Hessian), GEO_TENSION (tension part only) or GEO_NONE (Gauss-Newton).
  int mem_geo = GEO_EXACT;
  // wind (R19): off unless set; velocity w [m/s] and air density [kg/m^3]
  bool wind_on = false;
  double wind[3] = {0, 0, 0};
  double rho_air = 1.0;
  std::vector<int> rowptr, col;  // CSR pattern of the vertex blocks
  int last_status = ORC_OK;
  // anisotropic material (R20, R21): on when wang; per triangle the four measure
  // tensors in its local frame [nt][4][3], per hinge the direction weights [nh][3]
  bool wang = false;
  double wS[kWangStretch] = {}, wB[kWangBend] = {};
  std::vector<double> Nm, hdw;
};

// The stiffness parameters of the internal forces: the isotropic scales (k_s, k_b) or
// the anisotropic tables. The adjoint evaluates forces and stiffness products with
// unit parameters (the model is linear in every parameter for a fixed state).
struct Mat {
  bool wang = false;
  double ks = 0.0, kb = 0.0;
  double S[kWangStretch] = {}, B[kWangBend] = {};
};

Mat iso_mat(double ks, double kb) {
  Mat M;
  M.ks = ks;
  M.kb = kb;
  return M;
}

Mat problem_mat(const Problem& P) {
  Mat M = iso_mat(P.ks, P.kb);
  M.wang = P.wang;
  std::copy(P.wS, P.wS + kWangStretch, M.S);
  std::copy(P.wB, P.wB + kWangBend, M.B);
  return M;
}

// Hinge e's bending response at the angle change dth: the force scale s = dE/dtheta
// and the Gauss-Newton weight w = d^2E/dtheta^2 (and the energy).
void hinge_response(const Problem& P, const Mat& M, int e, double dth, double& s, double& w,
                    double* energy = nullptr) {
  const double ce = P.hce[e];
  if (!M.wang) {
    s = 2.0 * M.kb * ce * dth;
    w = 2.0 * M.kb * ce;
    if (energy) *energy = M.kb * ce * dth * dth;
    return;
  }
  double keff[5];
  for (int j = 0; j < 5; ++j) {
    keff[j] = 0.0;
    for (int a = 0; a < 3; ++a) keff[j] += P.hdw[3 * e + a] * M.B[5 * a + j];
  }
  const double t = std::fabs(dth);
  double sig, psi, kt;
  pw_response(t, keff, kBendBreaks, 5, sig, psi, kt);
  s = 2.0 * ce * (dth < 0.0 ? -sig : sig);
  w = 2.0 * ce * kt;
  if (energy) *energy = 2.0 * ce * psi;
}

template <class S>
void mem_gradient(const Problem& P, const Mat& M, int t, const S* xa, const S* xb, const S* xc,
                  S* ga, S* gb, S* gc) {
  if (M.wang)
    wang_membrane_gradient<S>(xa, xb, xc, &P.Bm[4 * t], P.area[t], &P.Nm[12 * t], M.S, ga, gb, gc);
  else
    membrane_gradient<S>(xa, xb, xc, &P.Bm[4 * t], P.area[t], M.ks, ga, gb, gc);
}

template <class S>
void mem_hvp(const Problem& P, const Mat& M, int t, const S* xa, const S* xb, const S* xc,
             const S* ua, const S* ub, const S* uc, int geo, S* oa, S* ob, S* oc) {
  if (M.wang)
    wang_membrane_hvp<S>(xa, xb, xc, ua, ub, uc, &P.Bm[4 * t], P.area[t], &P.Nm[12 * t], M.S, geo,
                         oa, ob, oc);
  else
    membrane_hvp<S>(xa, xb, xc, ua, ub, uc, &P.Bm[4 * t], P.area[t], M.ks, geo, oa, ob, oc);
}

// The warp axis of a rest plane with unit normal n: the x axis projected into the plane,
// or the y axis where x is within about 0.06 degrees of the normal (R20).
void material_axis(const double* n, double* u) {
  double ax[3] = {1.0, 0.0, 0.0};
  double d = dot3(ax, n);
  for (int k = 0; k < 3; ++k) u[k] = ax[k] - d * n[k];
  double l = std::sqrt(dot3(u, u));
  if (!(l > 1e-3)) {
    double ay[3] = {0.0, 1.0, 0.0};
    d = dot3(ay, n);
    for (int k = 0; k < 3; ++k) u[k] = ay[k] - d * n[k];
    l = std::sqrt(dot3(u, u));
  }
  for (int k = 0; k < 3; ++k) u[k] /= l;
}

int build_problem(Problem& P, int nv, int nt, const int* tris, const double* rest, const int* pins,
                  int npins) {
  if (nv <= 0 || nt <= 0 || !tris || !rest) return ORC_E_INVALID;
  P.nv = nv;
  P.nt = nt;
  P.tri.assign(tris, tris + 3 * nt);
  P.rest.assign(rest, rest + 3 * nv);
  P.pinned.assign(nv, 0);
  for (int k = 0; k < npins; ++k) {
    if (pins[k] < 0 || pins[k] >= nv) return ORC_E_INVALID;
    P.pinned[pins[k]] = 1;
  }
  for (int k = 0; k < 3 * nt; ++k)
    if (P.tri[k] < 0 || P.tri[k] >= nv) return ORC_E_MESH;
  for (int k = 0; k < 3 * nv; ++k)
    if (!std::isfinite(rest[k])) return ORC_E_MESH;
  // Length scale for the degenerate-triangle test: bounding-box diagonal.
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], rest[3 * i + k]);
      hi[k] = std::max(hi[k], rest[3 * i + k]);
    }
  double diag2 = 0;
  for (int k = 0; k < 3; ++k) diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);

  // Rest frame per triangle: e1 along X_b - X_a, e2 = n x e1 (in-plane), D_m in that frame.
  P.Bm.assign(4 * nt, 0.0);
  P.Nm.clear();
  P.area.assign(nt, 0.0);
  P.varea.assign(nv, 0.0);
  for (int t = 0; t < nt; ++t) {
    const double* Xa = &rest[3 * P.tri[3 * t]];
    const double* Xb = &rest[3 * P.tri[3 * t + 1]];
    const double* Xc = &rest[3 * P.tri[3 * t + 2]];
    double d1[3], d2[3], n[3], e1[3], e2[3];
    sub3(Xb, Xa, d1);
    sub3(Xc, Xa, d2);
    cross3(d1, d2, n);
    double ln = std::sqrt(dot3(n, n)), l1 = std::sqrt(dot3(d1, d1));
    if (!(0.5 * ln > 1e-14 * diag2) || !(l1 > 0)) return ORC_E_MESH;
    for (int k = 0; k < 3; ++k) {
      e1[k] = d1[k] / l1;
      n[k] /= ln;
    }
    cross3(n, e1, e2);
    double Dm00 = dot3(d1, e1), Dm01 = dot3(d2, e1), Dm10 = dot3(d1, e2), Dm11 = dot3(d2, e2);
    double det = Dm00 * Dm11 - Dm01 * Dm10;
    P.area[t] = 0.5 * det;
    if (!(P.area[t] > 1e-14 * diag2)) return ORC_E_MESH;
    P.Bm[4 * t + 0] = Dm11 / det;
    P.Bm[4 * t + 1] = -Dm01 / det;
    P.Bm[4 * t + 2] = -Dm10 / det;
    P.Bm[4 * t + 3] = Dm00 / det;
    for (int k = 0; k < 3; ++k) P.varea[P.tri[3 * t + k]] += P.area[t] / 3.0;
    // material frame (R20): u = the rest x axis projected into the plane (y if x is
    // nearly normal to it), v = n x u, written in the local frame (e1, e2)
    double u3[3];
    material_axis(n, u3);
    const double u0 = dot3(u3, e1), u1 = dot3(u3, e2);
    const double v0 = -u1, v1 = u0, r2 = std::sqrt(2.0);
    const double Nt[12] = {u0 * u0, u0 * u1, u1 * u1, v0 * v0, v0 * v1, v1 * v1,
                           r2 * u0 * v0, (u0 * v1 + v0 * u1) / r2, r2 * u1 * v1, 1.0, 0.0, 1.0};
    P.Nm.insert(P.Nm.end(), Nt, Nt + 12);
  }

  // Hinges: every edge used once in each direction by two triangles.
  std::map<std::pair<int, int>, std::pair<int, int>> directed;  // (i,j) -> (triangle, opposite)
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int i = P.tri[3 * t + k], j = P.tri[3 * t + (k + 1) % 3], o = P.tri[3 * t + (k + 2) % 3];
      if (i == j || j == o || i == o) return ORC_E_MESH;
      auto key = std::make_pair(i, j);
      if (directed.count(key)) return ORC_E_MESH;  // inconsistent orientation / non-manifold
      directed[key] = std::make_pair(t, o);
    }
  P.hv.clear();
  P.hce.clear();
  P.hrest.clear();
  P.hdw.clear();
  for (auto& kv : directed) {
    int i = kv.first.first, j = kv.first.second;
    if (i > j) continue;  // visit each undirected edge once, from its smaller endpoint
    auto it = directed.find(std::make_pair(j, i));
    if (it == directed.end()) continue;  // boundary edge
    int t1 = kv.second.first, o1 = kv.second.second;
    int t2 = it->second.first, o2 = it->second.second;
    P.hv.push_back(i);
    P.hv.push_back(j);
    P.hv.push_back(o1);
    P.hv.push_back(o2);
    double e[3];
    sub3(&rest[3 * j], &rest[3 * i], e);
    P.hce.push_back(3.0 * dot3(e, e) / (P.area[t1] + P.area[t2]));
    P.hrest.push_back(hinge_theta(&rest[3 * i], &rest[3 * j], &rest[3 * o1], &rest[3 * o2]));
    // bending direction (R21): in the first triangle's plane, normal to the edge; its
    // angle phi to that triangle's warp axis, folded into [0, 90] degrees, weights the
    // 0, 45 and 90 degree tables linearly
    double d2[3], n1[3], ue[3], bd[3], u3[3];
    sub3(&rest[3 * o1], &rest[3 * i], d2);
    cross3(e, d2, n1);
    const double ln1 = std::sqrt(dot3(n1, n1)), le = std::sqrt(dot3(e, e));
    for (int k = 0; k < 3; ++k) {
      n1[k] /= ln1;
      ue[k] = e[k] / le;
    }
    cross3(n1, ue, bd);
    material_axis(n1, u3);
    const double cphi = std::min(1.0, std::fabs(dot3(bd, u3)));
    const double q = std::acos(cphi) / (std::atan(1.0));   // phi / 45 degrees, in [0, 2]
    P.hdw.push_back(q <= 1.0 ? 1.0 - q : 0.0);
    P.hdw.push_back(q <= 1.0 ? q : 2.0 - q);
    P.hdw.push_back(q <= 1.0 ? 0.0 : q - 1.0);
  }
  P.nh = (int)P.hce.size();

  // Block sparsity pattern: vertices coupled by a triangle or by a hinge.
  std::vector<std::vector<int>> adj(nv);
  auto link = [&](int a, int b) { adj[a].push_back(b); };
  for (int t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) link(P.tri[3 * t + a], P.tri[3 * t + b]);
  for (int e = 0; e < P.nh; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) link(P.hv[4 * e + a], P.hv[4 * e + b]);
  P.rowptr.assign(nv + 1, 0);
  P.col.clear();
  for (int i = 0; i < nv; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
    P.rowptr[i + 1] = P.rowptr[i] + (int)adj[i].size();
    P.col.insert(P.col.end(), adj[i].begin(), adj[i].end());
  }
  return ORC_OK;
}

// ----------------------------------------------------- global force routines
// Internal energy E = E_m + E_b.
double internal_energy(const Problem& P, const double* x, double* em_out, double* eb_out) {
  const Mat M = problem_mat(P);
  double em = 0, eb = 0;
  for (int t = 0; t < P.nt; ++t) {
    const int* v = &P.tri[3 * t];
    if (M.wang)
      em += wang_membrane_energy<double>(&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &P.Bm[4 * t],
                                         P.area[t], &P.Nm[12 * t], M.S);
    else
      em += membrane_energy<double>(&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &P.Bm[4 * t],
                                    P.area[t], P.ks);
  }
  for (int e = 0; e < P.nh; ++e) {
    const int* v = &P.hv[4 * e];
    double th = hinge_theta<double>(&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &x[3 * v[3]]);
    double s, w, en;
    hinge_response(P, M, e, th - P.hrest[e], s, w, &en);
    eb += en;
  }
  if (em_out) *em_out = em;
  if (eb_out) *eb_out = eb;
  return em + eb;
}

// Internal force f = -dE/dx for the stiffness parameters M (the adjoint passes unit
// parameters for the material derivatives).
void internal_force(const Problem& P, const double* x, const Mat& M, double* f) {
  std::fill(f, f + 3 * P.nv, 0.0);
  for (int t = 0; t < P.nt; ++t) {
    const int* v = &P.tri[3 * t];
    double g[3][3];
    mem_gradient<double>(P, M, t, &x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], g[0], g[1], g[2]);
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) f[3 * v[a] + k] -= g[a][k];
  }
  for (int e = 0; e < P.nh; ++e) {
    const int* v = &P.hv[4 * e];
    double g[4][3];
    const double* X[4] = {&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &x[3 * v[3]]};
    double th = hinge_theta<double>(X[0], X[1], X[2], X[3]);
    hinge_theta_grad<double>(X[0], X[1], X[2], X[3], g[0], g[1], g[2], g[3]);
    double s, w;
    hinge_response(P, M, e, th - P.hrest[e], s, w);
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) f[3 * v[a] + k] -= s * g[a][k];
  }
}

// out = K u. exact = true: the true Hessian of E (for the parameters M). exact =
// false: the system matrix K_sys (Gauss-Newton bending and the configured membrane
// block).
void stiffness_apply(const Problem& P, const double* x, const double* u, const Mat& M, bool exact,
                     double* out) {
  std::fill(out, out + 3 * P.nv, 0.0);
  for (int t = 0; t < P.nt; ++t) {
    const int* v = &P.tri[3 * t];
    double o[3][3];
    mem_hvp<double>(P, M, t, &x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &u[3 * v[0]], &u[3 * v[1]],
                    &u[3 * v[2]], exact ? GEO_EXACT : P.mem_geo, o[0], o[1], o[2]);
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) out[3 * v[a] + k] += o[a][k];
  }
  for (int e = 0; e < P.nh; ++e) {
    const int* v = &P.hv[4 * e];
    double g[4][3];
    const double* X[4] = {&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &x[3 * v[3]]};
    hinge_theta_grad<double>(X[0], X[1], X[2], X[3], g[0], g[1], g[2], g[3]);
    double th = hinge_theta<double>(X[0], X[1], X[2], X[3]);
    double s, w;
    hinge_response(P, M, e, th - P.hrest[e], s, w);
    double gu = 0;
    for (int a = 0; a < 4; ++a) gu += dot3(g[a], &u[3 * v[a]]);
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) out[3 * v[a] + k] += w * gu * g[a][k];
    if (exact) {
      // s * Hess(theta) u, the directional derivative of grad(theta) along u
      Dual Xd[4][3], gd[4][3];
      for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) Xd[a][k] = Dual(X[a][k], u[3 * v[a] + k]);
      hinge_theta_grad<Dual>(Xd[0], Xd[1], Xd[2], Xd[3], gd[0], gd[1], gd[2], gd[3]);
      for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) out[3 * v[a] + k] += s * deriv_of(gd[a][k]);
    }
  }
}

// out = grad_x [ mu^T K_sys(x) w ], each element differentiated by dual numbers
// along every one of its coordinates.
void third_contraction(const Problem& P, const double* x, const double* mu, const double* w,
                       double* out) {
  const Mat M = problem_mat(P);
  std::fill(out, out + 3 * P.nv, 0.0);
  for (int t = 0; t < P.nt; ++t) {
    const int* v = &P.tri[3 * t];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) {
        Dual X[3][3], W[3][3], o[3][3];
        for (int b = 0; b < 3; ++b)
          for (int m = 0; m < 3; ++m) {
            X[b][m] = Dual(x[3 * v[b] + m], (a == b && k == m) ? 1.0 : 0.0);
            W[b][m] = Dual(w[3 * v[b] + m]);
          }
        mem_hvp<Dual>(P, M, t, X[0], X[1], X[2], W[0], W[1], W[2], P.mem_geo, o[0], o[1], o[2]);
        double s = 0;
        for (int b = 0; b < 3; ++b)
          for (int m = 0; m < 3; ++m) s += mu[3 * v[b] + m] * deriv_of(o[b][m]);
        out[3 * v[a] + k] += s;
      }
  }
  for (int e = 0; e < P.nh; ++e) {
    const int* v = &P.hv[4 * e];
    // the Gauss-Newton weight: constant in x on the angle segment (R8: everywhere)
    double s_unused, wgt;
    hinge_response(P, M, e,
                   hinge_theta<double>(&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &x[3 * v[3]]) -
                       P.hrest[e],
                   s_unused, wgt);
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) {
        Dual X[4][3], g[4][3];
        for (int b = 0; b < 4; ++b)
          for (int m = 0; m < 3; ++m)
            X[b][m] = Dual(x[3 * v[b] + m], (a == b && k == m) ? 1.0 : 0.0);
        hinge_theta_grad<Dual>(X[0], X[1], X[2], X[3], g[0], g[1], g[2], g[3]);
        Dual gm(0.0), gw(0.0);
        for (int b = 0; b < 4; ++b)
          for (int m = 0; m < 3; ++m) {
            gm = gm + g[b][m] * Dual(mu[3 * v[b] + m]);
            gw = gw + g[b][m] * Dual(w[3 * v[b] + m]);
          }
        Dual phi = Dual(wgt) * gm * gw;
        out[3 * v[a] + k] += deriv_of(phi);
      }
  }
}

// ------------------------------------------------------- assembled K_sys (CSR)
int find_slot(const Problem& P, int i, int j) {
  const int* b = &P.col[P.rowptr[i]];
  const int* e = &P.col[P.rowptr[i + 1]];
  const int* it = std::lower_bound(b, e, j);
  return (int)(it - &P.col[0]);
}

// K_sys blocks (nnzb * 9, row-major 3x3), assembled by probing each element's
// Hessian-vector product with unit vectors.
void assemble_ksys(const Problem& P, const double* x, std::vector<double>& K) {
  const Mat M = problem_mat(P);
  K.assign(9 * P.col.size(), 0.0);
  for (int t = 0; t < P.nt; ++t) {
    const int* v = &P.tri[3 * t];
    const double* X[3] = {&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]]};
    for (int b = 0; b < 3; ++b)
      for (int m = 0; m < 3; ++m) {
        double U[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        U[b][m] = 1.0;
        double o[3][3];
        mem_hvp<double>(P, M, t, X[0], X[1], X[2], U[0], U[1], U[2], P.mem_geo, o[0], o[1], o[2]);
        // column (b, m) of the element Hessian
        for (int a = 0; a < 3; ++a) {
          int s = find_slot(P, v[a], v[b]);
          for (int k = 0; k < 3; ++k) K[9 * s + 3 * k + m] += o[a][k];
        }
      }
  }
  for (int e = 0; e < P.nh; ++e) {
    const int* v = &P.hv[4 * e];
    double g[4][3];
    hinge_theta_grad<double>(&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &x[3 * v[3]], g[0], g[1],
                             g[2], g[3]);
    double s_unused, w;
    hinge_response(P, M, e,
                   hinge_theta<double>(&x[3 * v[0]], &x[3 * v[1]], &x[3 * v[2]], &x[3 * v[3]]) -
                       P.hrest[e],
                   s_unused, w);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int s = find_slot(P, v[a], v[b]);
        for (int k = 0; k < 3; ++k)
          for (int m = 0; m < 3; ++m) K[9 * s + 3 * k + m] += w * g[a][k] * g[b][m];
      }
  }
}

void csr_apply(const Problem& P, const std::vector<double>& K, const double* u, double* out) {
  for (int i = 0; i < P.nv; ++i) {
    double acc[3] = {0, 0, 0};
    for (int s = P.rowptr[i]; s < P.rowptr[i + 1]; ++s) {
      const double* blk = &K[9 * s];
      const double* uj = &u[3 * P.col[s]];
      for (int k = 0; k < 3; ++k) acc[k] += blk[3 * k] * uj[0] + blk[3 * k + 1] * uj[1] + blk[3 * k + 2] * uj[2];
    }
    for (int k = 0; k < 3; ++k) out[3 * i + k] = acc[k];
  }
}

bool invert3(const double* a, double* inv) {
  double c00 = a[4] * a[8] - a[5] * a[7];
  double c01 = a[5] * a[6] - a[3] * a[8];
  double c02 = a[3] * a[7] - a[4] * a[6];
  double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (!(std::fabs(det) > 0) || !std::isfinite(det)) return false;
  double id = 1.0 / det;
  inv[0] = c00 * id;
  inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  inv[3] = c01 * id;
  inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  inv[6] = c02 * id;
  inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  return true;
}

// Wind force (R19) at (x, v), added to f [V][3].
void wind_force(const Problem& P, const double* x, const double* v, double* f) {
  for (int t = 0; t < P.nt; ++t) {
    const int* a = &P.tri[3 * t];
    double F[3];
    aero_force<double>(&x[3 * a[0]], &x[3 * a[1]], &x[3 * a[2]], &v[3 * a[0]], &v[3 * a[1]],
                       &v[3 * a[2]], P.wind, P.rho_air * P.area[t], F);
    for (int q = 0; q < 3; ++q)
      for (int k = 0; k < 3; ++k) f[3 * a[q] + k] += F[k] / 3.0;
  }
}

// D = -df_wind/dv in CSR blocks, each element's velocity Jacobian probed column by
// column with dual numbers.
void wind_damping(const Problem& P, const double* x, const double* v, std::vector<double>& D) {
  D.assign(9 * P.col.size(), 0.0);
  for (int t = 0; t < P.nt; ++t) {
    const int* a = &P.tri[3 * t];
    Dual X[3][3], W[3];
    for (int q = 0; q < 3; ++q)
      for (int k = 0; k < 3; ++k) X[q][k] = Dual(x[3 * a[q] + k]);
    for (int k = 0; k < 3; ++k) W[k] = Dual(P.wind[k]);
    for (int b = 0; b < 3; ++b)
      for (int m = 0; m < 3; ++m) {
        Dual Vd[3][3], F[3];
        for (int q = 0; q < 3; ++q)
          for (int k = 0; k < 3; ++k) Vd[q][k] = Dual(v[3 * a[q] + k], (q == b && k == m) ? 1.0 : 0.0);
        aero_force<Dual>(X[0], X[1], X[2], Vd[0], Vd[1], Vd[2], W, P.rho_air * P.area[t], F);
        // column (b, m): d f_q / d v_{b,m} = dF / 3 for every vertex q of the triangle
        for (int q = 0; q < 3; ++q) {
          int s = find_slot(P, a[q], a[b]);
          for (int k = 0; k < 3; ++k) D[9 * s + 3 * k + m] -= deriv_of(F[k]) / 3.0;
        }
      }
  }
}

// System matrix A = M + h D + h^2 K_sys (D the wind damping at (x, v), zero without
// wind) with Dirichlet rows/columns of pinned vertices.
void system_matrix(const Problem& P, const double* x, const double* v, const std::vector<double>& K,
                   std::vector<double>& A) {
  A.assign(K.size(), 0.0);
  std::vector<double> D;
  if (P.wind_on) wind_damping(P, x, v, D);
  double h2 = P.h * P.h;
  for (int i = 0; i < P.nv; ++i)
    for (int s = P.rowptr[i]; s < P.rowptr[i + 1]; ++s) {
      int j = P.col[s];
      double* blk = &A[9 * s];
      if (P.pinned[i] || P.pinned[j]) {
        if (i == j)
          for (int k = 0; k < 3; ++k) blk[4 * k] = 1.0;
        continue;
      }
      for (int q = 0; q < 9; ++q) blk[q] = h2 * K[9 * s + q] + (P.wind_on ? P.h * D[9 * s + q] : 0.0);
      if (i == j) {
        double m = P.dens * P.varea[i];
        for (int k = 0; k < 3; ++k) blk[4 * k] += m;
      }
    }
}

// Block-Jacobi preconditioned CG from zero; stops at ||r|| <= tol ||b||.
int pcg(const Problem& P, const std::vector<double>& A, const double* b, double* x, int* iters) {
  int n = 3 * P.nv;
  std::vector<double> Jinv(9 * P.nv), r(b, b + n), z(n), p(n), q(n);
  std::fill(x, x + n, 0.0);
  *iters = 0;
  for (int i = 0; i < P.nv; ++i) {
    int s = find_slot(P, i, i);
    if (!invert3(&A[9 * s], &Jinv[9 * i])) return ORC_E_INDEFINITE;
  }
  auto precond = [&](const std::vector<double>& in, std::vector<double>& out) {
    for (int i = 0; i < P.nv; ++i)
      for (int k = 0; k < 3; ++k)
        out[3 * i + k] = Jinv[9 * i + 3 * k] * in[3 * i] + Jinv[9 * i + 3 * k + 1] * in[3 * i + 1] +
                         Jinv[9 * i + 3 * k + 2] * in[3 * i + 2];
  };
  double bn = 0;
  for (int k = 0; k < n; ++k) bn += b[k] * b[k];
  bn = std::sqrt(bn);
  if (!std::isfinite(bn)) return ORC_E_NONFINITE;
  if (bn == 0.0) return ORC_OK;
  precond(r, z);
  p = z;
  double rz = 0;
  for (int k = 0; k < n; ++k) rz += r[k] * z[k];
  for (int it = 1; it <= P.cg_max_iter; ++it) {
    csr_apply(P, A, p.data(), q.data());
    double pq = 0;
    for (int k = 0; k < n; ++k) pq += p[k] * q[k];
    if (!std::isfinite(pq)) return ORC_E_NONFINITE;
    if (!(pq > 0)) {
      *iters = it;
      return ORC_E_INDEFINITE;
    }
    double alpha = rz / pq;
    double rr = 0;
    for (int k = 0; k < n; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * q[k];
      rr += r[k] * r[k];
    }
    *iters = it;
    if (std::sqrt(rr) <= P.cg_tol * bn) return ORC_OK;
    precond(r, z);
    double rz2 = 0;
    for (int k = 0; k < n; ++k) rz2 += r[k] * z[k];
    double beta = rz2 / rz;
    rz = rz2;
    for (int k = 0; k < n; ++k) p[k] = z[k] + beta * p[k];
  }
  return ORC_E_NOT_CONVERGED;
}

// Right-hand side of the linearised step (Eq. 4 with Eq. 5 substituted, df/dv = 0):
// b = h (f(x) + m g + F - h K_sys v) on free rows, 0 on pinned rows.
void step_rhs(const Problem& P, const double* x, const double* v, const double* F,
              const std::vector<double>& K, double* b) {
  int n = 3 * P.nv;
  std::vector<double> f(n), Kv(n);
  internal_force(P, x, problem_mat(P), f.data());
  if (P.wind_on) wind_force(P, x, v, f.data());
  csr_apply(P, K, v, Kv.data());
  for (int i = 0; i < P.nv; ++i) {
    double m = P.dens * P.varea[i];
    for (int k = 0; k < 3; ++k) {
      double ext = m * P.grav[k] + (F ? F[3 * i + k] : 0.0);
      b[3 * i + k] = P.pinned[i] ? 0.0 : P.h * (f[3 * i + k] + ext - P.h * Kv[3 * i + k]);
    }
  }
}

bool all_finite(const double* a, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) return false;
  return true;
}

// One step of Eq. 4-5: solve (M + h^2 K_sys) dv = b, v' = v + dv, x' = x + h v'.
// v must already be zero on pinned rows.
int one_step(const Problem& P, const double* x, const double* v, const double* F, double* xo,
             double* vo, double* dvo, int* iters) {
  int n = 3 * P.nv;
  std::vector<double> K, A, b(n), dv(n);
  assemble_ksys(P, x, K);
  system_matrix(P, x, v, K, A);
  step_rhs(P, x, v, F, K, b.data());
  if (!all_finite(b.data(), n) || !all_finite(A.data(), A.size())) return ORC_E_NONFINITE;
  int st = pcg(P, A, b.data(), dv.data(), iters);
  for (int i = 0; i < P.nv; ++i)
    for (int k = 0; k < 3; ++k) {
      double d = P.pinned[i] ? 0.0 : dv[3 * i + k];
      double vn = P.pinned[i] ? 0.0 : v[3 * i + k] + d;
      vo[3 * i + k] = vn;
      xo[3 * i + k] = x[3 * i + k] + P.h * vn;
      if (dvo) dvo[3 * i + k] = d;
    }
  if (st == ORC_OK && !all_finite(xo, n)) st = ORC_E_NONFINITE;
  return st;
}

int merge_status(int a, int b) {
  // keep the first hard error; NOT_CONVERGED is the mildest
  if (a != ORC_OK && a != ORC_E_NOT_CONVERGED) return a;
  if (b != ORC_OK) return b;
  return a;
}

bool valid_frames(const int* frames, int nloss, int nsteps) {
  int prev = 0;
  for (int k = 0; k < nloss; ++k) {
    if (frames[k] <= prev || frames[k] > nsteps) return false;
    prev = frames[k];
  }
  return true;
}

// Forward rollout storing every state (x_s, v_s, dv_s), s = 0..nsteps.
int rollout_store(const Problem& P, int nsteps, const double* x0, const double* v0,
                  const double* forces, std::vector<double>& X, std::vector<double>& Vv,
                  std::vector<double>& DV, int* iters) {
  int n = 3 * P.nv;
  X.assign((size_t)(nsteps + 1) * n, 0.0);
  Vv.assign((size_t)(nsteps + 1) * n, 0.0);
  DV.assign((size_t)(nsteps + 1) * n, 0.0);
  std::copy(x0, x0 + n, X.begin());
  for (int i = 0; i < P.nv; ++i)
    for (int k = 0; k < 3; ++k) Vv[3 * i + k] = P.pinned[i] ? 0.0 : v0[3 * i + k];
  int st = ORC_OK;
  for (int s = 1; s <= nsteps; ++s) {
    const double* F = forces ? forces + (size_t)(s - 1) * n : nullptr;
    int it = 0;
    int r = one_step(P, &X[(size_t)(s - 1) * n], &Vv[(size_t)(s - 1) * n], F, &X[(size_t)s * n],
                     &Vv[(size_t)s * n], &DV[(size_t)s * n], &it);
    if (iters) iters[s - 1] = it;
    st = merge_status(st, r);
    if (st != ORC_OK && st != ORC_E_NOT_CONVERGED) return st;
  }
  return st;
}


// Right-hand side of one adjoint solve (step 2 of the backward sweep):
// u = mask(gv + h gx), zero on pinned rows.
void adjoint_rhs(const Problem& P, const double* gx, const double* gv, double* u) {
  for (int i = 0; i < P.nv; ++i)
    for (int k = 0; k < 3; ++k)
      u[3 * i + k] = P.pinned[i] ? 0.0 : gv[3 * i + k] + P.h * gx[3 * i + k];
}

// The wind's part of one backward step (R19): with G = mu . f_wind(x, v, w) and A's
// wind block h D = -h df_wind/dv, the step's b and A contribute h dG/dc and
// -h d(mu^T D dv_s)/dc = h d^2 G(x, v + e dv_s, w)/dc de to the gradient with respect
// to every input c of every triangle (its positions, velocities and w), all at
// (x_{s-1}, v_{s-1}). Each triangle is evaluated in hyper-dual numbers: part a seeds c,
// part b seeds the velocities with dv_s. Adds to wx, wv [V][3] and ww[3].
void wind_adjoint(const Problem& P, const double* xp, const double* vp, const double* dvs,
                  const double* mu, double* wx, double* wv, double* ww) {
  for (int t = 0; t < P.nt; ++t) {
    const int* a = &P.tri[3 * t];
    for (int c = 0; c < 21; ++c) {   // 9 position, 9 velocity and 3 wind coordinates
      HDual X[3][3], V[3][3], Wd[3], F[3];
      for (int q = 0; q < 3; ++q)
        for (int k = 0; k < 3; ++k) {
          X[q][k] = HDual(xp[3 * a[q] + k], c == 3 * q + k ? 1.0 : 0.0, 0.0, 0.0);
          V[q][k] = HDual(vp[3 * a[q] + k], c == 9 + 3 * q + k ? 1.0 : 0.0, dvs[3 * a[q] + k], 0.0);
        }
      for (int k = 0; k < 3; ++k) Wd[k] = HDual(P.wind[k], c == 18 + k ? 1.0 : 0.0, 0.0, 0.0);
      aero_force<HDual>(X[0], X[1], X[2], V[0], V[1], V[2], Wd, P.rho_air * P.area[t], F);
      HDual G(0.0);
      for (int q = 0; q < 3; ++q)
        for (int k = 0; k < 3; ++k) G = G + HDual(mu[3 * a[q] + k] / 3.0) * F[k];
      const double d = P.h * (G.a + G.ab);
      if (c < 9) wx[3 * a[c / 3] + c % 3] += d;
      else if (c < 18) wv[3 * a[(c - 9) / 3] + (c - 9) % 3] += d;
      else ww[c - 18] += d;
    }
  }
}

// Steps 5-9 of one backward step of the implicit differentiation of Eq. 4, given
// the adjoint solution mu of A(x_{s-1}) mu = u, the state (x_{s-1}, v_{s-1}), the
// new velocity v_s and the increment dv_s: accumulates the material gradient in gmat
// ((dL/dk_s, dL/dk_b, dL/dd), or (dL/dS [24], dL/dB [15], dL/dd) with the anisotropic
// model) and the wind gradient dL/dw in gwind, and
// replaces (gx, gv) by the gradients with respect to (x_{s-1}, v_{s-1}).
void adjoint_update(const Problem& P, const double* xp, const double* vp, const double* vs,
                    const double* dvs, const double* mu, const double* u, double* gx, double* gv,
                    double* gmat, double* gwind) {
  const int n = 3 * P.nv;
  const double h1 = P.h, h2 = P.h * P.h;
  std::vector<double> tmp(n), tmp2(n), fh(n), wx(n, 0.0), wv(n, 0.0);
  if (P.wind_on) wind_adjoint(P, xp, vp, dvs, mu, wx.data(), wv.data(), gwind);
  // 5.-6. each stiffness parameter theta (the force and K_sys are linear in it):
  // dL/dtheta += mu . (h f_theta - h^2 K_sys,theta v_s), f_theta and K_sys,theta those of
  // the unit parameter
  const Mat M = problem_mat(P);
  const int nstiff = M.wang ? kWangStretch + kWangBend : 2;
  for (int q = 0; q < nstiff; ++q) {
    Mat U;
    U.wang = M.wang;
    if (!M.wang) (q == 0 ? U.ks : U.kb) = 1.0;
    else if (q < kWangStretch) U.S[q] = 1.0;
    else U.B[q - kWangStretch] = 1.0;
    internal_force(P, xp, U, fh.data());
    stiffness_apply(P, xp, vs, U, false, tmp.data());
    for (int k = 0; k < n; ++k) gmat[q] += mu[k] * (h1 * fh[k] - h2 * tmp[k]);
  }
  // 7. dL/dd += mu . (h A_vert g - A_vert dv_s)  (the last material entry)
  for (int i = 0; i < P.nv; ++i)
    for (int k = 0; k < 3; ++k)
      gmat[nstiff] += mu[3 * i + k] * P.varea[i] * (h1 * P.grav[k] - dvs[3 * i + k]);
  // 8. gx -= h K_exact mu + h^2 grad_x(mu^T K_sys v_s)
  stiffness_apply(P, xp, mu, M, true, tmp.data());
  third_contraction(P, xp, mu, vs, tmp2.data());
  for (int k = 0; k < n; ++k) gx[k] -= h1 * tmp[k] + h2 * tmp2[k];
  // 9. gv = mask(u - h^2 K_sys mu), plus the wind's velocity terms
  stiffness_apply(P, xp, mu, M, false, tmp.data());
  for (int i = 0; i < P.nv; ++i)
    for (int k = 0; k < 3; ++k)
      gv[3 * i + k] = P.pinned[i] ? 0.0 : u[3 * i + k] - h2 * tmp[3 * i + k] + wv[3 * i + k];
  if (P.wind_on)
    for (int k = 0; k < n; ++k) gx[k] += wx[k];
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

void* orc_create(int nv, int nt, const int* tris, const double* rest, const int* pins, int npins,
                 int* status) {
  Problem* P = new Problem();
  int st = build_problem(*P, nv, nt, tris, rest, pins, npins);
  if (status) *status = st;
  if (st != ORC_OK) {
    delete P;
    return nullptr;
  }
  return P;
}

void orc_destroy(void* h) { delete static_cast<Problem*>(h); }

int orc_set_params(void* h, double ks, double kb, double dens, double dt, double gx, double gy,
                   double gz, double cg_tol, int cg_max_iter) {
  Problem* P = static_cast<Problem*>(h);
  if (!P || !(dt > 0) || !(cg_tol > 0) || cg_max_iter < 1) return ORC_E_INVALID;
  if (!std::isfinite(ks) || !std::isfinite(kb) || !std::isfinite(dens)) return ORC_E_NONFINITE;
  P->ks = ks;
  P->kb = kb;
  P->dens = dens;
  P->h = dt;
  P->grav[0] = gx;
  P->grav[1] = gy;
  P->grav[2] = gz;
  P->cg_tol = cg_tol;
  P->cg_max_iter = cg_max_iter;
  return ORC_OK;
}

// Stress term of the system matrix's membrane block: 1 = exact Hessian (default),
// 2 = tension part, 0 = none (Gauss-Newton).
int orc_set_membrane_system(void* h, int geo) {
  if (geo < GEO_NONE || geo > GEO_TENSION) return ORC_E_INVALID;
  if (geo == GEO_TENSION && static_cast<Problem*>(h)->wang) return ORC_E_INVALID;
  static_cast<Problem*>(h)->mem_geo = geo;
  return ORC_OK;
}

int orc_num_hinges(void* h) { return static_cast<Problem*>(h)->nh; }
int orc_num_blocks(void* h) { return (int)static_cast<Problem*>(h)->col.size(); }

void orc_get_geometry(void* h, double* tri_B, double* tri_area, double* vert_area, int* hinge_v,
                      double* hinge_ce, double* hinge_rest) {
  Problem* P = static_cast<Problem*>(h);
  if (tri_B) std::copy(P->Bm.begin(), P->Bm.end(), tri_B);
  if (tri_area) std::copy(P->area.begin(), P->area.end(), tri_area);
  if (vert_area) std::copy(P->varea.begin(), P->varea.end(), vert_area);
  if (hinge_v) std::copy(P->hv.begin(), P->hv.end(), hinge_v);
  if (hinge_ce) std::copy(P->hce.begin(), P->hce.end(), hinge_ce);
  if (hinge_rest) std::copy(P->hrest.begin(), P->hrest.end(), hinge_rest);
}

double orc_energy(void* h, const double* x, double* em, double* eb) {
  return internal_energy(*static_cast<Problem*>(h), x, em, eb);
}

void orc_internal_force(void* h, const double* x, double* f) {
  Problem* P = static_cast<Problem*>(h);
  internal_force(*P, x, problem_mat(*P), f);
}

void orc_ksys_apply(void* h, const double* x, const double* u, double* out) {
  Problem* P = static_cast<Problem*>(h);
  stiffness_apply(*P, x, u, problem_mat(*P), false, out);
}

void orc_kexact_apply(void* h, const double* x, const double* u, double* out) {
  Problem* P = static_cast<Problem*>(h);
  stiffness_apply(*P, x, u, problem_mat(*P), true, out);
}

void orc_ksys_assembled_apply(void* h, const double* x, const double* u, double* out) {
  Problem* P = static_cast<Problem*>(h);
  std::vector<double> K;
  assemble_ksys(*P, x, K);
  csr_apply(*P, K, u, out);
}

void orc_third(void* h, const double* x, const double* mu, const double* w, double* out) {
  third_contraction(*static_cast<Problem*>(h), x, mu, w, out);
}

double orc_hinge_theta(const double* x4) {
  return hinge_theta<double>(x4, x4 + 3, x4 + 6, x4 + 9);
}

void orc_hinge_theta_grad(const double* x4, double* g12) {
  hinge_theta_grad<double>(x4, x4 + 3, x4 + 6, x4 + 9, g12, g12 + 3, g12 + 6, g12 + 9);
}

// Dense system (3V x 3V, row-major) and right-hand side of one step; small meshes only.
int orc_system(void* h, const double* x, const double* v, const double* F, double* A_dense,
               double* b) {
  Problem* P = static_cast<Problem*>(h);
  int n = 3 * P->nv;
  std::vector<double> vm(v, v + n);
  for (int i = 0; i < P->nv; ++i)
    if (P->pinned[i])
      for (int k = 0; k < 3; ++k) vm[3 * i + k] = 0.0;
  std::vector<double> K, A;
  assemble_ksys(*P, x, K);
  system_matrix(*P, x, vm.data(), K, A);
  step_rhs(*P, x, vm.data(), F, K, b);
  std::fill(A_dense, A_dense + (size_t)n * n, 0.0);
  for (int i = 0; i < P->nv; ++i)
    for (int s = P->rowptr[i]; s < P->rowptr[i + 1]; ++s) {
      int j = P->col[s];
      for (int k = 0; k < 3; ++k)
        for (int m = 0; m < 3; ++m) A_dense[(size_t)(3 * i + k) * n + 3 * j + m] = A[9 * s + 3 * k + m];
    }
  return ORC_OK;
}

// Linear solve of the step's system by the oracle's PCG (for the library-solve pin).
int orc_solve_step(void* h, const double* x, const double* v, const double* F, double* dv,
                   int* iters) {
  Problem* P = static_cast<Problem*>(h);
  int n = 3 * P->nv;
  std::vector<double> vm(v, v + n);
  for (int i = 0; i < P->nv; ++i)
    if (P->pinned[i])
      for (int k = 0; k < 3; ++k) vm[3 * i + k] = 0.0;
  std::vector<double> K, A, b(n);
  assemble_ksys(*P, x, K);
  system_matrix(*P, x, vm.data(), K, A);
  step_rhs(*P, x, vm.data(), F, K, b.data());
  return pcg(*P, A, b.data(), dv, iters);
}

// Residual r = b - A dv of one step's system (Eq. 4-5) for a given increment dv,
// and ||b||: how well dv solves the step, without forming a dense matrix.
int orc_step_residual(void* h, const double* x, const double* v, const double* F,
                      const double* dv, double* r, double* bnorm) {
  Problem* P = static_cast<Problem*>(h);
  int n = 3 * P->nv;
  std::vector<double> vm(v, v + n);
  for (int i = 0; i < P->nv; ++i)
    if (P->pinned[i])
      for (int k = 0; k < 3; ++k) vm[3 * i + k] = 0.0;
  std::vector<double> K, A, b(n), Adv(n);
  assemble_ksys(*P, x, K);
  system_matrix(*P, x, vm.data(), K, A);
  step_rhs(*P, x, vm.data(), F, K, b.data());
  csr_apply(*P, A, dv, Adv.data());
  double bn = 0.0;
  for (int k = 0; k < n; ++k) {
    r[k] = b[k] - Adv[k];
    bn += b[k] * b[k];
  }
  *bnorm = std::sqrt(bn);
  return all_finite(r, n) ? ORC_OK : ORC_E_NONFINITE;
}

// One full step from (x, v) with force slice F (may be NULL).
int orc_step(void* h, const double* x, const double* v, const double* F, double* xo, double* vo,
             double* dvo, int* iters) {
  Problem* P = static_cast<Problem*>(h);
  int n = 3 * P->nv;
  std::vector<double> vm(v, v + n);
  for (int i = 0; i < P->nv; ++i)
    if (P->pinned[i])
      for (int k = 0; k < 3; ++k) vm[3 * i + k] = 0.0;
  int it = 0;
  int st = one_step(*P, x, vm.data(), F, xo, vo, dvo, &it);
  if (iters) *iters = it;
  return st;
}

// Rollout (Eq. 1 applied nsteps times). forces: [nsteps][V][3] or NULL;
// x_out: [nloss][V][3] positions at the loss frames (1-based step indices).
int orc_rollout(void* h, int nsteps, const double* x0, const double* v0, const double* forces,
                const int* loss_frames, int nloss, double* x_out, double* v_final, int* iters) {
  Problem* P = static_cast<Problem*>(h);
  if (nsteps < 1 || !valid_frames(loss_frames, nloss, nsteps)) return ORC_E_INVALID;
  int n = 3 * P->nv;
  std::vector<double> X, Vv, DV;
  int st = rollout_store(*P, nsteps, x0, v0, forces, X, Vv, DV, iters);
  for (int k = 0; k < nloss; ++k)
    std::copy(&X[(size_t)loss_frames[k] * n], &X[(size_t)loss_frames[k] * n] + n,
              x_out + (size_t)k * n);
  if (v_final) std::copy(&Vv[(size_t)nsteps * n], &Vv[(size_t)nsteps * n] + n, v_final);
  P->last_status = st;
  return st;
}

// Rollout followed by the adjoint sweep (implicit differentiation of Eq. 4 with
// a per-frame loss whose gradient dl_dx [nloss][V][3] the caller supplies).
// Outputs: dl_dmat = (dL/dk_s, dL/dk_b, dL/dd), or [40] = (dL/dS, dL/dB, dL/dd) with the
// anisotropic model; dl_dF [nsteps][V][3];
// dl_dx0, dl_dv0 [V][3]. Any output pointer may be NULL.
int orc_gradient(void* h, int nsteps, const double* x0, const double* v0, const double* forces,
                 const int* loss_frames, int nloss, const double* dl_dx, double* dl_dmat,
                 double* dl_dwind, double* dl_dF, double* dl_dx0, double* dl_dv0, int* iters_fwd,
                 int* iters_adj) {
  Problem* P = static_cast<Problem*>(h);
  if (nsteps < 1 || !valid_frames(loss_frames, nloss, nsteps)) return ORC_E_INVALID;
  int n = 3 * P->nv;
  std::vector<double> X, Vv, DV;
  int st = rollout_store(*P, nsteps, x0, v0, forces, X, Vv, DV, iters_fwd);
  if (st != ORC_OK && st != ORC_E_NOT_CONVERGED) return st;

  std::vector<double> gx(n, 0.0), gv(n, 0.0), u(n), mu(n), K, A;
  double gmat[kWangParams] = {}, gwind[3] = {0.0, 0.0, 0.0};
  int frame = nloss - 1;
  for (int s = nsteps; s >= 1; --s) {
    const double* xp = &X[(size_t)(s - 1) * n];
    // 1. loss gradient of frame s
    if (frame >= 0 && loss_frames[frame] == s) {
      for (int k = 0; k < n; ++k) gx[k] += dl_dx[(size_t)frame * n + k];
      --frame;
    }
    // 2. u = mask(gv + h gx)
    adjoint_rhs(*P, gx.data(), gv.data(), u.data());
    // 3. A(x_{s-1}) mu = u  (A is symmetric)
    assemble_ksys(*P, xp, K);
    system_matrix(*P, xp, &Vv[(size_t)(s - 1) * n], K, A);
    int it = 0;
    int r = pcg(*P, A, u.data(), mu.data(), &it);
    if (iters_adj) iters_adj[s - 1] = it;
    st = merge_status(st, r);
    if (st != ORC_OK && st != ORC_E_NOT_CONVERGED) return st;
    // 4. dL/dF_{s-1} = h mu
    if (dl_dF)
      for (int k = 0; k < n; ++k) dl_dF[(size_t)(s - 1) * n + k] = P->h * mu[k];
    // 5.-9. material, state and velocity gradients through the step
    adjoint_update(*P, xp, &Vv[(size_t)(s - 1) * n], &Vv[(size_t)s * n], &DV[(size_t)s * n],
                   mu.data(), u.data(), gx.data(), gv.data(), gmat, gwind);
  }
  if (dl_dmat)
    for (int q = 0; q < (P->wang ? kWangParams : 3); ++q) dl_dmat[q] = gmat[q];
  if (dl_dwind)
    for (int k = 0; k < 3; ++k) dl_dwind[k] = gwind[k];
  if (dl_dx0) std::copy(gx.begin(), gx.end(), dl_dx0);
  if (dl_dv0) std::copy(gv.begin(), gv.end(), dl_dv0);
  P->last_status = st;
  return st;
}

// Block sparsity pattern of the step matrix (CSR over vertices): rowptr [V+1], col [nnzb].
void orc_pattern(void* h, int* rowptr, int* col) {
  Problem* P = static_cast<Problem*>(h);
  std::copy(P->rowptr.begin(), P->rowptr.end(), rowptr);
  std::copy(P->col.begin(), P->col.end(), col);
}

// The step's system (Eq. 4 with Eq. 5 substituted) in the block pattern of
// orc_pattern: A_blocks [nnzb][3][3] = M + h^2 K_sys with pinned rows and columns
// replaced by the identity, and b [V][3]. Lets a caller solve the step by any
// method (the exact sparse solve of the golden-file driver).
int orc_system_blocks(void* h, const double* x, const double* v, const double* F,
                      double* A_blocks, double* b) {
  Problem* P = static_cast<Problem*>(h);
  int n = 3 * P->nv;
  std::vector<double> vm(v, v + n);
  for (int i = 0; i < P->nv; ++i)
    if (P->pinned[i])
      for (int k = 0; k < 3; ++k) vm[3 * i + k] = 0.0;
  std::vector<double> K, A;
  assemble_ksys(*P, x, K);
  system_matrix(*P, x, vm.data(), K, A);
  step_rhs(*P, x, vm.data(), F, K, b);
  std::copy(A.begin(), A.end(), A_blocks);
  return all_finite(b, n) && all_finite(A.data(), A.size()) ? ORC_OK : ORC_E_NONFINITE;
}

// u = mask(gv + h gx): the right-hand side of one backward step's solve.
void orc_adjoint_rhs(void* h, const double* gx, const double* gv, double* u) {
  adjoint_rhs(*static_cast<Problem*>(h), gx, gv, u);
}

// The rest of one backward step once mu solves A(x_{s-1}, v_{s-1}) mu = u: accumulates
// (dL/dk_s, dL/dk_b, dL/dd) into gmat[3] (anisotropic model: gmat[40]) and dL/dw into
// gwind[3], and replaces (gx, gv)
// in place by the gradients with respect to (x_{s-1}, v_{s-1}). dL/dF_{s-1} is h mu.
void orc_adjoint_update(void* h, const double* xp, const double* vp, const double* vs,
                        const double* dvs, const double* mu, const double* u, double* gx,
                        double* gv, double* gmat, double* gwind) {
  adjoint_update(*static_cast<Problem*>(h), xp, vp, vs, dvs, mu, u, gx, gv, gmat, gwind);
}

// Wind (R19): on != 0 switches the aerodynamic force on with velocity (wx, wy, wz)
// [m/s] and air density rho [kg/m^3].
// Material model of the internal forces: 0 = isotropic (k_s, k_b of orc_set_params),
// 1 = anisotropic (R20, R21) with stretch table S [4][6] and bend table B [3][5];
// density stays that of orc_set_params. The anisotropic model takes the exact or the
// Gauss-Newton membrane block, not the tension variant.
int orc_set_material(void* h, int model, const double* S24, const double* B15) {
  Problem* P = static_cast<Problem*>(h);
  if (model != 0 && model != 1) return ORC_E_INVALID;
  if (model == 1) {
    if (!S24 || !B15 || P->mem_geo == GEO_TENSION) return ORC_E_INVALID;
    for (int q = 0; q < kWangStretch; ++q)
      if (!std::isfinite(S24[q])) return ORC_E_NONFINITE;
    for (int q = 0; q < kWangBend; ++q)
      if (!std::isfinite(B15[q])) return ORC_E_NONFINITE;
    std::copy(S24, S24 + kWangStretch, P->wS);
    std::copy(B15, B15 + kWangBend, P->wB);
  }
  P->wang = model == 1;
  return ORC_OK;
}

int orc_num_material(void* h) { return static_cast<Problem*>(h)->wang ? kWangParams : 3; }

// The anisotropic model's geometry: per triangle the measure tensors N_1..N_4 in its
// local frame (N_00, N_01, N_11 each) [nt][12], per hinge the direction weights [nh][3].
void orc_get_material_frames(void* h, double* N12, double* hdw) {
  Problem* P = static_cast<Problem*>(h);
  if (N12) std::copy(P->Nm.begin(), P->Nm.end(), N12);
  if (hdw) std::copy(P->hdw.begin(), P->hdw.end(), hdw);
}

int orc_set_wind(void* h, int on, double wx, double wy, double wz, double rho) {
  Problem* P = static_cast<Problem*>(h);
  if (!std::isfinite(wx) || !std::isfinite(wy) || !std::isfinite(wz) || !(rho >= 0.0))
    return ORC_E_INVALID;
  P->wind_on = on != 0;
  P->wind[0] = wx;
  P->wind[1] = wy;
  P->wind[2] = wz;
  P->rho_air = rho;
  return ORC_OK;
}

// The wind force alone at (x, v) [V][3] (zero when the wind is off).
void orc_wind_force(void* h, const double* x, const double* v, double* f) {
  Problem* P = static_cast<Problem*>(h);
  std::fill(f, f + 3 * P->nv, 0.0);
  if (P->wind_on) wind_force(*P, x, v, f);
}

}  // extern "C"

// mesh_prep.cpp -- host preparation of the device layout (runs once per handle).
//
// Rest geometry follows the deformation model of the paper (Sec. 3.1): lumped
// mass from density and surface area, stretching measured against the rest
// triangle, bending on the dihedral angle of every interior edge.

#include "mesh_prep.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <unordered_map>

namespace phisft {
namespace {

inline void vsub(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
inline double vdot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void vcross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Rest dihedral angle of hinge (x0, x1 | x2, x3), same convention as the kernels.
double rest_angle(const double* x0, const double* x1, const double* x2, const double* x3) {
  double e[3], a[3], me[3], d[3], n1[3], n2[3], c[3];
  vsub(x1, x0, e);
  vsub(x2, x0, a);
  vsub(x0, x1, me);
  vsub(x3, x1, d);
  vcross(e, a, n1);
  vcross(me, d, n2);
  vcross(n1, n2, c);
  double le = std::sqrt(vdot(e, e));
  return std::atan2(vdot(c, e) / le, vdot(n1, n2));
}

inline uint64_t edge_key(int i, int j) { return ((uint64_t)(uint32_t)i << 32) | (uint32_t)j; }

// Recursive coordinate bisection: orders ids[lo, hi) so that every run of `leaf`
// consecutive vertices counted from lo is a compact patch of the rest shape. Each
// split is along the longest side of the bounding box, at a multiple of `leaf`.
void rcb(const std::vector<double>& rest, std::vector<int>& ids, int lo, int hi, int leaf,
         int inner) {
  const int n = hi - lo;
  if (n <= leaf) {
    // a leaf is ordered again into runs of `inner` vertices (the middle level)
    if (inner > 0 && inner < leaf && n > inner) rcb(rest, ids, lo, hi, inner, 0);
    else std::sort(ids.begin() + lo, ids.begin() + hi);
    return;
  }
  const int k = (n + leaf - 1) / leaf;
  const int mid = lo + (k / 2) * leaf;
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int q = lo; q < hi; ++q)
    for (int c = 0; c < 3; ++c) {
      mn[c] = std::min(mn[c], rest[3 * (size_t)ids[q] + c]);
      mx[c] = std::max(mx[c], rest[3 * (size_t)ids[q] + c]);
    }
  int ax = 0;
  for (int c = 1; c < 3; ++c)
    if (mx[c] - mn[c] > mx[ax] - mn[ax]) ax = c;
  std::nth_element(ids.begin() + lo, ids.begin() + mid, ids.begin() + hi, [&](int a, int b) {
    const double xa = rest[3 * (size_t)a + ax], xb = rest[3 * (size_t)b + ax];
    return xa < xb || (xa == xb && a < b);
  });
  rcb(rest, ids, lo, mid, leaf, inner);
  rcb(rest, ids, mid, hi, leaf, inner);
}

// Warp axis of a rest plane with unit normal n: the x axis projected into the plane
// (the y axis where x is within about 0.06 degrees of the normal), unit length.
void warp_axis(const double n[3], double u[3]) {
  const double ax[3] = {1.0, 0.0, 0.0}, ay[3] = {0.0, 1.0, 0.0};
  const double* a = ax;
  double d = vdot(a, n);
  for (int k = 0; k < 3; ++k) u[k] = a[k] - d * n[k];
  double l = std::sqrt(vdot(u, u));
  if (!(l > 1e-3)) {
    a = ay;
    d = vdot(a, n);
    for (int k = 0; k < 3; ++k) u[k] = a[k] - d * n[k];
    l = std::sqrt(vdot(u, u));
  }
  for (int k = 0; k < 3; ++k) u[k] /= l;
}

// Coarse modes an aggregate supports: rigid motions (6) when its free vertices are
// at least three and not collinear, translations (3) with one or two free vertices
// (or collinear ones), none when every vertex is pinned.
int aggregate_modes(const std::vector<double>& rest, const std::vector<int>& pinned, int voff,
                    int v0, int v1) {
  std::vector<int> fr;  // sheet-local ids (rest is the sheet's, pinned is global)
  for (int i = v0; i < v1; ++i)
    if (!pinned[voff + i]) fr.push_back(i);
  if (fr.empty()) return 0;
  if (fr.size() < 3) return 3;
  const double* p0 = &rest[3 * (size_t)fr[0]];
  double far2 = 0.0, d[3];
  int f = fr[0];
  for (int i : fr) {
    vsub(&rest[3 * (size_t)i], p0, d);
    if (vdot(d, d) > far2) {
      far2 = vdot(d, d);
      f = i;
    }
  }
  if (!(far2 > 0.0)) return 3;
  double e[3], c[3], best = 0.0;
  vsub(&rest[3 * (size_t)f], p0, e);
  for (int i : fr) {
    vsub(&rest[3 * (size_t)i], p0, d);
    vcross(d, e, c);
    best = std::max(best, std::sqrt(vdot(c, c)) / far2);
  }
  return best > 1e-6 ? 6 : 3;
}

}  // namespace

int build_layout(const std::vector<HostSheet>& sheets_in, int agg_size, int max_aggs,
                 HostLayout& L, std::string& err) {
  L = HostLayout();
  L.ninst = (int)sheets_in.size();
  if (L.ninst < 1) {
    err = "no sheets";
    return -1;
  }
  if (agg_size < 0 || max_aggs < 1) {
    err = "invalid coarse-space size";
    return -1;
  }
  // ---- renumber every sheet's vertices (compact runs); indices are checked first
  std::vector<HostSheet> sheets(sheets_in.size());
  std::vector<std::vector<int>> order(sheets_in.size());
  std::vector<int> leaf(sheets_in.size());
  for (size_t b = 0; b < sheets_in.size(); ++b) {
    const HostSheet& s = sheets_in[b];
    if (s.nv < 3 || s.nt < 1 || (int)s.tris.size() != 3 * s.nt || (int)s.rest.size() != 3 * s.nv) {
      err = "sheet sizes do not match its arrays";
      return -1;
    }
    for (int v : s.tris)
      if (v < 0 || v >= s.nv) {
        err = "triangle vertex id out of range";
        return -2;
      }
    for (int p : s.pins)
      if (p < 0 || p >= s.nv) {
        err = "pin index out of range";
        return -1;
      }
    const int base = agg_size > 0 ? agg_size : 64;
    leaf[b] = std::max(base, (s.nv + max_aggs - 1) / max_aggs);
    // coarse aggregates are whole runs of the middle level
    if (agg_size > 0) leaf[b] = (leaf[b] + kMidSize - 1) / kMidSize * kMidSize;
    std::vector<int>& ids = order[b];
    ids.resize(s.nv);
    for (int i = 0; i < s.nv; ++i) ids[i] = i;
    rcb(s.rest, ids, 0, s.nv, leaf[b], agg_size > 0 ? kMidSize : 0);
    std::vector<int> inv(s.nv);
    for (int q = 0; q < s.nv; ++q) inv[ids[q]] = q;
    HostSheet& t = sheets[b];
    t.nv = s.nv;
    t.nt = s.nt;
    t.rest.resize(s.rest.size());
    for (int q = 0; q < s.nv; ++q)
      for (int c = 0; c < 3; ++c) t.rest[3 * (size_t)q + c] = s.rest[3 * (size_t)ids[q] + c];
    t.tris.resize(s.tris.size());
    for (size_t k = 0; k < s.tris.size(); ++k) t.tris[k] = inv[s.tris[k]];
    for (int p : s.pins) t.pins.push_back(inv[p]);
    for (int k = 0; k < 3; ++k) t.mat[k] = s.mat[k];
  }
  // ---- sizes and offsets
  for (const HostSheet& s : sheets) {
    if (s.nv < 3 || s.nt < 1 || (int)s.tris.size() != 3 * s.nt || (int)s.rest.size() != 3 * s.nv) {
      err = "sheet sizes do not match its arrays";
      return -1;
    }
    L.inst_voff.push_back(L.nv);
    L.inst_nv.push_back(s.nv);
    L.inst_toff.push_back(L.nt);
    L.inst_nt.push_back(s.nt);
    if ((long)L.nv + s.nv > (1 << 26) || (long)L.nt + s.nt > (1 << 26)) {
      err = "mesh too large";
      return -1;
    }
    L.nv += s.nv;
    L.nt += s.nt;
  }
  L.varea.assign(L.nv, 0.0);
  L.pinned.assign(L.nv, 0);
  L.vert_inst.assign(L.nv, 0);
  L.tri_v.assign(3 * (size_t)L.nt, 0);
  L.tri_B.assign(4 * (size_t)L.nt, 0.0);
  L.tri_N.assign(12 * (size_t)L.nt, 0.0);
  L.tri_area.assign(L.nt, 0.0);
  L.tri_inst.assign(L.nt, 0);
  std::vector<int> hv;   // [nh][4] global
  std::vector<double> hce, hrest, hdw;
  std::vector<int> hinst;

  for (int b = 0; b < L.ninst; ++b) {
    const HostSheet& s = sheets[b];
    const int voff = L.inst_voff[b], toff = L.inst_toff[b];
    for (int i = 0; i < s.nv; ++i) {
      L.vert_inst[voff + i] = b;
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(s.rest[3 * i + k])) {
          err = "non-finite rest position";
          return -2;
        }
    }
    for (int p : s.pins) {
      if (p < 0 || p >= s.nv) {
        err = "pin index out of range";
        return -1;
      }
      L.pinned[voff + p] = 1;
    }
    for (int k = 0; k < 3; ++k) L.mat.push_back(s.mat[k]);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < s.nv; ++i)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], s.rest[3 * i + k]);
        hi[k] = std::max(hi[k], s.rest[3 * i + k]);
      }
    double diag2 = 0.0;
    for (int k = 0; k < 3; ++k) diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
    // ---- triangles: rest frame (e1 along the first edge, e2 in-plane), B = D_m^-1
    std::unordered_map<uint64_t, int> dir;  // directed edge -> local triangle * 3 + corner
    dir.reserve(3 * (size_t)s.nt);
    for (int t = 0; t < s.nt; ++t) {
      const int* v = &s.tris[3 * t];
      for (int a = 0; a < 3; ++a)
        if (v[a] < 0 || v[a] >= s.nv) {
          err = "triangle vertex id out of range";
          return -2;
        }
      if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) {
        err = "triangle repeats a vertex";
        return -2;
      }
      const double* X0 = &s.rest[3 * v[0]];
      const double* X1 = &s.rest[3 * v[1]];
      const double* X2 = &s.rest[3 * v[2]];
      double d1[3], d2[3], n[3], e1[3], e2[3];
      vsub(X1, X0, d1);
      vsub(X2, X0, d2);
      vcross(d1, d2, n);
      double ln = std::sqrt(vdot(n, n)), l1 = std::sqrt(vdot(d1, d1));
      if (!(0.5 * ln > 1e-14 * diag2) || !(l1 > 0.0)) {
        err = "degenerate rest triangle";
        return -2;
      }
      for (int k = 0; k < 3; ++k) {
        e1[k] = d1[k] / l1;
        n[k] /= ln;
      }
      vcross(n, e1, e2);
      double m00 = vdot(d1, e1), m01 = vdot(d2, e1), m10 = vdot(d1, e2), m11 = vdot(d2, e2);
      double det = m00 * m11 - m01 * m10;
      if (!(0.5 * det > 1e-14 * diag2)) {
        err = "degenerate rest triangle";
        return -2;
      }
      const int gt = toff + t;
      L.tri_B[0 * (size_t)L.nt + gt] = m11 / det;
      L.tri_B[1 * (size_t)L.nt + gt] = -m01 / det;
      L.tri_B[2 * (size_t)L.nt + gt] = -m10 / det;
      L.tri_B[3 * (size_t)L.nt + gt] = m00 / det;
      L.tri_area[gt] = 0.5 * det;
      L.tri_inst[gt] = b;
      {
        // strain measures of the anisotropic model in the local frame (e1, e2): warp
        // u u^T, weft v v^T, shear (u v^T + v u^T) / sqrt 2, area I, with u the warp axis
        // and v = n x u
        double u3[3];
        warp_axis(n, u3);
        const double a0 = vdot(u3, e1), a1 = vdot(u3, e2), b0 = -a1, b1 = a0;
        const double r2 = std::sqrt(2.0);
        const double Nq[12] = {a0 * a0, a0 * a1, a1 * a1, b0 * b0, b0 * b1, b1 * b1,
                               r2 * a0 * b0, (a0 * b1 + a1 * b0) / r2, r2 * a1 * b1,
                               1.0, 0.0, 1.0};
        for (int q = 0; q < 12; ++q) L.tri_N[q * (size_t)L.nt + gt] = Nq[q];
      }
      for (int a = 0; a < 3; ++a) {
        L.tri_v[a * (size_t)L.nt + gt] = voff + v[a];
        L.varea[voff + v[a]] += L.tri_area[gt] / 3.0;
        uint64_t key = edge_key(v[a], v[(a + 1) % 3]);
        if (dir.count(key)) {
          err = "edge used twice in the same direction (orientation or manifoldness)";
          return -2;
        }
        dir[key] = 3 * t + a;
      }
    }
    // ---- hinges: every directed edge i->j (i < j) whose reverse exists
    L.inst_hoff.push_back((int)hce.size());
    for (int t = 0; t < s.nt; ++t) {
      const int* v = &s.tris[3 * t];
      for (int a = 0; a < 3; ++a) {
        int i = v[a], j = v[(a + 1) % 3], o = v[(a + 2) % 3];
        if (i > j) continue;
        auto it = dir.find(edge_key(j, i));
        if (it == dir.end()) continue;
        int t2 = it->second / 3, c2 = it->second % 3;
        int o2 = s.tris[3 * t2 + (c2 + 2) % 3];
        hv.push_back(voff + i);
        hv.push_back(voff + j);
        hv.push_back(voff + o);
        hv.push_back(voff + o2);
        double e[3];
        vsub(&s.rest[3 * j], &s.rest[3 * i], e);
        double A1 = L.tri_area[toff + t], A2 = L.tri_area[toff + t2];
        hce.push_back(3.0 * vdot(e, e) / (A1 + A2));
        hrest.push_back(rest_angle(&s.rest[3 * i], &s.rest[3 * j], &s.rest[3 * o], &s.rest[3 * o2]));
        hinst.push_back(b);
        {
          // bending direction: in the plane of the triangle (i, j, o), normal to the
          // edge; its angle to that plane's warp axis, folded into [0, 90] degrees,
          // weights the 0, 45 and 90 degree tables linearly
          double d2[3], n1[3], ue[3], bd[3], u3[3];
          vsub(&s.rest[3 * o], &s.rest[3 * i], d2);
          vcross(e, d2, n1);
          const double ln1 = std::sqrt(vdot(n1, n1)), le = std::sqrt(vdot(e, e));
          for (int k = 0; k < 3; ++k) {
            n1[k] /= ln1;
            ue[k] = e[k] / le;
          }
          vcross(n1, ue, bd);
          warp_axis(n1, u3);
          const double q = std::acos(std::min(1.0, std::fabs(vdot(bd, u3)))) / std::atan(1.0);
          hdw.push_back(q <= 1.0 ? 1.0 - q : 0.0);
          hdw.push_back(q <= 1.0 ? q : 2.0 - q);
          hdw.push_back(q <= 1.0 ? 0.0 : q - 1.0);
        }
      }
    }
    L.inst_nh.push_back((int)hce.size() - L.inst_hoff.back());
  }
  L.nh = (int)hce.size();
  if ((long)L.nh * 16 > (1L << 30) || (long)L.nt * 9 > (1L << 30)) {
    err = "mesh too large";
    return -1;
  }
  L.hin_v.assign(4 * (size_t)L.nh, 0);
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 4; ++a) L.hin_v[a * (size_t)L.nh + e] = hv[4 * (size_t)e + a];
  L.hin_ce = hce;
  L.hin_rest = hrest;
  L.hin_inst = hinst;
  L.hin_dw.assign(3 * (size_t)L.nh, 0.0);
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 3; ++a) L.hin_dw[a * (size_t)L.nh + e] = hdw[3 * (size_t)e + a];

  // ---- block rows: neighbours through a triangle or a hinge, sorted, with self
  std::vector<std::vector<int>> nb(L.nv);
  for (int t = 0; t < L.nt; ++t)
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) nb[L.tri_v[a * (size_t)L.nt + t]].push_back(L.tri_v[c * (size_t)L.nt + t]);
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) nb[hv[4 * (size_t)e + a]].push_back(hv[4 * (size_t)e + c]);
  L.maxnz = 0;
  for (int i = 0; i < L.nv; ++i) {
    auto& r = nb[i];
    r.push_back(i);
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    L.maxnz = std::max(L.maxnz, (int)r.size());
  }
  const int nv = L.nv, mz = L.maxnz;
  L.ell_col.assign((size_t)mz * nv, -1);
  L.diag_k.assign(nv, -1);
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < (int)nb[i].size(); ++k) {
      L.ell_col[(size_t)k * nv + i] = nb[i][k];
      if (nb[i][k] == i) L.diag_k[i] = k;
    }
  auto slot_of = [&](int i, int j) {
    const auto& r = nb[i];
    int k = (int)(std::lower_bound(r.begin(), r.end(), j) - r.begin());
    return k * nv + i;
  };
  // ---- slot contributions (counting sort; triangles then hinges, element order)
  const size_t nslot = (size_t)mz * nv;
  std::vector<int> cnt(nslot + 1, 0);
  for (int t = 0; t < L.nt; ++t)
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) cnt[slot_of(L.tri_v[a * (size_t)L.nt + t], L.tri_v[c * (size_t)L.nt + t]) + 1]++;
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) cnt[slot_of(hv[4 * (size_t)e + a], hv[4 * (size_t)e + c]) + 1]++;
  L.slot_ptr.assign(nslot + 1, 0);
  for (size_t s = 0; s < nslot; ++s) L.slot_ptr[s + 1] = L.slot_ptr[s] + cnt[s + 1];
  L.slot_ref.assign(L.slot_ptr[nslot], 0);
  std::vector<int> fill(L.slot_ptr.begin(), L.slot_ptr.end() - 1);
  for (int t = 0; t < L.nt; ++t)
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        int s = slot_of(L.tri_v[a * (size_t)L.nt + t], L.tri_v[c * (size_t)L.nt + t]);
        L.slot_ref[fill[s]++] = t * 9 + a * 3 + c;
      }
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        int s = slot_of(hv[4 * (size_t)e + a], hv[4 * (size_t)e + c]);
        L.slot_ref[fill[s]++] = -(e * 16 + a * 4 + c) - 1;
      }
  // ---- vertex incidence
  std::vector<int> vc(nv + 1, 0);
  for (int t = 0; t < L.nt; ++t)
    for (int a = 0; a < 3; ++a) vc[L.tri_v[a * (size_t)L.nt + t] + 1]++;
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 4; ++a) vc[hv[4 * (size_t)e + a] + 1]++;
  L.vinc_ptr.assign(nv + 1, 0);
  for (int i = 0; i < nv; ++i) L.vinc_ptr[i + 1] = L.vinc_ptr[i] + vc[i + 1];
  L.vinc_ref.assign(L.vinc_ptr[nv], 0);
  std::vector<int> vf(L.vinc_ptr.begin(), L.vinc_ptr.end() - 1);
  for (int t = 0; t < L.nt; ++t)
    for (int a = 0; a < 3; ++a) L.vinc_ref[vf[L.tri_v[a * (size_t)L.nt + t]]++] = t * 3 + a;
  for (int e = 0; e < L.nh; ++e)
    for (int a = 0; a < 4; ++a) L.vinc_ref[vf[hv[4 * (size_t)e + a]]++] = -(e * 4 + a) - 1;

  // ---- internal -> caller vertex order
  L.vold.assign(nv, 0);
  for (int b = 0; b < L.ninst; ++b)
    for (int q = 0; q < L.inst_nv[b]; ++q) L.vold[L.inst_voff[b] + q] = L.inst_voff[b] + order[b][q];

  // ---- aggregates and the coarse pattern
  L.vert_agg.assign(nv, -1);
  L.agg_v0.clear();
  for (int b = 0; b < L.ninst; ++b) {
    L.inst_agg0.push_back(L.nagg);
    if (agg_size == 0) {
      L.inst_nagg.push_back(0);
      L.inst_nc.push_back(0);
      L.inst_np.push_back(0);
      L.inst_coff.push_back(L.coarse_doubles);
      continue;
    }
    const int n = L.inst_nv[b], voff = L.inst_voff[b];
    const int k = (n + leaf[b] - 1) / leaf[b];
    for (int a = 0; a < k; ++a) {
      const int v0 = voff + a * leaf[b], v1 = std::min(voff + n, v0 + leaf[b]);
      L.agg_v0.push_back(v0);
      L.agg_inst.push_back(b);
      L.agg_modes.push_back(aggregate_modes(sheets[b].rest, L.pinned, voff, v0 - voff, v1 - voff));
      for (int i = v0; i < v1; ++i) L.vert_agg[i] = L.nagg;
      ++L.nagg;
    }
    L.inst_nagg.push_back(k);
    const int np = (6 * k + 31) / 32 * 32;  // stored with an identity block up to 32 | np
    L.inst_nc.push_back(6 * k);
    L.inst_np.push_back(np);
    L.inst_coff.push_back(L.coarse_doubles);
    L.coarse_doubles += (long long)np * np;
    L.max_nc = std::max(L.max_nc, 6 * k);
  }
  L.agg_v0.push_back(nv);
  if (agg_size > 0) {
    std::vector<std::vector<int>> bucket;   // per pair
    std::unordered_map<uint64_t, int> pid;
    for (int i = 0; i < nv; ++i) {
      if (L.pinned[i]) continue;
      for (int k = 0; k < mz; ++k) {
        const int j = L.ell_col[(size_t)k * nv + i];
        if (j < 0 || L.pinned[j]) continue;
        const int a = L.vert_agg[i], c = L.vert_agg[j];
        if (a > c) continue;
        const uint64_t key = edge_key(a, c);
        auto it = pid.find(key);
        int q;
        if (it == pid.end()) {
          q = (int)bucket.size();
          pid[key] = q;
          bucket.emplace_back();
        } else {
          q = it->second;
        }
        bucket[q].push_back(k * nv + i);
      }
    }
    std::vector<std::pair<uint64_t, int>> keys(pid.begin(), pid.end());
    std::sort(keys.begin(), keys.end());
    L.pair_ptr.assign(1, 0);
    for (auto& kv : keys) {
      L.pair_a.push_back((int)(kv.first >> 32));
      L.pair_b.push_back((int)(kv.first & 0xffffffffu));
      auto& v = bucket[kv.second];
      std::sort(v.begin(), v.end(), [&](int x, int y) {
        const int ix = x % nv, iy = y % nv;
        return ix < iy || (ix == iy && x < y);
      });
      L.pair_slot.insert(L.pair_slot.end(), v.begin(), v.end());
      L.pair_ptr.push_back((int)L.pair_slot.size());
    }
  } else {
    L.pair_ptr.assign(1, 0);
  }
  // ---- middle level: runs of kMidSize vertices from every sheet's start
  L.mid_ptr.assign(1, 0);
  L.vert_mid.assign(agg_size > 0 ? nv : 0, 0);
  if (agg_size > 0) {
    for (int b = 0; b < L.ninst; ++b) {
      const int n = L.inst_nv[b], voff = L.inst_voff[b];
      L.inst_mid0.push_back(L.nmid);
      for (int v0 = 0; v0 < n; v0 += kMidSize) {
        const int v1 = std::min(n, v0 + kMidSize);
        L.mid_v0.push_back(voff + v0);
        L.mid_modes.push_back(aggregate_modes(sheets[b].rest, L.pinned, voff, v0, v1));
        for (int i = voff + v0; i < voff + v1; ++i) L.vert_mid[i] = L.nmid;
        for (int i = voff + v0; i < voff + v1; ++i) {
          if (L.pinned[i]) continue;
          for (int k = 0; k < mz; ++k) {
            const int j = L.ell_col[(size_t)k * nv + i];
            if (j >= voff + v0 && j < voff + v1 && !L.pinned[j]) L.mid_slot.push_back(k * nv + i);
          }
        }
        L.mid_ptr.push_back((int)L.mid_slot.size());
        ++L.nmid;
      }
    }
    L.mid_v0.push_back(nv);
  }
  return 0;
}

bool check_layout(const HostLayout& L, std::string& err) {
  auto bad = [&](const char* what) {
    err = std::string("layout check failed: ") + what;
    return false;
  };
  const int nv = L.nv, nt = L.nt, nh = L.nh;
  if ((int)L.varea.size() != nv || (int)L.pinned.size() != nv || (int)L.diag_k.size() != nv)
    return bad("vertex array sizes");
  for (int i = 0; i < nv; ++i) {
    if (L.diag_k[i] < 0 || L.diag_k[i] >= L.maxnz) return bad("diagonal slot");
    if (L.ell_col[(size_t)L.diag_k[i] * nv + i] != i) return bad("diagonal column");
    if (!(L.varea[i] > 0.0)) return bad("vertex without area");
    if (L.vert_inst[i] < 0 || L.vert_inst[i] >= L.ninst) return bad("vertex instance");
  }
  for (size_t s = 0; s < L.ell_col.size(); ++s) {
    int j = L.ell_col[s];
    if (j < -1 || j >= nv) return bad("ell column");
    int i = (int)(s % nv);
    if (j >= 0 && L.vert_inst[j] != L.vert_inst[i]) return bad("column crosses instances");
    if (j < 0 && L.slot_ptr[s + 1] != L.slot_ptr[s]) return bad("padding slot with contributions");
  }
  if (L.slot_ptr.size() != L.ell_col.size() + 1) return bad("slot_ptr size");
  for (size_t c = 0; c < L.slot_ref.size(); ++c) {
    int r = L.slot_ref[c];
    if (r >= 0 ? (r / 9 >= nt) : ((-r - 1) / 16 >= nh)) return bad("slot reference");
  }
  // every element block appears exactly once
  if ((long)L.slot_ref.size() != 9L * nt + 16L * nh) return bad("slot reference count");
  if ((int)L.vinc_ptr.size() != nv + 1 || (long)L.vinc_ref.size() != 3L * nt + 4L * nh)
    return bad("incidence size");
  for (int r : L.vinc_ref)
    if (r >= 0 ? (r / 3 >= nt) : ((-r - 1) / 4 >= nh)) return bad("incidence reference");
  for (int v : L.tri_v)
    if (v < 0 || v >= nv) return bad("triangle vertex");
  for (int v : L.hin_v)
    if (v < 0 || v >= nv) return bad("hinge vertex");
  for (int t = 0; t < nt; ++t)
    if (L.tri_inst[t] < 0 || L.tri_inst[t] >= L.ninst) return bad("triangle instance");
  for (int e = 0; e < nh; ++e)
    if (L.hin_inst[e] < 0 || L.hin_inst[e] >= L.ninst) return bad("hinge instance");
  // vertex order is a permutation within each sheet
  if ((int)L.vold.size() != nv) return bad("vertex order size");
  std::vector<char> seen(nv, 0);
  for (int i = 0; i < nv; ++i) {
    const int o = L.vold[i];
    if (o < 0 || o >= nv || seen[o] || L.vert_inst[o] != L.vert_inst[i]) return bad("vertex order");
    seen[o] = 1;
  }
  // aggregates: consecutive runs covering their sheets
  if ((int)L.agg_v0.size() != L.nagg + 1 || (int)L.agg_modes.size() != L.nagg) return bad("aggregates");
  for (int a = 0; a < L.nagg; ++a) {
    if (L.agg_v0[a] < 0 || L.agg_v0[a + 1] <= L.agg_v0[a] || L.agg_v0[a + 1] > nv) return bad("aggregate range");
    for (int i = L.agg_v0[a]; i < L.agg_v0[a + 1]; ++i)
      if (L.vert_agg[i] != a || L.vert_inst[i] != L.agg_inst[a]) return bad("aggregate member");
  }
  for (int b = 0; b < L.ninst; ++b) {
    if (L.inst_nagg[b] > 0 && (L.agg_v0[L.inst_agg0[b]] != L.inst_voff[b] ||
                               L.agg_v0[L.inst_agg0[b] + L.inst_nagg[b]] != L.inst_voff[b] + L.inst_nv[b]))
      return bad("aggregates of a sheet");
    if (L.inst_nc[b] != 6 * L.inst_nagg[b] || L.inst_np[b] < L.inst_nc[b] || L.inst_np[b] % 32 != 0)
      return bad("coarse size");
  }
  if (L.pair_ptr.size() != L.pair_a.size() + 1 || L.pair_ptr.back() != (int)L.pair_slot.size())
    return bad("coarse pairs");
  for (size_t q = 0; q < L.pair_a.size(); ++q) {
    const int a = L.pair_a[q], c = L.pair_b[q];
    if (a < 0 || c < a || c >= L.nagg || L.agg_inst[a] != L.agg_inst[c]) return bad("coarse pair");
    for (int t = L.pair_ptr[q]; t < L.pair_ptr[q + 1]; ++t) {
      const int sl = L.pair_slot[t];
      if (sl < 0 || sl >= L.maxnz * nv) return bad("coarse pair slot");
      const int i = sl % nv, j = L.ell_col[sl];
      if (j < 0 || L.vert_agg[i] != a || L.vert_agg[j] != c) return bad("coarse pair slot");
    }
  }
  if (L.nmid > 0) {
    if ((int)L.mid_v0.size() != L.nmid + 1 || (int)L.mid_modes.size() != L.nmid ||
        (int)L.mid_ptr.size() != L.nmid + 1 || L.mid_ptr.back() != (int)L.mid_slot.size())
      return bad("middle level sizes");
    for (int a = 0; a < L.nmid; ++a) {
      const int v0 = L.mid_v0[a], v1 = L.mid_v0[a + 1];
      if (v1 - v0 < 1 || v1 - v0 > kMidSize || v1 > nv || L.vert_inst[v0] != L.vert_inst[v1 - 1])
        return bad("middle aggregate");
      for (int t = L.mid_ptr[a]; t < L.mid_ptr[a + 1]; ++t) {
        const int sl = L.mid_slot[t];
        if (sl < 0 || sl >= L.maxnz * nv) return bad("middle slot");
        const int i = sl % nv, j = L.ell_col[sl];
        if (i < v0 || i >= v1 || j < v0 || j >= v1) return bad("middle slot");
      }
    }
  }
  return true;
}

HostPlan make_plan(const HostLayout& L, int rows, int group) {
  HostPlan P;
  P.rows = rows;
  int slot = L.ninst;  // root counters first
  for (int b = 0; b < L.ninst; ++b) {
    int n = L.inst_nv[b];
    int k = (n + rows - 1) / rows;
    P.inst_wg0.push_back(P.nwg);
    P.inst_nwg.push_back(k);
    P.inst_grp0.push_back(slot);
    if (k > group) slot += 2 * ((k + group - 1) / group);
    for (int w = 0; w < k; ++w) {
      P.wg_inst.push_back(b);
      P.wg_row0.push_back(L.inst_voff[b] + w * rows);
      P.wg_nrows.push_back(std::min(rows, n - w * rows));
    }
    P.nwg += k;
  }
  P.barrier_slots = slot;
  // halo of every workgroup and the local column table
  {
    const int nv = L.nv, mz = L.maxnz;
    P.lcol.assign((size_t)mz * nv, 0);
    P.halo_ptr.assign(1, 0);
    std::vector<int> h;
    for (int w = 0; w < P.nwg; ++w) {
      const int r0 = P.wg_row0[w], n = P.wg_nrows[w];
      h.clear();
      for (int i = r0; i < r0 + n; ++i)
        for (int k = 0; k < mz; ++k) {
          const int j = L.ell_col[(size_t)k * nv + i];
          if (j >= 0 && (j < r0 || j >= r0 + n)) h.push_back(j);
        }
      std::sort(h.begin(), h.end());
      h.erase(std::unique(h.begin(), h.end()), h.end());
      for (int i = r0; i < r0 + n; ++i)
        for (int k = 0; k < mz; ++k) {
          const int j = L.ell_col[(size_t)k * nv + i];
          int loc;
          if (j < 0) loc = i - r0;
          else if (j >= r0 && j < r0 + n) loc = j - r0;
          else loc = rows + (int)(std::lower_bound(h.begin(), h.end(), j) - h.begin());
          P.lcol[(size_t)k * nv + i] = loc;
        }
      P.halo_idx.insert(P.halo_idx.end(), h.begin(), h.end());
      P.halo_ptr.push_back((int)P.halo_idx.size());
      P.max_halo = std::max(P.max_halo, (int)h.size());
    }
  }

  // workgroup / aggregate overlaps (both are runs of consecutive vertices)
  if (L.nagg > 0) {
    P.wg_agg0.resize(P.nwg);
    P.wg_nagg.resize(P.nwg);
    for (int w = 0; w < P.nwg; ++w) {
      const int r0 = P.wg_row0[w], r1 = r0 + P.wg_nrows[w] - 1;
      P.wg_agg0[w] = L.vert_agg[r0];
      P.wg_nagg[w] = L.vert_agg[r1] - L.vert_agg[r0] + 1;
      P.max_wg_agg = std::max(P.max_wg_agg, P.wg_nagg[w]);
    }
    P.agg_wg0.resize(L.nagg);
    P.agg_nwg.resize(L.nagg);
    for (int a = 0; a < L.nagg; ++a) {
      const int b = L.agg_inst[a], voff = L.inst_voff[b];
      const int w0 = P.inst_wg0[b] + (L.agg_v0[a] - voff) / rows;
      const int w1 = P.inst_wg0[b] + (L.agg_v0[a + 1] - 1 - voff) / rows;
      P.agg_wg0[a] = w0;
      P.agg_nwg[a] = w1 - w0 + 1;
      P.max_agg_wg = std::max(P.max_agg_wg, w1 - w0 + 1);
    }
  }
  return P;
}

bool group_plan(HostPlan& P, int capacity, int max_groups) {
  P.group_wg0.assign(1, 0);
  int used = 0;
  for (size_t b = 0; b < P.inst_nwg.size(); ++b) {
    const int k = P.inst_nwg[b];
    if (k > capacity) return false;
    if (used + k > capacity) {
      P.group_wg0.push_back(P.inst_wg0[b]);
      used = 0;
    }
    used += k;
  }
  P.group_wg0.push_back(P.nwg);
  return (int)P.group_wg0.size() - 1 <= max_groups;
}

}  // namespace phisft

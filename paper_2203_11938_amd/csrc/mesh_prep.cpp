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

}  // namespace

int build_layout(const std::vector<HostSheet>& sheets, HostLayout& L, std::string& err) {
  L = HostLayout();
  L.ninst = (int)sheets.size();
  if (L.ninst < 1) {
    err = "no sheets";
    return -1;
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
  L.tri_area.assign(L.nt, 0.0);
  L.tri_inst.assign(L.nt, 0);
  std::vector<int> hv;   // [nh][4] global
  std::vector<double> hce, hrest;
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

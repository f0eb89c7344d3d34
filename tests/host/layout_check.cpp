// Host-side check of the layout builder (vertex order, aggregates, coarse pairs):
// a C wrapper around build_layout / check_layout / make_plan for the CPU tests.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "mesh_prep.h"

using namespace phisft;

extern "C" int layout_check(int nsheets, const int* nv, const int* nt, const int* tris,
                            const double* rest, const int* npins, const int* pins, int agg_size,
                            int max_aggs, int rows, int* out_vold, int* out_vert_agg,
                            int* out_counts, char* err, int errlen) {
  std::vector<HostSheet> sheets(nsheets);
  size_t to = 0, ro = 0, po = 0;
  for (int b = 0; b < nsheets; ++b) {
    HostSheet& s = sheets[b];
    s.nv = nv[b];
    s.nt = nt[b];
    s.tris.assign(tris + to, tris + to + 3 * (size_t)nt[b]);
    s.rest.assign(rest + ro, rest + ro + 3 * (size_t)nv[b]);
    s.pins.assign(pins + po, pins + po + npins[b]);
    s.mat[0] = 1e3;
    s.mat[1] = 1e-4;
    s.mat[2] = 0.1;
    to += 3 * (size_t)nt[b];
    ro += 3 * (size_t)nv[b];
    po += npins[b];
  }
  HostLayout L;
  std::string e;
  int rc = build_layout(sheets, agg_size, max_aggs, L, e);
  if (rc == 0 && !check_layout(L, e)) rc = -3;
  if (rc != 0) {
    std::strncpy(err, e.c_str(), errlen - 1);
    err[errlen - 1] = 0;
    return rc;
  }
  HostPlan P = make_plan(L, rows, 16);
  for (int i = 0; i < L.nv; ++i) {
    out_vold[i] = L.vold[i];
    out_vert_agg[i] = L.vert_agg[i];
  }
  int six = 0, three = 0, zero = 0;
  for (int m : L.agg_modes) (m == 6 ? six : m == 3 ? three : zero)++;
  out_counts[0] = L.nagg;
  out_counts[1] = L.max_nc;
  out_counts[2] = (int)L.pair_a.size();
  out_counts[3] = P.max_wg_agg;
  out_counts[4] = six;
  out_counts[5] = three;
  out_counts[6] = zero;
  out_counts[7] = L.maxnz;
  // every aggregate is covered by the workgroups that the plan says overlap it
  int bad = 0;
  for (int a = 0; a < L.nagg; ++a)
    for (int i = L.agg_v0[a]; i < L.agg_v0[a + 1]; ++i) {
      int w = -1;
      for (int q = P.agg_wg0[a]; q < P.agg_wg0[a] + P.agg_nwg[a]; ++q)
        if (i >= P.wg_row0[q] && i < P.wg_row0[q] + P.wg_nrows[q]) w = q;
      if (w < 0 || a - P.wg_agg0[w] < 0 || a - P.wg_agg0[w] >= P.wg_nagg[w]) ++bad;
    }
  out_counts[8] = bad;
  // halo tables: every local column names the right vertex
  int hbad = 0;
  for (int w = 0; w < P.nwg; ++w) {
    const int r0 = P.wg_row0[w], n = P.wg_nrows[w];
    const int h0 = P.halo_ptr[w], nh = P.halo_ptr[w + 1] - h0;
    if (nh > P.max_halo) ++hbad;
    for (int h = 0; h < nh; ++h) {
      const int j = P.halo_idx[h0 + h];
      if (j >= r0 && j < r0 + n) ++hbad;          // own rows are not halo
      if (h > 0 && P.halo_idx[h0 + h - 1] >= j) ++hbad;  // sorted, unique
    }
    for (int i = r0; i < r0 + n; ++i)
      for (int k = 0; k < L.maxnz; ++k) {
        const int j = L.ell_col[(size_t)k * L.nv + i], loc = P.lcol[(size_t)k * L.nv + i];
        int named;
        if (loc < 0 || loc >= rows + nh) { ++hbad; continue; }
        named = loc < rows ? r0 + loc : P.halo_idx[h0 + loc - rows];
        if (loc < rows && loc >= n) ++hbad;
        if (named != (j < 0 ? i : j)) ++hbad;
      }
  }
  out_counts[9] = hbad;
  out_counts[10] = P.max_halo;
  return 0;
}

// chamfer.hip -- Chamfer distance between two point sets on gfx950 (phi-SfT's
// evaluation metric, Sec. 4.2, Eq. 10):
//   Ch(G, M) = 1/|G| sum_g min_m |g - m|^2 + 1/|M| sum_m min_g |m - g|^2.
//
// Both nearest-neighbour searches run in one launch of k_chamfer_nn. A workgroup takes
// a block of 1024 query points (four per lane, coordinates in registers) and a tile of
// kChTile database points staged in LDS as three coordinate arrays (every lane reads the
// same point: an LDS broadcast), and keeps each query's smallest squared distance and
// its index; the tiles of one query block go to different workgroups, which merge their
// results with a 64-bit atomic minimum on (distance bits << 32 | index). Non-negative
// floats order like their bit patterns, so the merged value is the smallest distance
// and, among equal distances, the smallest index: the result does not depend on the
// order in which workgroups finish. Differences are formed coordinate by coordinate in
// FP32 (no |g|^2 + |m|^2 - 2 g.m expansion, whose cancellation would swamp the nearest
// distances), the means are accumulated in FP64 in a fixed order.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/phisft_sim.h"

namespace phisft {

constexpr int kChThreads = 256;
constexpr int kChQ = 4;                          // query points per lane
constexpr int kChBlockQ = kChThreads * kChQ;     // query points per workgroup
constexpr int kChTile = 2048;                    // database points per workgroup (LDS)

struct ChamferPass {
  const float* q;        // [3][nq] query points
  const float* db;       // [3][nd] database points
  int nq, nd;
  int qblocks;           // query blocks of this pass
  unsigned long long* best;   // [nq] packed minimum (distance bits << 32 | index)
};

__global__ void __launch_bounds__(kChThreads) k_chamfer_init(unsigned long long* best, long n,
                                                             int* bad) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) best[k] = ~0ull;
  if (k == 0) *bad = 0;
}

// Sum over the 64 lanes of a wavefront, the same in every lane (each step adds the
// same two values in either order).
__device__ __forceinline__ double wave_sum64(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __shfl_xor(t.x, o);
    t.y = __shfl_xor(t.y, o);
    v += *reinterpret_cast<double*>(&t);
  }
  return v;
}

// Workgroups [0, nb0) serve pass 0 (queries G, database M), the rest pass 1 (M into G):
// block b of a pass covers query block b % qblocks and database tile b / qblocks.
__global__ void __launch_bounds__(kChThreads) k_chamfer_nn(ChamferPass p0, ChamferPass p1,
                                                           int nb0, int* bad) {
  __shared__ float sx[kChTile], sy[kChTile], sz[kChTile];
  const bool second = (int)blockIdx.x >= nb0;
  const ChamferPass& p = second ? p1 : p0;
  const int b = second ? (int)blockIdx.x - nb0 : (int)blockIdx.x;
  const int qb = b % p.qblocks, tile = b / p.qblocks;
  const int d0 = tile * kChTile, nloc = min(kChTile, p.nd - d0);
  const int tid = threadIdx.x;
  for (int j = tid; j < nloc; j += kChThreads) {
    sx[j] = p.db[d0 + j];
    sy[j] = p.db[p.nd + d0 + j];
    sz[j] = p.db[2 * p.nd + d0 + j];
  }
  float qx[kChQ], qy[kChQ], qz[kChQ], bd[kChQ];
  int bi[kChQ];
#pragma unroll
  for (int k = 0; k < kChQ; ++k) {
    // lanes past the last query search with a copy of it and store nothing
    const int i = min(qb * kChBlockQ + k * kChThreads + tid, p.nq - 1);
    qx[k] = p.q[i];
    qy[k] = p.q[p.nq + i];
    qz[k] = p.q[2 * p.nq + i];
    bd[k] = INFINITY;
    bi[k] = 0;
  }
  // every point is a query of exactly one block of its pass (tile 0 checks it)
  if (tile == 0) {
    bool fin = true;
#pragma unroll
    for (int k = 0; k < kChQ; ++k) fin = fin && isfinite(qx[k]) && isfinite(qy[k]) && isfinite(qz[k]);
    if (!fin) atomicOr(bad, 1);
  }
  __syncthreads();
  for (int j = 0; j < nloc; ++j) {
    const float x = sx[j], y = sy[j], z = sz[j];
#pragma unroll
    for (int k = 0; k < kChQ; ++k) {
      const float dx = qx[k] - x, dy = qy[k] - y, dz = qz[k] - z;
      const float d = dx * dx + dy * dy + dz * dz;
      if (d < bd[k]) {   // strictly smaller: the first index among equal distances stays
        bd[k] = d;
        bi[k] = j;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kChQ; ++k) {
    const int i = qb * kChBlockQ + k * kChThreads + tid;
    if (i < p.nq && nloc > 0) {
      const unsigned long long v =
          ((unsigned long long)__float_as_uint(bd[k]) << 32) | (unsigned)(d0 + bi[k]);
      atomicMin(p.best + i, v);
    }
  }
}

// Unpacks the minima of one set (distance and index, either output optional) and sums
// the distances per workgroup in FP64 (fixed order: a butterfly per wavefront, then the
// wavefronts in order).
__global__ void __launch_bounds__(kChThreads) k_chamfer_unpack(const unsigned long long* best, int n,
                                                               float* d, int* idx, double* part) {
  __shared__ double s_w[kChThreads / 64];
  const int i = blockIdx.x * kChThreads + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const unsigned long long w = best[i];
    const float dist = __uint_as_float((unsigned)(w >> 32));
    if (d) d[i] = dist;
    if (idx) idx[i] = (int)(unsigned)(w & 0xffffffffu);
    v = dist;
  }
  v = wave_sum64(v);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kChThreads / 64; ++w) t += s_w[w];
    part[blockIdx.x] = t;
  }
}

// Ch = (sum of G's partials) / |G| + (sum of M's partials) / |M|, one workgroup, fixed
// order; NaN when an input coordinate was not finite.
__global__ void __launch_bounds__(kChThreads) k_chamfer_sum(const double* pg, int nbg, int ng,
                                                            const double* pm, int nbm, int nm,
                                                            const int* bad, double* ch) {
  __shared__ double s_w[2][kChThreads / 64];
  double a = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nbg; k += kChThreads) a += pg[k];
  for (int k = threadIdx.x; k < nbm; k += kChThreads) c += pm[k];
  a = wave_sum64(a);
  c = wave_sum64(c);
  if ((threadIdx.x & 63) == 0) {
    s_w[0][threadIdx.x >> 6] = a;
    s_w[1][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sc = 0.0;
    for (int w = 0; w < kChThreads / 64; ++w) {
      sa += s_w[0][w];
      sc += s_w[1][w];
    }
    *ch = *bad ? NAN : sa / ng + sc / nm;
  }
}

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

struct ChamferLayout {
  size_t best_g, best_m, part_g, part_m, bad, total;
  int nbg, nbm;
};

static ChamferLayout chamfer_layout(int ng, int nm) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  ChamferLayout L{};
  L.nbg = cdiv(ng, kChThreads);
  L.nbm = cdiv(nm, kChThreads);
  L.best_g = 0;
  L.best_m = up(8 * (size_t)ng);
  L.part_g = L.best_m + up(8 * (size_t)nm);
  L.part_m = L.part_g + up(8 * (size_t)L.nbg);
  L.bad = L.part_m + up(8 * (size_t)L.nbm);
  L.total = L.bad + 256;
  return L;
}

}  // namespace phisft

using namespace phisft;

extern "C" {

size_t sim_chamfer_workspace_bytes(int32_t n_g, int32_t n_m) {
  if (n_g < 1 || n_m < 1) return 0;
  return chamfer_layout(n_g, n_m).total;
}

sim_status sim_chamfer(const float* g, int32_t n_g, const float* m, int32_t n_m, double* ch,
                       float* d_g, int32_t* i_g, float* d_m, int32_t* i_m, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (!g || !m || !ch || !workspace || n_g < 1 || n_m < 1) return SIM_E_INVALID;
  const ChamferLayout L = chamfer_layout(n_g, n_m);
  if (workspace_bytes < L.total) return SIM_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  auto* bg = reinterpret_cast<unsigned long long*>(w + L.best_g);
  auto* bm = reinterpret_cast<unsigned long long*>(w + L.best_m);
  auto* pg = reinterpret_cast<double*>(w + L.part_g);
  auto* pm = reinterpret_cast<double*>(w + L.part_m);
  int* bad = reinterpret_cast<int*>(w + L.bad);
  // the two packed-minimum arrays are contiguous up to alignment padding, which the
  // fill covers as well (it lies inside the workspace)
  const long nfill = (long)(L.part_g - L.best_g) / 8;
  hipLaunchKernelGGL(k_chamfer_init, dim3(cdiv(nfill, kChThreads)), dim3(kChThreads), 0, st, bg,
                     nfill, bad);
  ChamferPass p0{g, m, n_g, n_m, cdiv(n_g, kChBlockQ), bg};
  ChamferPass p1{m, g, n_m, n_g, cdiv(n_m, kChBlockQ), bm};
  const long nb0 = (long)p0.qblocks * cdiv(n_m, kChTile), nb1 = (long)p1.qblocks * cdiv(n_g, kChTile);
  if (nb0 + nb1 > 0x7fffffffL) return SIM_E_INVALID;
  hipLaunchKernelGGL(k_chamfer_nn, dim3((unsigned)(nb0 + nb1)), dim3(kChThreads), 0, st, p0, p1,
                     (int)nb0, bad);
  hipLaunchKernelGGL(k_chamfer_unpack, dim3(L.nbg), dim3(kChThreads), 0, st, bg, n_g, d_g, i_g, pg);
  hipLaunchKernelGGL(k_chamfer_unpack, dim3(L.nbm), dim3(kChThreads), 0, st, bm, n_m, d_m, i_m, pm);
  hipLaunchKernelGGL(k_chamfer_sum, dim3(1), dim3(kChThreads), 0, st, pg, L.nbg, n_g, pm, L.nbm,
                     n_m, bad, ch);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_E_HIP;
}

}  // extern "C"

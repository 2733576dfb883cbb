// FE <-> FFT mapping by nearest Gauss point: the Gauss points of a finite
// element mesh seed a Voronoi tessellation of the FFT grid, every cell takes
// the data of the Gauss point nearest to its centre, and every Gauss point
// takes the mean of the cells of its domain (see include/pf.h).
//
// Build: the points are counting-sorted into a uniform grid of bins of about
// one point each (bounding box on the device, bin grid sized on the host
// from it); one thread per cell then searches shells of bins of growing
// Chebyshev radius around the cell's bin, in FP64, until no unvisited bin
// can hold a point as near as the best one found. Ties go to the lower point
// index, so the result does not depend on the order inside a bin.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <climits>
#include <cmath>
#include <cstdint>
#include "../../include/pf.h"

namespace pfv {

struct BinGrid {
  double lo[3];  // corner of the bin box
  double h;      // bin edge
  int nb[3];     // bins per axis
  int nbins;
};

struct SortedPoint {
  double x, y, z;
  int idx;
  int pad;
};

constexpr int kThreads = 256;

// Workspace: [bbox 8 doubles][counts][offsets nbins_max + 1][fill nbins_max]
// [sorted points][point offsets n_points + 1][cell iota n_cells][sorted keys
// n_cells][cell lists n_cells][library scratch]. The point offsets and the
// cell lists (each point's cells, ascending) stay valid from pf_vmap_build
// to pf_vmap_to_points.
inline size_t align256(size_t n) { return (n + 255) / 256 * 256; }
inline int64_t max_bins(int32_t n_points) { return 2 * (int64_t)n_points + 64; }
inline int key_bits(int32_t n_points) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n_points) ++b;
  return b;
}

struct WsLayout {
  size_t bbox, counts, offsets, fill, sorted, poff, iota, keys, plist, temp, temp_bytes, total;
};

inline WsLayout ws_layout(int64_t n_cells, int32_t n_points) {
  WsLayout w{};
  const int64_t nb = max_bins(n_points);
  const int64_t ncount = (nb > n_points ? nb : n_points) + 1;
  size_t t1 = 0, t2 = 0, t3 = 0;
  hipcub::DeviceScan::ExclusiveSum(nullptr, t1, (int*)nullptr, (int*)nullptr, (int)(nb + 1));
  hipcub::DeviceScan::ExclusiveSum(nullptr, t2, (int*)nullptr, (int*)nullptr, n_points + 1);
  hipcub::DeviceRadixSort::SortPairs(nullptr, t3, (const unsigned*)nullptr, (unsigned*)nullptr, (const int*)nullptr,
                                     (int*)nullptr, (int)n_cells, 0, key_bits(n_points));
  w.temp_bytes = t1 > t2 ? (t1 > t3 ? t1 : t3) : (t2 > t3 ? t2 : t3);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  w.bbox = take(8 * sizeof(double));
  w.counts = take(sizeof(int) * ncount);
  w.offsets = take(sizeof(int) * (nb + 1));
  w.fill = take(sizeof(int) * nb);
  w.sorted = take(sizeof(SortedPoint) * (size_t)n_points);
  w.poff = take(sizeof(int) * ((size_t)n_points + 1));
  w.iota = take(sizeof(int) * (size_t)n_cells);
  w.keys = take(sizeof(int) * (size_t)n_cells);
  w.plist = take(sizeof(int) * (size_t)n_cells);
  w.temp = take(w.temp_bytes);
  w.total = off;
  return w;
}

// ------------------------------------------------------------------ build
// Bounding box of the points and a flag for non-finite coordinates (one block).
__global__ __launch_bounds__(1024) void k_bbox(const double* __restrict__ pts, int n, double* __restrict__ out) {
  __shared__ double red[6][32];
  __shared__ int bad_any;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  if (threadIdx.x == 0) bad_any = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = pts[3 * (size_t)i + d];
      if (!isfinite(v)) bad = 1;
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
    }
  }
  if (bad) atomicOr(&bad_any, 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn[d] = fmin(mn[d], __shfl_xor(mn[d], o, 64));
      mx[d] = fmax(mx[d], __shfl_xor(mx[d], o, 64));
    }
  if (lane == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[d][wave] = mn[d];
      red[3 + d][wave] = mx[d];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    double v = red[d][0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = d < 3 ? fmin(v, red[d][w]) : fmax(v, red[d][w]);
    out[d] = v;
  }
  if (threadIdx.x == 0) out[6] = bad_any ? 1.0 : 0.0;
}

__device__ __forceinline__ int bin_axis(double v, double lo, double h, int nb) {
  int b = (int)floor((v - lo) / h);
  return b < 0 ? 0 : (b >= nb ? nb - 1 : b);
}

__device__ __forceinline__ int bin_of(const BinGrid& g, double x, double y, double z) {
  const int bx = bin_axis(x, g.lo[0], g.h, g.nb[0]);
  const int by = bin_axis(y, g.lo[1], g.h, g.nb[1]);
  const int bz = bin_axis(z, g.lo[2], g.h, g.nb[2]);
  return (bz * g.nb[1] + by) * g.nb[0] + bx;
}

__global__ void k_zero_int(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_count(const double* __restrict__ pts, int n, const BinGrid g, int* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* p = pts + 3 * (size_t)i;
  atomicAdd(&counts[bin_of(g, p[0], p[1], p[2])], 1);
}

__global__ void k_scatter(const double* __restrict__ pts, int n, const BinGrid g, const int* __restrict__ offsets,
                          int* __restrict__ fill, SortedPoint* __restrict__ sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* p = pts + 3 * (size_t)i;
  const int b = bin_of(g, p[0], p[1], p[2]);
  const int slot = offsets[b] + atomicAdd(&fill[b], 1);
  sorted[slot] = SortedPoint{p[0], p[1], p[2], i, 0};
}

// Nearest point of every cell centre. The shell of radius r around the
// cell's bin holds the bins at Chebyshev distance r; after shells 0..r every
// point outside the visited block lies beyond the nearest face of the block
// that has bins behind it, so the search stops once that distance (shrunk by
// a margin for the rounding of the bin assignment) exceeds the best one.
__global__ __launch_bounds__(kThreads) void k_search(const BinGrid g, const int* __restrict__ offsets,
                                                     const SortedPoint* __restrict__ sorted, int nx, int ny,
                                                     int nz, double dx, int32_t* __restrict__ cell_point) {
  // the squared distance decides an index: rounded multiplies and adds in
  // a fixed order, never contracted to fused multiply-adds
#pragma clang fp contract(off)
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncell = (int64_t)nx * ny * nz;
  if (cell >= ncell) return;
  const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / ((int64_t)nx * ny));
  const double c[3] = {(i + 0.5) * dx, (j + 0.5) * dx, (k + 0.5) * dx};
  int b0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) b0[d] = bin_axis(c[d], g.lo[d], g.h, g.nb[d]);
  double best = INFINITY;
  int bidx = INT_MAX;
  const double margin = 1e-9 * g.h;
  for (int r = 0;; ++r) {
    for (int dz = -r; dz <= r; ++dz) {
      const int bz = b0[2] + dz;
      if (bz < 0 || bz >= g.nb[2]) continue;
      for (int dy = -r; dy <= r; ++dy) {
        const int by = b0[1] + dy;
        if (by < 0 || by >= g.nb[1]) continue;
        const bool face = dz == -r || dz == r || dy == -r || dy == r;
        const int step = (face || r == 0) ? 1 : 2 * r;
        for (int dxb = -r; dxb <= r; dxb += step) {
          const int bx = b0[0] + dxb;
          if (bx < 0 || bx >= g.nb[0]) continue;
          const int b = (bz * g.nb[1] + by) * g.nb[0] + bx;
          const int e = offsets[b + 1];
          for (int s = offsets[b]; s < e; ++s) {
            const SortedPoint p = sorted[s];
            double d2 = (p.x - c[0]) * (p.x - c[0]);
            d2 = d2 + (p.y - c[1]) * (p.y - c[1]);
            d2 = d2 + (p.z - c[2]) * (p.z - c[2]);
            if (d2 < best || (d2 == best && p.idx < bidx)) {
              best = d2;
              bidx = p.idx;
            }
          }
        }
      }
    }
    // distance to the nearest face of the visited block with bins beyond it
    double bound = INFINITY;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (b0[d] - r > 0) bound = fmin(bound, c[d] - (g.lo[d] + (b0[d] - r) * g.h));
      if (b0[d] + r + 1 < g.nb[d]) bound = fmin(bound, g.lo[d] + (b0[d] + r + 1) * g.h - c[d]);
    }
    if (bound == INFINITY) break;  // the block covers every bin
    const double bs = bound - margin;
    if (bs > 0.0 && bs * bs > best) break;
  }
  cell_point[cell] = bidx;
}

// ---------------------------------------------------------------- transfer
// Four consecutive cells per thread: one 16-byte index load, the point
// values gathered (they stay in L2), one 16-byte store per component.
// vec: the host found ncell a multiple of 4 and both arrays 16-byte aligned.
__global__ void k_to_cells(int64_t ncell, const int32_t* __restrict__ cp, int npts, int ncomp,
                           const float* __restrict__ pv, float* __restrict__ cv, int vec) {
  const int64_t c0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (c0 >= ncell) return;
  if (vec) {
    const int4 p = *reinterpret_cast<const int4*>(cp + c0);
    for (int c = 0; c < ncomp; ++c) {
      const float* v = pv + (int64_t)c * npts;
      *reinterpret_cast<float4*>(cv + c * ncell + c0) = make_float4(v[p.x], v[p.y], v[p.z], v[p.w]);
    }
    return;
  }
  for (int64_t cell = c0; cell < c0 + 4 && cell < ncell; ++cell) {
    const int p = cp[cell];
    for (int c = 0; c < ncomp; ++c) cv[c * ncell + cell] = pv[(int64_t)c * npts + p];
  }
}

// Per-point cell lists: a stable radix sort of (point, cell) pairs taken in
// ascending cell order leaves each point's cells ascending, so every sum
// over a domain runs in cell order; the counts give the row offsets.
__global__ void k_cell_count(int64_t ncell, const int32_t* __restrict__ cp, int* __restrict__ pcount) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < ncell) atomicAdd(&pcount[cp[cell]], 1);
}

__global__ void k_iota(int64_t n, int* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int)i;
}

// Mean over each point's domain: FP64 sum in ascending cell order, one
// division; an empty domain takes the cell that contains the point.
__global__ void k_to_points(int npts, int ncomp, const int* __restrict__ poff, const int* __restrict__ plist,
                            const double* __restrict__ pts, int nx, int ny, int nz, double dx, int64_t ncell,
                            const float* __restrict__ cv, float* __restrict__ pv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const int b = poff[p], e = poff[p + 1];
  if (e > b) {
    const double cnt = (double)(e - b);
    for (int c = 0; c < ncomp; ++c) {
      const float* v = cv + c * ncell;
      double s = 0.0;
      for (int k = b; k < e; ++k) s += (double)v[plist[k]];
      pv[(int64_t)c * npts + p] = (float)(s / cnt);
    }
    return;
  }
  const double* q = pts + 3 * (size_t)p;
  const int n[3] = {nx, ny, nz};
  int64_t ix[3];
  for (int d = 0; d < 3; ++d) {
    const double f = floor(q[d] / dx);
    ix[d] = f < 0.0 ? 0 : (f >= n[d] ? n[d] - 1 : (int64_t)f);
  }
  const int64_t cell = (ix[2] * ny + ix[1]) * nx + ix[0];
  for (int c = 0; c < ncomp; ++c) pv[(int64_t)c * npts + p] = cv[c * ncell + cell];
}

inline int blocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

}  // namespace pfv

using namespace pfv;

namespace {
int grid_ok(int32_t nx, int32_t ny, int32_t nz, double dx) {
  if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !std::isfinite(dx)) return 0;
  return (int64_t)nx * ny * nz < ((int64_t)1 << 31);
}
int hip_rc(hipError_t e) { return e == hipSuccess ? PF_OK : PF_EDEVICE; }
}  // namespace

extern "C" {

int pf_vmap_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t n_points, size_t* bytes) {
  if (!bytes || !grid_ok(nx, ny, nz, 1.0) || n_points < 1 || n_points > (1 << 28)) return PF_EINVAL;
  *bytes = ws_layout((int64_t)nx * ny * nz, n_points).total;
  return PF_OK;
}

int pf_vmap_build(int32_t nx, int32_t ny, int32_t nz, double dx, int32_t n_points, const double* points,
                  void* workspace, size_t ws_bytes, void* hip_stream, int32_t* cell_point) {
  if (!grid_ok(nx, ny, nz, dx) || n_points < 1 || n_points > (1 << 28) || !points || !workspace || !cell_point)
    return PF_EINVAL;
  const int64_t ncell = (int64_t)nx * ny * nz;
  const WsLayout w = ws_layout(ncell, n_points);
  if (ws_bytes < w.total) return PF_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char* ws = static_cast<char*>(workspace);
  double* bbox = reinterpret_cast<double*>(ws + w.bbox);
  k_bbox<<<1, 1024, 0, s>>>(points, n_points, bbox);
  hipError_t e = hipGetLastError();
  double hb[7];
  if (e == hipSuccess) e = hipMemcpyAsync(hb, bbox, sizeof(hb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return PF_EDEVICE;
  if (hb[6] != 0.0) return PF_EINVAL;  // a non-finite coordinate
  // bin box: the points and the cell centres together; bins of about one point
  BinGrid g{};
  const double clo[3] = {0.5 * dx, 0.5 * dx, 0.5 * dx};
  const double chi[3] = {(nx - 0.5) * dx, (ny - 0.5) * dx, (nz - 0.5) * dx};
  double ext[3];
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    g.lo[d] = std::fmin(hb[d], clo[d]);
    const double hi = std::fmax(hb[3 + d], chi[d]);
    ext[d] = std::fmax(hi - g.lo[d], dx);
    vol *= ext[d];
  }
  g.h = std::cbrt(vol / n_points);
  const int64_t cap = max_bins(n_points);
  for (;;) {
    int64_t tot = 1;
    for (int d = 0; d < 3; ++d) {
      const double nbd = std::ceil(ext[d] / g.h);
      g.nb[d] = nbd < 1.0 ? 1 : (nbd > 1e6 ? 1000000 : (int)nbd);
      tot *= g.nb[d];
    }
    if (tot <= cap) {
      g.nbins = (int)tot;
      break;
    }
    g.h *= 1.25;
  }
  int* counts = reinterpret_cast<int*>(ws + w.counts);
  int* offsets = reinterpret_cast<int*>(ws + w.offsets);
  int* fill = reinterpret_cast<int*>(ws + w.fill);
  SortedPoint* sorted = reinterpret_cast<SortedPoint*>(ws + w.sorted);
  void* temp = ws + w.temp;
  size_t tb = w.temp_bytes;
  k_zero_int<<<blocks(g.nbins + 1), kThreads, 0, s>>>(counts, g.nbins + 1);
  k_zero_int<<<blocks(g.nbins), kThreads, 0, s>>>(fill, g.nbins);
  k_count<<<blocks(n_points), kThreads, 0, s>>>(points, n_points, g, counts);
  if ((e = hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, offsets, g.nbins + 1, s)) != hipSuccess)
    return PF_EDEVICE;
  k_scatter<<<blocks(n_points), kThreads, 0, s>>>(points, n_points, g, offsets, fill, sorted);
  k_search<<<blocks(ncell), kThreads, 0, s>>>(g, offsets, sorted, nx, ny, nz, dx, cell_point);
  // each point's cells, ascending
  int* poff = reinterpret_cast<int*>(ws + w.poff);
  int* iota = reinterpret_cast<int*>(ws + w.iota);
  unsigned* keys = reinterpret_cast<unsigned*>(ws + w.keys);
  int* plist = reinterpret_cast<int*>(ws + w.plist);
  k_zero_int<<<blocks(n_points + 1), kThreads, 0, s>>>(counts, n_points + 1);
  k_cell_count<<<blocks(ncell), kThreads, 0, s>>>(ncell, cell_point, counts);
  tb = w.temp_bytes;
  if ((e = hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, poff, n_points + 1, s)) != hipSuccess)
    return PF_EDEVICE;
  k_iota<<<blocks(ncell), kThreads, 0, s>>>(ncell, iota);
  tb = w.temp_bytes;
  if ((e = hipcub::DeviceRadixSort::SortPairs(temp, tb, reinterpret_cast<const unsigned*>(cell_point), keys,
                                              iota, plist, (int)ncell, 0, key_bits(n_points), s)) != hipSuccess)
    return PF_EDEVICE;
  return hip_rc(hipGetLastError());
}

int pf_vmap_to_cells(int64_t n_cells, const int32_t* cell_point, int32_t n_points, int32_t ncomp,
                     const float* point_values, float* cell_values, void* hip_stream) {
  if (n_cells < 1 || n_points < 1 || ncomp < 1 || !cell_point || !point_values || !cell_values) return PF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int vec = (n_cells % 4 == 0) && reinterpret_cast<uintptr_t>(cell_point) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(cell_values) % 16 == 0;
  k_to_cells<<<blocks((n_cells + 3) / 4), kThreads, 0, s>>>(n_cells, cell_point, n_points, ncomp, point_values,
                                                              cell_values, vec);
  return hip_rc(hipGetLastError());
}

int pf_vmap_to_points(int32_t nx, int32_t ny, int32_t nz, double dx, const int32_t* cell_point, int32_t n_points,
                      const double* points, int32_t ncomp, const float* cell_values, float* point_values,
                      const void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!grid_ok(nx, ny, nz, dx) || n_points < 1 || n_points > (1 << 28) || ncomp < 1 || !cell_point || !points ||
      !cell_values || !point_values || !workspace)
    return PF_EINVAL;
  const int64_t ncell = (int64_t)nx * ny * nz;
  const WsLayout w = ws_layout(ncell, n_points);
  if (ws_bytes < w.total) return PF_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const char* ws = static_cast<const char*>(workspace);
  const int* poff = reinterpret_cast<const int*>(ws + w.poff);
  const int* plist = reinterpret_cast<const int*>(ws + w.plist);
  k_to_points<<<blocks(n_points), kThreads, 0, s>>>(n_points, ncomp, poff, plist, points, nx, ny, nz, dx, ncell,
                                                    cell_values, point_values);
  return hip_rc(hipGetLastError());
}

}  // extern "C"

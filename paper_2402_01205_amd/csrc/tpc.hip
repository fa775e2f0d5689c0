// MI355X (gfx950) TPC track reconstruction: kernels and the C ABI host runtime.
//
// Stages (see include/tpc.h): grid build (counting sort into per-row cell grids),
// neighbour links + cleaning + chain starts, tracklet construction (one lane per
// tracklet, FP32 Kalman filter), selection (max-key ownership), refit and
// sector merge; around them, cluster finding from digits, track-model compression
// and the rANS coder.  No stage uses MFMA: nothing here is a dense contraction;
// every kernel is bound by HBM traffic, instruction issue or dependent-load latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpc.h"
#include "tpc_kernels.h"
#include "tpc_math.h"

#pragma clang fp contract(off)

using namespace tpc;

namespace {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ int cell_of(float v, float lo, float inv, int n) {
  float c = (v - lo) * inv;
  c = fminf(fmaxf(c, 0.f), (float)(n - 1));
  return (int)c;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if ((int)(threadIdx.x & 63) >= o) v += t;
  }
  return v;
}

// block-wide exclusive scan of one value per thread (blockDim.x <= 1024, multiple of 64)
__device__ __forceinline__ int block_excl_scan(int v, int* lds_waves, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int inc = wave_incl_scan(v);
  if (lane == 63) lds_waves[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    int w = lane < nw ? lds_waves[lane] : 0;
    const int wi = wave_incl_scan(w);
    if (lane < nw) lds_waves[lane] = wi - w;
    if (lane == nw - 1) lds_waves[32] = wi;
  }
  __syncthreads();
  total = lds_waves[32];
  const int r = inc - v + lds_waves[wave];
  __syncthreads();
  return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs by block index; remapping
// block b to logical tile (b % 8) * ceil(nb / 8) + b / 8 gives each XCD (and its L2)
// a contiguous range of tiles.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t per = (nb + kXcds - 1) / kXcds;
  const int64_t x = b % kXcds, i = b / kXcds;
  const int64_t full = nb % kXcds == 0 ? kXcds : nb % kXcds;  // XCDs that get `per` tiles
  return x < full ? x * per + i : full * per + (x - full) * (per - 1) + i;
}

// ------------------------------------------------------------------ fill / scan
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = v;
}
__global__ void k_fill_range_u8(uint8_t* p, Bound lo, Bound hi, uint8_t v) {
  const int32_t a = lo.get(), b = hi.get();
  for (int64_t k = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < b;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}
__global__ void k_fill_range_i32(int32_t* p, Bound lo, Bound hi, int32_t v) {
  const int32_t a = lo.get(), b = hi.get();
  for (int64_t k = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < b;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

// Exclusive scan of in[lo..hi) into out[lo..hi], out[lo] = base (base = *base_p or 0), in
// tiles of kScanTile elements.  Loads and stores are striped (element q * 256 + j of a tile
// goes to thread j, so a wave touches 64 consecutive ints); the apply pass turns the tile
// into 8 consecutive elements per thread through LDS for the per-thread scan.
// The scanned input is int32 or bytes (0/1 flags); sums are int32.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T* in, Bound lo_b, Bound hi_b, int32_t* bsum) {
  __shared__ int lds[40];
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int64_t start = (int64_t)lo + (int64_t)blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t i = start + (int64_t)q * kScanThreads + threadIdx.x;
    if (i < hi) s += (int)in[i];
  }
  int total;
  block_excl_scan(s, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}
// base_from_out: the scan continues a previous one whose total sits in out[lo].
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t* bsum, Bound lo_b, Bound hi_b,
                                                      int32_t base_from_out, int32_t* out) {
  __shared__ int lds[40];
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int nb = hi > lo ? (int)((hi - lo + kScanTile - 1) / kScanTile) : 0;
  int carry = base_from_out ? out[lo] : 0;
  __syncthreads();
  for (int c = 0; c < nb; c += blockDim.x) {
    const int i = c + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int total;
    const int e = block_excl_scan(v, lds, total);
    if (i < nb) bsum[i] = carry + e;
    carry += total;
  }
  if (threadIdx.x == 0) out[hi > lo ? hi : lo] = carry;
}
// LDS slot of tile element i: one padding word per 32 keeps the per-thread reads of 8
// consecutive elements from piling onto the same banks.
__device__ __forceinline__ int scan_slot(int i) { return i + (i >> 5); }
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const T* in, int32_t* out, Bound lo_b, Bound hi_b,
                                                             const int32_t* bsum) {
  __shared__ int lds[40];
  __shared__ int tile[kScanTile + kScanTile / 32];
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int64_t start = (int64_t)lo + (int64_t)blockIdx.x * kScanTile;
  if (start >= hi) return;
  const int j = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t i = start + (int64_t)q * kScanThreads + j;
    tile[scan_slot(q * kScanThreads + j)] = i < hi ? (int)in[i] : 0;
  }
  __syncthreads();
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = tile[scan_slot(j * kScanItems + q)];
    s += v[q];
  }
  int total;
  int e = block_excl_scan(s, lds, total) + bsum[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    tile[scan_slot(j * kScanItems + q)] = e;
    e += v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t i = start + (int64_t)q * kScanThreads + j;
    if (i < hi) out[i] = tile[scan_slot(q * kScanThreads + j)];
  }
}

// ------------------------------------------------------------------ a1: grid build
struct In {
  const uint8_t* sector;
  const int16_t* row;
  const float* y;
  const float* z;
  const int32_t* job_off;
  int32_t n_jobs;
};

__device__ __forceinline__ int job_of(const int32_t* job_off, int n_jobs, int32_t i) {
  int a = 0, b = n_jobs;  // job_off[a] <= i < job_off[b]
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if (job_off[m] <= i) a = m; else b = m;
  }
  return a;
}

// Validate each input cluster, compute its slot, count clusters per slot and the
// per-slot z range (order-preserving integer min/max); each cluster's rank in its slot
// comes from the count.
__global__ void k_grid_count(In in, Bound lo_b, Bound hi_b, int32_t* ckey, int32_t* srank, int32_t* slot_cnt,
                             uint32_t* zmin, uint32_t* zmax, int32_t* counters) {
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int32_t i = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hi) return;
  const int s = in.sector[i];
  const int r = in.row[i];
  const float y = in.y[i], z = in.z[i];
  const bool ok = s < kSectors && r >= 0 && r < kRows && finite_f(y) && finite_f(z);
  if (!ok) {
    ckey[i] = -1;
    atomicOr(&counters[kCntStatus], kStatusRange);
    return;
  }
  const int j = job_of(in.job_off, in.n_jobs, i);
  const int32_t slot = (j * kSectors + s) * kRows + r;
  ckey[i] = slot;
  srank[i] = atomicAdd(&slot_cnt[slot], 1);
  const uint32_t oz = f2ord(z);
  atomicMin(&zmin[slot], oz);
  atomicMax(&zmax[slot], oz);
}

// Same as k_grid_count, with the per-slot counters and z ranges of the block's job
// privatised in LDS (a block covers kCountTile consecutive input clusters, almost
// always of one job) and flushed with one global atomic per touched slot.  Clusters
// of another job (at a job boundary) update global memory directly.  A cluster's rank in
// its slot is its rank in the block's LDS count plus the block's base, which the flush's
// atomic returns.
constexpr int kCountThreads = 1024;
constexpr int kCountTile = kCountThreads * 4;
__global__ __launch_bounds__(kCountThreads) void k_grid_count_lds(In in, Bound lo_b, Bound hi_b, int32_t* ckey,
                                                                   int32_t* srank, int32_t* slot_cnt, uint32_t* zmin,
                                                                   uint32_t* zmax, int32_t* counters) {
  extern __shared__ uint32_t lds[];
  uint32_t* s_cnt = lds;
  uint32_t* s_zmin = lds + kSlotsPerJob;
  uint32_t* s_zmax = lds + 2 * kSlotsPerJob;
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int64_t base = (int64_t)lo + (int64_t)blockIdx.x * kCountTile;
  if (base >= hi) return;
  const int32_t end = (int32_t)std::min<int64_t>(base + kCountTile, hi);
  const int job0 = job_of(in.job_off, in.n_jobs, (int32_t)base);
  const bool one_job = in.job_off[job0 + 1] >= end;
  for (int s = threadIdx.x; s < kSlotsPerJob; s += kCountThreads) {
    s_cnt[s] = 0u;
    s_zmin[s] = 0xFFFFFFFFu;
    s_zmax[s] = 0u;
  }
  __syncthreads();
  bool bad = false;
  constexpr int kQ = kCountTile / kCountThreads;
  int lslot[kQ], lrank[kQ];  // LDS slot (-1: none) and rank in the block's count
#pragma unroll
  for (int q = 0; q < kQ; ++q) lslot[q] = -1;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int32_t i = (int32_t)base + q * kCountThreads + threadIdx.x;
    if (i >= end) break;
    const int s = in.sector[i];
    const int r = in.row[i];
    const float y = in.y[i], z = in.z[i];
    if (!(s < kSectors && r >= 0 && r < kRows && finite_f(y) && finite_f(z))) {
      ckey[i] = -1;
      bad = true;
      continue;
    }
    const int j = one_job ? job0 : job_of(in.job_off, in.n_jobs, i);
    const int local = s * kRows + r;
    const int32_t slot = j * kSlotsPerJob + local;
    ckey[i] = slot;
    const uint32_t oz = f2ord(z);
    if (j == job0) {
      lslot[q] = local;
      lrank[q] = (int)atomicAdd(&s_cnt[local], 1u);
      atomicMin(&s_zmin[local], oz);
      atomicMax(&s_zmax[local], oz);
    } else {
      srank[i] = atomicAdd(&slot_cnt[slot], 1);
      atomicMin(&zmin[slot], oz);
      atomicMax(&zmax[slot], oz);
    }
  }
  if (bad) atomicOr(&counters[kCntStatus], kStatusRange);
  __syncthreads();
  for (int s = threadIdx.x; s < kSlotsPerJob; s += kCountThreads) {
    const uint32_t c = s_cnt[s];
    if (c) {
      const int32_t slot = job0 * kSlotsPerJob + s;
      s_cnt[s] = (uint32_t)atomicAdd(&slot_cnt[slot], (int32_t)c);
      atomicMin(&zmin[slot], s_zmin[s]);
      atomicMax(&zmax[slot], s_zmax[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    if (lslot[q] >= 0) srank[base + q * kCountThreads + threadIdx.x] = (int32_t)s_cnt[lslot[q]] + lrank[q];
}

// Cell geometry of every slot: roughly cells_per_cluster cells per cluster, square
// cells in (y, z) over the row's acceptance in y and the slot's z range.  Non-empty
// slots are appended (in no particular order) to slot_list, whose count sits in front.
constexpr int kListCount = 0, kListFirst = 1;
__global__ void k_slot_geometry(const int32_t* slot_cnt, const uint32_t* zmin, const uint32_t* zmax,
                                SlotGrid* sg, int32_t* ncell, int32_t* slot_list, int32_t s0, int32_t s1,
                                Consts k, float cpc) {
  const int32_t s = s0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= s1) return;
  const int n = slot_cnt[s];
  if (n > 0) slot_list[kListFirst + atomicAdd(&slot_list[kListCount], 1)] = s;
  SlotGrid g;
  g.cbase = 0;
  if (n == 0) {
    g.ylo = g.zlo = g.inv_by = g.inv_bz = 0.f;
    g.ny = g.nz = g.ncell = 0;
  } else {
    const float x = k.x[s % kRows];
    const float yh = x * k.tan10 + 1.f;
    const float ywid = 2.f * yh;
    const float z0 = ord2f(zmin[s]), z1 = ord2f(zmax[s]);
    const float zspan = fmaxf(z1 - z0, 1e-3f) * 1.000001f + 1e-3f;
    const float target = fmaxf(1.f, (float)n * cpc);
    const float b = fmaxf(sqrtf(ywid * zspan / target), 0.2f);
    int ny = (int)(ywid / b);
    ny = max(1, min(ny, min(1024, max(1, (int)target))));
    int nz = max(1, min((int)(target / (float)ny), 1 << 22));
    g.ylo = -yh;
    g.zlo = z0;
    g.inv_by = (float)ny / ywid;
    g.inv_bz = (float)nz / zspan;
    g.ny = ny;
    g.nz = nz;
    g.ncell = ny * nz;
  }
  sg[s] = g;
  ncell[s] = g.ncell;
}

// the slot's first global cell index, once the cell counts are scanned
__global__ void k_slot_cellbase(SlotGrid* sg, const int32_t* cell_base, int32_t s0, int32_t s1) {
  const int32_t s = s0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (s < s1) sg[s].cbase = cell_base[s];
}

// Clusters in slot order: each valid cluster's {y, z, input index} goes to
// slot_off[slot] + its rank in the slot (the input of the per-slot cell sort).  Blocks
// take the count's tiles, so the clusters that one count block ranked in a slot (one
// contiguous run of destinations) are written by one block, whose L2 joins the run's
// lines before they go out.
__global__ __launch_bounds__(kCountThreads) void k_slot_scatter(In in, Bound lo_b, Bound hi_b,
                                                                 const int32_t* ckey, const int32_t* srank,
                                                                 const int32_t* slot_off, int4* srec) {
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int64_t base = (int64_t)lo + (int64_t)blockIdx.x * kCountTile;
#pragma unroll
  for (int q = 0; q < kCountTile / kCountThreads; ++q) {
    const int64_t i = base + q * kCountThreads + threadIdx.x;
    if (i >= hi) break;
    const int32_t slot = ckey[i];
    if (slot < 0) continue;
    const int32_t p = slot_off[slot] + srank[i];
    srec[p] = make_int4(__float_as_int(in.y[i]), __float_as_int(in.z[i]), (int32_t)i, 0);
  }
}

// Counting sort of one slot's clusters by cell, one workgroup per slot, in LDS.  The
// slot's cells are taken in ranges of kSortWords counters; each range is counted, turned
// into offsets within the slot (continuing over the ranges) and its clusters placed.
// Counters are 16 bits wide, two per word, when the slot holds fewer than 2^16 clusters
// (no count or offset within the slot reaches that, so a low half never carries into its
// high half), 32 bits otherwise.  Loads are batched kSortBatch per thread ahead of the
// LDS atomics.  Each placed cluster is written twice in grid order: the 16-byte record
// and its position alone.  A slot of up to kSortPerm clusters places only its slot-order
// index in LDS and then writes both arrays in one coalesced pass (random placements
// straight into HBM leave partly written lines: twice the bytes); larger slots write
// each cluster where the counter puts it.
constexpr int kSortThreads = 512;
constexpr int kSortWords = 4096;
constexpr int kSortPerm = 8192;
constexpr int kSortBatch = 2;
static_assert(kSortWords % (4 * kSortThreads) == 0, "offset passes read 4 words per thread");
struct SlotSort {
  const int4* srec;  // {y, z, input index, unused}, slot order
  int32_t* cell_off;
  GHit* gh;
  float2* gyz;
};
__device__ __forceinline__ float2 srec_yz(const int4* r) { return *reinterpret_cast<const float2*>(r); }

__device__ __forceinline__ int slot_cell(const SlotGrid& g, float2 v) {
  return cell_of(v.y, g.zlo, g.inv_bz, g.nz) * g.ny + cell_of(v.x, g.ylo, g.inv_by, g.ny);
}

template <bool kWide, bool kStage>
__device__ void sort_slot(const SlotSort& S, const SlotGrid& g, int32_t slot, int32_t n, int32_t base,
                          uint32_t* cnt, uint16_t* perm, int* lds) {
  constexpr int kPer = kWide ? 1 : 2;  // counters per word
  constexpr int kRange = kSortWords * kPer;
  constexpr uint32_t kMask = kWide ? 0xFFFFFFFFu : 0xFFFFu;
  int carry = 0;
  for (int r0 = 0; r0 < g.ncell; r0 += kRange) {
    const int nc = min(kRange, g.ncell - r0);
    const int nw = (nc + kPer - 1) / kPer;
    for (int w = threadIdx.x; w < nw; w += kSortThreads) cnt[w] = 0u;
    __syncthreads();
    for (int p0 = 0; p0 < n; p0 += kSortThreads * kSortBatch) {
      int c[kSortBatch];
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) {
        const int p = p0 + k * kSortThreads + threadIdx.x;
        c[k] = p < n ? slot_cell(g, srec_yz(S.srec + base + p)) - r0 : -1;
      }
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k)
        if ((unsigned)c[k] < (unsigned)nc) atomicAdd(&cnt[c[k] / kPer], 1u << ((c[k] % kPer) * 16));
    }
    __syncthreads();
    // offsets, 4 words per thread and pass (w + 3 < kSortWords always: kSortWords is a
    // multiple of 4 kSortThreads)
    for (int w0 = 0; w0 < nw; w0 += kSortThreads * 4) {
      const int w = w0 + threadIdx.x * 4;
      const uint4 q = *reinterpret_cast<const uint4*>(cnt + w);
      const uint32_t v[4] = {q.x, q.y, q.z, q.w};
      int sum = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (w + k < nw) sum += kWide ? (int)v[k] : (int)((v[k] & kMask) + (v[k] >> 16));
      int total;
      int e = carry + block_excl_scan(sum, lds, total);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (w + k >= nw) break;
        const int c = r0 + kPer * (w + k);
        const int a = e;
        e += (int)(v[k] & kMask);
        S.cell_off[g.cbase + c] = base + a;
        if (kWide) {
          cnt[w + k] = (uint32_t)a;
        } else {
          const int b = e;
          e += (int)(v[k] >> 16);
          cnt[w + k] = (uint32_t)a | ((uint32_t)b << 16);
          if (c + 1 < r0 + nc) S.cell_off[g.cbase + c + 1] = base + b;
        }
      }
      carry += total;
    }
    __syncthreads();
    for (int p0 = 0; p0 < n; p0 += kSortThreads * kSortBatch) {
      int4 v[kSortBatch];
      int c[kSortBatch];
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) {
        const int p = p0 + k * kSortThreads + threadIdx.x;
        c[k] = -1;
        if (p < n) {
          v[k] = S.srec[base + p];
          c[k] = slot_cell(g, make_float2(__int_as_float(v[k].x), __int_as_float(v[k].y))) - r0;
        }
      }
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) {
        if ((unsigned)c[k] >= (unsigned)nc) continue;
        const uint32_t sh = (uint32_t)(c[k] % kPer) * 16;
        const uint32_t old = atomicAdd(&cnt[c[k] / kPer], 1u << sh);
        const int32_t q = (int32_t)((old >> sh) & kMask);
        if (kStage) {
          perm[q] = (uint16_t)(p0 + k * kSortThreads + threadIdx.x);
        } else {
          const float y = __int_as_float(v[k].x), z = __int_as_float(v[k].y);
          sth(S.gh + base + q, y, z, slot, v[k].z);
          S.gyz[base + q] = make_float2(y, z);
        }
      }
    }
    __syncthreads();
  }
  if (kStage) {
    for (int q0 = 0; q0 < n; q0 += kSortThreads * kSortBatch) {
      int4 v[kSortBatch];
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) {
        const int q = q0 + k * kSortThreads + threadIdx.x;
        if (q < n) v[k] = S.srec[base + perm[q]];
      }
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) {
        const int q = q0 + k * kSortThreads + threadIdx.x;
        if (q >= n) break;
        const float y = __int_as_float(v[k].x), z = __int_as_float(v[k].y);
        sth(S.gh + base + q, y, z, slot, v[k].z);
        S.gyz[base + q] = make_float2(y, z);
      }
    }
    __syncthreads();
  }
}

// Workgroups take the non-empty slots of the list in turn; the cell offsets end with
// the total at the range's last cell.
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_cell_sort(
    SlotSort S, const int32_t* slot_list, const int32_t* slot_cnt, const int32_t* slot_off, const SlotGrid* sg,
    const int32_t* cell_base, int32_t s1) {
  __shared__ __align__(16) uint32_t cnt[kSortWords];
  __shared__ uint16_t perm[kSortPerm];
  __shared__ int lds[40];
  const int32_t n_list = slot_list[kListCount];
  for (int32_t k = blockIdx.x; k < n_list; k += gridDim.x) {
    const int32_t s = slot_list[kListFirst + k];
    const int32_t n = slot_cnt[s];
    const SlotGrid g = sg[s];
    const int32_t base = slot_off[s];
    if (n <= kSortPerm) sort_slot<false, true>(S, g, s, n, base, cnt, perm, lds);
    else if (n < 65536) sort_slot<false, false>(S, g, s, n, base, cnt, perm, lds);
    else sort_slot<true, false>(S, g, s, n, base, cnt, perm, lds);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) S.cell_off[cell_base[s1]] = slot_off[s1];
}

// ------------------------------------------------------------------ a2: neighbours
struct GridView {
  const GHit* gh;
  const SlotGrid* sg;
  const int32_t* cell_base;
  const int32_t* cell_off;
  const float2* yz;  // positions alone, grid order (8 bytes per cluster)
};

// For each cluster h (grid order): over delta = 1, then 2, the pair (d on row r-delta,
// u on row r+delta) with the smallest second difference inside the windows; ties go to
// the smaller input index of u, then of d.
constexpr int kLinkBatch = 2;
__device__ __forceinline__ void link_search(const GridView& G, int32_t slot, float yh, float zh,
                                            const Consts& k, int32_t& bu_out, int32_t& bd_out) {
  const int r = slot % kRows;
  const float y2 = yh + yh, z2 = zh + zh;
  const float m = 0.01f;
  int32_t bu = -1, bd = -1;
  // until a pair is found, best is the float just above the cut, so that "sc < best" alone
  // admits exactly the pairs within the cut (sc <= cut2; cut2 is a normal float)
  float best = k.cut2_above;
  for (int d = 1; d <= 2; ++d) {
    if (r - d < 0 || r + d >= kRows) break;
    const float dxu = k.x[r + d] - k.x[r];
    const float wy = k.win_dy_slope * dxu + k.win_dy_const;
    const float wz = k.win_dz_slope * dxu + k.win_dz_const;
    const float rho = div_rn(k.x[r + d], k.x[r]);
    const float yc = yh * rho;
    const int32_t su = slot + d, sd = slot - d;
    const SlotGrid gu = G.sg[su];
    const SlotGrid gd = G.sg[sd];
    if (gu.ncell == 0 || gd.ncell == 0) continue;
    const int32_t ubase = gu.cbase, dbase = gd.cbase;
    const int uy0 = cell_of(yc - wy - m, gu.ylo, gu.inv_by, gu.ny);
    const int uy1 = cell_of(yc + wy + m, gu.ylo, gu.inv_by, gu.ny);
    const int uz0 = cell_of(zh - wz - m, gu.zlo, gu.inv_bz, gu.nz);
    const int uz1 = cell_of(zh + wz + m, gu.zlo, gu.inv_bz, gu.nz);
    const int uzc = cell_of(zh, gu.zlo, gu.inv_bz, gu.nz);
    // Search radius of the down box: link_cut, shrunk to sqrt(best score) once a pair
    // is known.  A down cluster outside [p - r - m, p + r + m] has |ry| or |rz| > r, so
    // its score exceeds the best one and it cannot win (ties need an equal score).
    float rad = k.link_cut;
    const int maxd = max(uzc - uz0, uz1 - uzc);
    for (int q = 0; q <= 2 * maxd; ++q) {
      // cell rows in z from the window centre outwards (offsets 0, +1, -1, +2, -2, ...):
      // good pairs come early and shrink the boxes of the later candidates
      const int cz = uzc + ((q & 1) ? ((q + 1) >> 1) : -(q >> 1));
      if (cz < uz0 || cz > uz1) continue;
      const int32_t c0 = ubase + cz * gu.ny;
      const int32_t a0 = G.cell_off[c0 + uy0], a1 = G.cell_off[c0 + uy1 + 1];
      // candidates are read kLinkBatch at a time (positions only; input indices are read
      // for exact ties alone), so one memory wait serves several of them; wider batches
      // measured slower (the kernel is VALU-issue bound, and the predication costs VALU)
      for (int32_t ub = a0; ub < a1; ub += kLinkBatch) {
        float2 U[kLinkBatch];
#pragma unroll
        for (int i = 0; i < kLinkBatch; ++i) U[i] = ub + i < a1 ? G.yz[ub + i] : make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < kLinkBatch; ++i) {
          const int32_t u = ub + i;
          if (u >= a1) break;
          const float yu = U[i].x, zu = U[i].y;
          if (!(fabsf(yu - yc) <= wy) || !(fabsf(zu - zh) <= wz)) continue;
          const float py = y2 - yu, pz = z2 - zu;
          const int dy0 = cell_of(py - rad - m, gd.ylo, gd.inv_by, gd.ny);
          const int dy1 = cell_of(py + rad + m, gd.ylo, gd.inv_by, gd.ny);
          const int dz0 = cell_of(pz - rad - m, gd.zlo, gd.inv_bz, gd.nz);
          const int dz1 = cell_of(pz + rad + m, gd.zlo, gd.inv_bz, gd.nz);
          for (int ez0 = dz0; ez0 <= dz1; ez0 += kLinkBatch) {
            // the candidate ranges of up to kLinkBatch down cell rows at once
            int32_t B0[kLinkBatch], B1[kLinkBatch];
#pragma unroll
            for (int e = 0; e < kLinkBatch; ++e) {
              B0[e] = B1[e] = 0;
              if (ez0 + e <= dz1) {
                const int32_t e0 = dbase + (ez0 + e) * gd.ny;
                B0[e] = G.cell_off[e0 + dy0];
                B1[e] = G.cell_off[e0 + dy1 + 1];
              }
            }
#pragma unroll
            for (int e = 0; e < kLinkBatch; ++e) {
              for (int32_t db0 = B0[e]; db0 < B1[e]; db0 += kLinkBatch) {
                float2 D[kLinkBatch];
#pragma unroll
                for (int j = 0; j < kLinkBatch; ++j)  // past the range: a position whose score is inf
                  D[j] = db0 + j < B1[e] ? G.yz[db0 + j] : make_float2(__builtin_inff(), __builtin_inff());
#pragma unroll
                for (int j = 0; j < kLinkBatch; ++j) {
                  const int32_t dd = db0 + j;
                  const float ry = (yu + D[j].x) - y2;
                  const float rz = (zu + D[j].y) - z2;
                  const float sc = ry * ry + rz * rz;
                  // the best pair is kept with selects; only an equal score takes a branch (an
                  // exact tie, or before any pair a score just above the cut)
                  bool win = sc < best;
                  if (sc == best) {
                    if (bu >= 0) {
                      const int32_t uo = G.gh[u].idx, bo = G.gh[bu].idx;
                      win = uo < bo || (uo == bo && G.gh[dd].idx < G.gh[bd].idx);
                    }
                  }
                  best = win ? sc : best;
                  bu = win ? u : bu;
                  bd = win ? dd : bd;
                }
              }
            }
          }
          // (the radius only prunes, so the hardware square root, within a few ulp, does;
          // the 1e-4 margin keeps it above sqrt(best))
          if (bu >= 0) rad = fminf(k.link_cut, __builtin_amdgcn_sqrtf(best) * 1.0001f);
        }
      }
    }
    if (bu >= 0) break;
  }
  bu_out = bu;
  bd_out = bd;
}

// One lane per cluster.  Links are stored in grid order.
__global__ __launch_bounds__(256) void k_links(GridView G, Bound lo_b, Bound hi_b, int32_t* up_raw,
                                               int32_t* dn_raw, Consts k) {
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int32_t h = lo + (int32_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (h >= hi) return;
  const GHit Hh = ldh(G.gh + h);
  int32_t bu, bd;
  link_search(G, Hh.slot, Hh.y, Hh.z, k, bu, bd);
  up_raw[h] = bu;
  dn_raw[h] = bd;
}


// Cleaning and starts in one pass: the clean links of h, and whether h starts a chain
// (no clean down link, a clean up link whose own clean up link exists; the latter is
// evaluated from the raw links too), flagged at h's input index and, for the grid-ordered
// work list, at h itself.  Also clears h's hit weight for the tracklet stage.
__global__ void k_clean_starts(const int32_t* up_raw, const int32_t* dn_raw, const GHit* gh, int32_t* up,
                               int32_t* dn, uint8_t* flag, uint8_t* flagg, uint32_t* hitw, Bound lo_b,
                               Bound hi_b) {
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int32_t h = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= hi) return;
  const int32_t u = up_raw[h], d = dn_raw[h];
  const int32_t uc = (u >= 0 && dn_raw[u] == h) ? u : -1;
  const int32_t dc = (d >= 0 && up_raw[d] == h) ? d : -1;
  up[h] = uc;
  dn[h] = dc;
  bool start = false;
  if (dc < 0 && uc >= 0) {
    const int32_t u2 = up_raw[uc];
    start = u2 >= 0 && dn_raw[u2] == uc;
  }
  if (start) flag[gh[h].idx] = 1u;
  if (flagg) flagg[h] = start ? 1u : 0u;
  hitw[h] = 0u;
}

__global__ void k_job_offsets(const int32_t* scanned, const int32_t* job_off, int32_t* out_off,
                              int32_t j0, int32_t j1, int32_t cap) {
  const int32_t j = j0 + 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > j1) return;
  out_off[j] = scanned[min(job_off[j], cap)];
}


// start[t] = grid index of tracklet t's start; order[p] = id of the p-th start in grid order.
// When the starts up to this batch's end (thi) exceed the capacity, ids and positions below
// capT no longer pair up, so order[] becomes the identity: every kept id is then built.
// Starts are read from the grid-order flags when there are any (one byte per cluster),
// else tested on the clean links.
__global__ void k_write_starts(const int32_t* up, const int32_t* dn, const uint8_t* flagg, const GHit* gh,
                               const int32_t* fid, const int32_t* posg, const int32_t* T_off, int32_t* start,
                               int32_t* order, int32_t capT, Bound lo_b, Bound hi_b, Bound thi_b,
                               int32_t* counters) {
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int32_t h = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= hi) return;
  if (flagg) {
    if (!flagg[h]) return;
  } else {
    const int32_t u = up[h];
    if (!(dn[h] < 0 && u >= 0 && up[u] >= 0)) return;
  }
  const GHit H = ldh(gh + h);
  const int32_t t = fid[H.idx];
  if (t < capT) start[t] = h;
  else atomicOr(&counters[kCntStatus], kStatusCapacity);
  // the 32-bit hit-weight key holds a job-local tracklet id of 24 bits
  if (t - T_off[H.slot / kSlotsPerJob] > kLocalIdMax) atomicOr(&counters[kCntStatus], kStatusCapacity);
  if (order) {
    const int32_t p = posg[h];
    if (p < capT) order[p] = thi_b.get() > capT ? p : t;
  }
}

// ------------------------------------------------------------------ a4: tracklets
struct TrackletView {
  const int32_t* start;
  const int32_t* up_raw;
  const int32_t* dn_raw;
  const int32_t* up;
  int32_t* hits;      // [capT][kHitStride]: the hits of a tracklet are contiguous
  int32_t* nhits;     // [capT]
  float* state;       // [capT][kStateStride]: P[5], C[15], x
  uint32_t* hitw;     // [N] grid order: max key over the tracklets that took the cluster
  const int32_t* T_off;  // [J+1] first tracklet id of each job
  int32_t capT;
};

// Hit-weight key of a tracklet: (n_hits << 24) | (2^24-1 - job-local id).  Within one
// job (the only tracklets that can share a cluster) it orders like the 64-bit key
// (n_hits << 32) | (2^32-1 - id), since local ids and global ids differ by the job's
// first id.  0 when the local id does not fit in 24 bits (reported at the starts).
__device__ __forceinline__ uint32_t trk_key(const TrackletView& V, int32_t slot_base, int32_t t, int n) {
  const int32_t local = t - V.T_off[slot_base / kSlotsPerJob];
  if (local < 0 || local > kLocalIdMax) return 0u;
  return ((uint32_t)n << 24) | (uint32_t)(kLocalIdMax - local);
}
__device__ __forceinline__ int32_t key_tracklet(uint32_t key, const int32_t* T_off, int32_t slot) {
  return T_off[slot / kSlotsPerJob] + (kLocalIdMax - (int32_t)(key & (uint32_t)kLocalIdMax));
}

__device__ __forceinline__ void init_cov(State& S, const float* prior) {
#pragma unroll
  for (int i = 0; i < 15; ++i) S.C[i] = 0.f;
  S.C[tri(0, 0)] = prior[0];
  S.C[tri(1, 1)] = prior[1];
  S.C[tri(2, 2)] = prior[2];
  S.C[tri(3, 3)] = prior[3];
  S.C[tri(4, 4)] = prior[4];
}

// One lane per tracklet: Kalman filter along the chain (every chain cluster used),
// then following on the rows above (minimum chi2 in a 3-sigma window).  The tracklet
// runs as a step machine: a step propagates to the next plane (the next chain
// cluster's row, or the next row when following), picks the cluster (the chain link,
// or the window search) and updates.  Propagation and update are one code path for
// both phases, so the lanes of a wave in different phases do not diverge there.
// Each lane has 37 words of dynamic LDS (37 is odd, so the lanes of a wave hit distinct
// banks): the state recorded at the last accepted cluster (5 parameters, 15 covariance
// terms, x), which frees 21 registers, and a ring of the last 16 accepted hits, written
// to HBM as one full 64-byte line per 16 hits instead of one partial line per hit.
constexpr int kKeepWords = 21;
constexpr int kRingWords = 16;
constexpr int kLaneWords = kKeepWords + kRingWords;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) int32_t lds_i32;

struct TrkLane {
  State S;
  float x;
  lds_f32* keep;  // this lane's recorded state (21 words of LDS)
  lds_i32* ring;  // and its last kRingWords hits
  int32_t t, h, first, cur, slot_base;
  int n, last_row, r, misses, phase;  // phase 1: chain, 2: following
};

// Writes the first `cnt` ring words (the hits cnt..1 back from the n-th) to the
// tracklet's hit list: whole 16-byte stores when a full ring is flushed.
__device__ __forceinline__ void flush_ring(const TrackletView& V, const TrkLane& T, int cnt) {
  if (cnt == 0) return;
  const int base = (T.n - 1) & ~(kRingWords - 1);  // hit index of ring word 0
  int32_t* dst = V.hits + (int64_t)T.t * kHitStride + base;
  if (cnt == kRingWords) {
#pragma unroll
    for (int i = 0; i < kRingWords; i += 4)
      *reinterpret_cast<int4*>(dst + i) = make_int4(T.ring[i], T.ring[i + 1], T.ring[i + 2], T.ring[i + 3]);
  } else {
    for (int i = 0; i < cnt; ++i) dst[i] = T.ring[i];
  }
}

__device__ __forceinline__ void keep_state(TrkLane& T) {
#pragma unroll
  for (int i = 0; i < 5; ++i) T.keep[i] = T.S.P[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) T.keep[5 + i] = T.S.C[i];
  T.keep[20] = T.x;
}

__device__ __forceinline__ void trk_begin(const GridView& G, const TrackletView& V, TrkLane& T, int32_t t,
                                          const Consts& k) {
  T.t = t;
  T.h = V.start[t];
  const int32_t dr = V.dn_raw[T.h];
  T.first = (dr >= 0 && V.up_raw[dr] < 0) ? dr : T.h;
  const int32_t c1 = (T.first != T.h) ? T.h : V.up[T.first];
  const int32_t c2 = (c1 == T.first && T.first != T.h) ? T.h : V.up[c1];
  const GHit F0 = ldh(G.gh + T.first);
  const GHit F2 = ldh(G.gh + c2);
  const int r0 = F0.slot % kRows;
  T.slot_base = F0.slot - r0;
  const float dx2 = k.x[F2.slot % kRows] - k.x[r0];
  const float dy2 = F2.y - F0.y;
  const float dz2 = F2.z - F0.z;
  const float den = sqrt_rn(dx2 * dx2 + dy2 * dy2);
  T.S.P[0] = F0.y;
  T.S.P[1] = F0.z;
  T.S.P[2] = div_rn(dy2, den);
  T.S.P[3] = div_rn(dz2, den);
  T.S.P[4] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) T.S.L[i] = 0.f;
  init_cov(T.S, k.prior0);
  T.x = k.x[r0];
  keep_state(T);  // the recorded state is the initial one until a cluster is accepted
  T.n = 0;
  T.last_row = r0;
  T.cur = T.first;
  T.phase = 1;
  T.r = 0;
  T.misses = 0;
}

// The following's window search: the cluster of minimum chi2 inside the window
// |y - y_pred| <= wy, |z - z_pred| <= wz (ties: the smaller input index) among those
// `eligible` accepts, which is asked only about a candidate that would win.  The candidate
// ranges of two cell rows are read at a time, then their positions four at a time, so one
// memory wait serves several of them (rows of 1-4 and batches of 2-8 were measured: 2 and 4
// gave the shortest tracklet stage); the scan order, rows then cells, is unchanged.
constexpr int kFollowRows = 2;
constexpr int kFollowBatch = 4;
template <class Eligible>
__device__ __forceinline__ void window_best(const GridView& G, const SlotGrid& g, const State& S, const SInv& si,
                                            float wy, float wz, Eligible eligible, int32_t& cand, float& bchi,
                                            float& cy, float& cz) {
  if (g.ncell <= 0) return;
  const int32_t cb0 = g.cbase;
  const int y0c = cell_of(S.P[0] - wy - 0.01f, g.ylo, g.inv_by, g.ny);
  const int y1c = cell_of(S.P[0] + wy + 0.01f, g.ylo, g.inv_by, g.ny);
  const int z0c = cell_of(S.P[1] - wz - 0.01f, g.zlo, g.inv_bz, g.nz);
  const int z1c = cell_of(S.P[1] + wz + 0.01f, g.zlo, g.inv_bz, g.nz);
  for (int zc = z0c; zc <= z1c; zc += kFollowRows) {
    int32_t A0[kFollowRows], A1[kFollowRows];
#pragma unroll
    for (int e = 0; e < kFollowRows; ++e) {
      A0[e] = A1[e] = 0;
      if (zc + e <= z1c) {
        const int32_t e0 = cb0 + (zc + e) * g.ny;
        A0[e] = G.cell_off[e0 + y0c];
        A1[e] = G.cell_off[e0 + y1c + 1];
      }
    }
#pragma unroll
    for (int e = 0; e < kFollowRows; ++e) {
      for (int32_t c0 = A0[e]; c0 < A1[e]; c0 += kFollowBatch) {
        float2 Cb[kFollowBatch];
#pragma unroll
        for (int i = 0; i < kFollowBatch; ++i) Cb[i] = c0 + i < A1[e] ? G.yz[c0 + i] : make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < kFollowBatch; ++i) {
          const int32_t c = c0 + i;
          if (c >= A1[e]) break;
          const float rr0 = (Cb[i].x - S.P[0]) - S.L[0];
          const float rr1 = (Cb[i].y - S.P[1]) - S.L[1];
          if (!(fabsf(rr0) <= wy) || !(fabsf(rr1) <= wz)) continue;
          const float chi2 = chi2_of(si, rr0, rr1);
          // equal chi2: the smaller input index wins (read only for such ties)
          if (!(cand < 0 || chi2 < bchi || (chi2 == bchi && G.gh[c].idx < G.gh[cand].idx))) continue;
          if (!eligible(c)) continue;
          cand = c;
          bchi = chi2;
          cy = Cb[i].x;
          cz = Cb[i].y;
        }
      }
    }
  }
}

// One step; returns true when the tracklet has ended.
__device__ __forceinline__ bool trk_step(const GridView& G, const TrackletView& V, TrkLane& T,
                                         const Consts& k) {
  const bool chain = T.phase == 1;
  int row;
  float cy = 0.f, cz = 0.f;
  int32_t cand = -1;
  int32_t up_next = -1;
  if (chain) {
    // the chain's next link is read with the cluster, not after the update
    up_next = V.up[T.cur];
    const GHit Hc = ldh(G.gh + T.cur);
    row = Hc.slot % kRows;
    cy = Hc.y;
    cz = Hc.z;
    cand = T.cur;
  } else {
    row = T.r;
  }
  // the row's grid geometry is loaded before the transport, which hides its latency
  SlotGrid g{};
  if (!chain) g = G.sg[T.slot_base + row];
  const float xt = k.x[row];
  if (!propagate(T.S, T.x, xt, k)) return true;
  T.x = xt;
  bool take = chain;
  if (!chain) {
    const SInv si = s_inverse(T.S.C, k.vy, k.vz);
    if (!si.ok) return true;
    const float wy = k.nwin * sqrt_rn(T.S.C[0] + k.vy);
    const float wz = k.nwin * sqrt_rn(T.S.C[2] + k.vz);
    float bchi = 0.f;
    window_best(G, g, T.S, si, wy, wz, [](int32_t) { return true; }, cand, bchi, cy, cz);
    take = cand >= 0 && bchi <= k.chi2_follow;
  }
  if (take) {
    if (!kf_update(T.S, cy, cz, k, nullptr)) return true;
    T.ring[T.n & (kRingWords - 1)] = cand;
    ++T.n;
    if ((T.n & (kRingWords - 1)) == 0) flush_ring(V, T, kRingWords);
    keep_state(T);
    if (chain) {
      T.last_row = row;
      T.cur = (T.cur == T.first && T.first != T.h) ? T.h : up_next;
      if (T.cur < 0) {
        T.phase = 2;
        T.r = T.last_row + 1;
        T.misses = 0;
        return T.r >= kRows;
      }
      return false;
    }
    T.misses = 0;
  } else if (++T.misses >= k.max_miss) {
    return true;
  }
  return ++T.r >= kRows;
}

__device__ __forceinline__ void trk_finish(const TrackletView& V, const TrkLane& T, const Consts& k) {
  const int32_t t = T.t;
  V.nhits[t] = T.n;
  float* st = V.state + (int64_t)t * kStateStride;
#pragma unroll
  for (int i = 0; i < 20; i += 4)
    *reinterpret_cast<float4*>(st + i) = make_float4(T.keep[i], T.keep[i + 1], T.keep[i + 2], T.keep[i + 3]);
  st[20] = T.keep[20];
  flush_ring(V, T, T.n & (kRingWords - 1));
  const uint32_t key = trk_key(V, T.slot_base, t, T.n);
  st[21] = __uint_as_float(key);
  if (T.n >= k.min_hits && key != 0u) {
    for (int q = 0; q < T.n; ++q) atomicMax(&V.hitw[V.hits[(int64_t)t * kHitStride + q]], key);
  }
}

extern __shared__ float trk_keep[];
__device__ __forceinline__ void lane_lds(TrkLane& T) {
  T.keep = (lds_f32*)&trk_keep[threadIdx.x * kLaneWords];
  T.ring = (lds_i32*)&trk_keep[threadIdx.x * kLaneWords + kKeepWords];
}

__device__ __forceinline__ void build_tracklet(const GridView& G, const TrackletView& V, int32_t t,
                                               const Consts& k) {
  TrkLane T;
  lane_lds(T);
  trk_begin(G, V, T, t, k);
  while (!trk_step(G, V, T, k)) {
  }
  trk_finish(V, T, k);
}

// Lanes take tracklets in the grid order of their start clusters (order[]), so the
// lanes of a wave follow neighbouring tracks through the same cells.
__global__ __launch_bounds__(256) void k_tracklets(GridView G, TrackletView V, const int32_t* order,
                                                   Bound lo_b, Bound hi_b, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), V.capT);
  const int32_t p = lo + (int32_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (p >= hi) return;
  const int32_t t = order ? order[p] : p;
  if (t >= 0 && t < V.capT) build_tracklet(G, V, t, k);
}

// Persistent variant with lane refill.  The grid-ordered work list is cut into one
// contiguous range per XCD; each lane runs its tracklet as a step machine (one step =
// one chain cluster or one following row, the same operations in the same order as
// build_tracklet), and a lane whose tracklet has ended takes the next one: lanes that
// need work are counted with a ballot and served by one atomicAdd per wave on the
// ticket of the current range, then of the other ranges (stealing).  The wave exits
// when every range is exhausted and no lane holds a tracklet.
__global__ __launch_bounds__(256) void k_tracklets_persistent(GridView G, TrackletView V,
                                                              const int32_t* order, Bound lo_b,
                                                              Bound hi_b, Consts k, int32_t* ticket) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), V.capT);
  const int32_t nwork = hi > lo ? hi - lo : 0;
  const int32_t per = (nwork + kXcds - 1) / kXcds;
  const int lane = threadIdx.x & 63;
  const int x0 = blockIdx.x % kXcds;
  int qi = 0;  // ranges exhausted so far (wave-uniform)
  bool active = false;
  TrkLane T;
  lane_lds(T);
  for (;;) {
    // refill the lanes without a tracklet: one atomicAdd per wave and range
    while (qi < kXcds) {
      const uint64_t need = __ballot(!active);
      if (need == 0) break;
      const int cnt = __popcll(need);
      const int xr = (x0 + qi) % kXcds;
      const int32_t a = lo + xr * per;
      const int32_t b = min(hi, a + per);
      int32_t base = 0;
      if (lane == 0) base = atomicAdd(&ticket[xr], cnt);
      base = __shfl(base, 0, 64);
      const int rank = __popcll(need & ((1ull << lane) - 1ull));
      if (!active) {
        const int32_t p = a + base + rank;
        if (p < b) {
          const int32_t tt = order ? order[p] : p;
          if (tt >= 0 && tt < V.capT) {
            trk_begin(G, V, T, tt, k);
            active = true;
          }
        }
      }
      if (base + cnt >= b - a) ++qi;
    }
    if (!__any(active)) break;
    if (active && trk_step(G, V, T, k)) {
      trk_finish(V, T, k);
      active = false;
    }
  }
}

// Persistent variant without refill: a wave takes 64 consecutive tracklets of its
// XCD's range per ticket (one per lane), runs them to the end, then takes the next
// 64; exhausted ranges are followed by the other XCDs' ranges.
__global__ __launch_bounds__(256) void k_tracklets_chunked(
    GridView G, TrackletView V, const int32_t* order,
                                                           Bound lo_b, Bound hi_b, Consts k, int32_t* ticket) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), V.capT);
  const int32_t nwork = hi > lo ? hi - lo : 0;
  const int32_t per = (nwork + kXcds - 1) / kXcds;
  const int lane = threadIdx.x & 63;
  const int x0 = blockIdx.x % kXcds;
  int qi = 0;
  while (qi < kXcds) {
    const int xr = (x0 + qi) % kXcds;
    const int32_t a = lo + xr * per;
    const int32_t b = min(hi, a + per);
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&ticket[xr], 64);
    base = __shfl(base, 0, 64);
    if (a + base >= b) {
      ++qi;
      continue;
    }
    const int32_t p = a + base + lane;
    const int32_t tt = p < b ? (order ? order[p] : p) : -1;
    if (tt >= 0 && tt < V.capT) build_tracklet(G, V, tt, k);
  }
}

// ------------------------------------------------------------------ a5: selection
// Owned-hit counts from one coalesced pass over the clusters in grid order: a cluster's
// weight is the key of the tracklet that owns it, whose low 24 bits are 2^24-1 - its id
// within the job.  A block takes kOwnChunk consecutive grid positions (small enough that
// few chunks straddle a job boundary, large enough that few tracklets are split between
// chunks).  When they all belong to one job of at most kOwnLocal tracklets, it counts them
// in LDS (8-bit counters, four to a word: a tracklet holds fewer than 256 clusters) and adds
// each non-zero count with one atomic; otherwise every owned cluster adds its own.
constexpr int kOwnThreads = 1024;
constexpr int kOwnChunk = 16384;
constexpr int kOwnLocal = 65536;
constexpr int kOwnBatch = 4;
static_assert(kHitStride < 256, "8-bit ownership counters");
__global__ __launch_bounds__(kOwnThreads) void k_own_count(const uint32_t* hitw, const GHit* gh,
                                                           const int32_t* T_off, const int32_t* slot_off,
                                                           int32_t* own, int32_t j0, int32_t j1, Bound lo_b,
                                                           Bound hi_b, int32_t capT) {
  __shared__ uint32_t cnt[kOwnLocal / 4];
  __shared__ int32_t s_job;
  const int32_t lo = lo_b.get(), hi = hi_b.get();
  const int64_t a = (int64_t)lo + (int64_t)blockIdx.x * kOwnChunk;
  if (a >= hi) return;
  const int32_t b = (int32_t)std::min<int64_t>(a + kOwnChunk, hi);
  if (threadIdx.x == 0) {  // the job holding position a: slot_off[j K] <= a < slot_off[(j+1) K]
    int x = j0, y = j1;
    while (y - x > 1) {
      const int m = (x + y) >> 1;
      if (slot_off[(int64_t)m * kSlotsPerJob] <= a) x = m; else y = m;
    }
    s_job = x;
  }
  __syncthreads();
  const int32_t j = s_job;
  const int32_t t0 = T_off[j], ntr = T_off[j + 1] - t0;
  if (slot_off[(int64_t)(j + 1) * kSlotsPerJob] < b || ntr > kOwnLocal) {
    for (int64_t h0 = a; h0 < b; h0 += kOwnThreads * kOwnBatch) {
      uint32_t w[kOwnBatch];
#pragma unroll
      for (int k = 0; k < kOwnBatch; ++k) {
        const int64_t h = h0 + k * kOwnThreads + threadIdx.x;
        w[k] = h < b ? hitw[h] : 0u;
      }
#pragma unroll
      for (int k = 0; k < kOwnBatch; ++k) {
        if (w[k] == 0u) continue;
        const int32_t t = key_tracklet(w[k], T_off, gh[h0 + k * kOwnThreads + threadIdx.x].slot);
        if ((uint32_t)t < (uint32_t)capT) atomicAdd(&own[t], 1);
      }
    }
    return;
  }
  const int nw = (ntr + 3) >> 2;
  for (int q = threadIdx.x; q < nw; q += kOwnThreads) cnt[q] = 0u;
  __syncthreads();
  for (int64_t h0 = a; h0 < b; h0 += kOwnThreads * kOwnBatch) {
    uint32_t w[kOwnBatch];
#pragma unroll
    for (int k = 0; k < kOwnBatch; ++k) {
      const int64_t h = h0 + k * kOwnThreads + threadIdx.x;
      w[k] = h < b ? hitw[h] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kOwnBatch; ++k) {
      if (w[k] == 0u) continue;
      const int32_t id = kLocalIdMax - (int32_t)(w[k] & (uint32_t)kLocalIdMax);
      if ((uint32_t)id < (uint32_t)ntr) atomicAdd(&cnt[id >> 2], 1u << ((id & 3) << 3));
    }
  }
  __syncthreads();
  for (int32_t id = threadIdx.x; id < ntr; id += kOwnThreads) {
    const int32_t c = (int32_t)((cnt[id >> 2] >> ((id & 3) << 3)) & 0xFFu);
    if (c && (uint32_t)(t0 + id) < (uint32_t)capT) atomicAdd(&own[t0 + id], c);
  }
}

__global__ void k_select_count(TrackletView V, Bound lo_b, Bound hi_b, int32_t* own, int32_t* accf,
                               Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), V.capT);
  const int32_t t = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= hi) return;
  const int n = V.nhits[t];
  const int cnt = own[t];
  const bool a = n >= k.min_hits && cnt >= k.min_hits;
  own[t] = a ? cnt : 0;
  accf[t] = a ? 1 : 0;
}

__global__ void k_select_write(TrackletView V, Bound lo_b, Bound hi_b, const int32_t* accf,
                               const int32_t* kid, const int32_t* hoff, int32_t* sel_from,
                               int32_t* sel_off, int32_t capK, int32_t* counters) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), V.capT);
  const int32_t t = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= hi || !accf[t]) return;
  const int32_t kk = kid[t];
  if (kk >= capK) {
    atomicOr(&counters[kCntStatus], kStatusCapacity);
    return;
  }
  sel_from[kk] = t;
  sel_off[kk] = hoff[t];
}

// One wave per selected track: its owned hits, in tracklet order, compacted with a
// ballot per 64 hits (coalesced reads of the hit list, coalesced writes).
__global__ __launch_bounds__(256) void k_select_hits(TrackletView V, const int32_t* kid, int32_t j0, int32_t j1,
                                                     const int32_t* sel_from, const int32_t* sel_off,
                                                     int32_t* sel_hits, int32_t capK, int32_t capH,
                                                     int32_t* counters) {
  // selected tracks of jobs j0..j1-1: [kid[T_off[j0]], kid[T_off[j1]])
  const int32_t lo = kid[min(V.T_off[j0], V.capT)];
  const int32_t hi = min(kid[min(V.T_off[j1], V.capT)], capK);
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w0 = lo + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6); w0 < hi; w0 += nw) {
    const int32_t kk = (int32_t)w0;
    const int32_t t = sel_from[kk];
    const int32_t o = sel_off[kk];
    const int n = V.nhits[t];
    const uint32_t key = __float_as_uint(V.state[(int64_t)t * kStateStride + 21]);
    int w = 0;
    for (int q0 = 0; q0 < n; q0 += 64) {
      const int q = q0 + lane;
      int32_t c = 0;
      bool own = false;
      if (q < n) {
        c = V.hits[(int64_t)t * kHitStride + q];
        own = V.hitw[c] == key;
      }
      const uint64_t m = __ballot(own);
      if (own) {
        const int pos = o + w + __popcll(m & ((1ull << lane) - 1ull));
        if (pos < capH) sel_hits[pos] = c;
      }
      w += __popcll(m);
    }
    if (lane == 0 && o + w > capH) atomicOr(&counters[kCntStatus], kStatusCapacity);
  }
}

__global__ void k_select_finish(const int32_t* kid, const int32_t* hoff, Bound thi_b, int32_t capT,
                                int32_t* sel_off, int32_t capK, int32_t* counters) {
  const int32_t thi = min(thi_b.get(), capT);
  const int32_t K = kid[thi];
  const int32_t H = hoff[thi];
  counters[kCntSelected] = K;
  counters[kCntSelHits] = H;
  if (K <= capK) sel_off[K] = H;
}

// ------------------------------------------------------------------ a6: fit and merge
struct FitView {
  const int32_t* sel_from;
  const int32_t* sel_off;
  const int32_t* sel_hits;
  const int32_t* chain_next;  // merged outer piece of a track, -1 if none (NULL: no merge)
  const int32_t* chain_prev;  // merged inner piece, -1 if none; chains are walked from heads only
  const float* link_t0;       // collision time of a membrane link to the outer piece
  float* row;                 // [capK][kFitStride]: P[5], C[15], x, L[5] (one record per track)
  float* chi2;
  int32_t* ndf;
  int32_t capK;
};

// The fit record of track kk: the state at the innermost hit (with its compensation terms,
// which the downward extension continues from), chi2 and ndf; NaN parameters, zero
// covariance and ndf = -1 when the fit failed.
__device__ __forceinline__ void store_fit(const FitView& F, int32_t kk, const State& S, float x, float chi2,
                                          int nh, bool ok) {
  float v[kFitStride];
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = ok ? S.P[i] : __builtin_nanf("");
#pragma unroll
  for (int i = 0; i < 15; ++i) v[5 + i] = ok ? S.C[i] : 0.f;
  v[20] = ok ? x : 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) v[21 + i] = ok ? S.L[i] : 0.f;
#pragma unroll
  for (int i = 26; i < kFitStride; ++i) v[i] = 0.f;
  float* dst = F.row + (int64_t)kk * kFitStride;
#pragma unroll
  for (int i = 0; i < kFitStride; i += 4)
    *reinterpret_cast<float4*>(dst + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
  F.chi2[kk] = ok ? chi2 : 0.f;
  F.ndf[kk] = ok ? 2 * nh - 5 : -1;
}

__device__ __forceinline__ void load_fit(const FitView& F, int32_t kk, State& S, float& x) {
  const float* src = F.row + (int64_t)kk * kFitStride;
  float v[28];
#pragma unroll
  for (int i = 0; i < 28; i += 4) {
    const float4 q = *reinterpret_cast<const float4*>(src + i);
    v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) S.P[i] = v[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) S.C[i] = v[5 + i];
  x = v[20];
#pragma unroll
  for (int i = 0; i < 5; ++i) S.L[i] = v[21 + i];
}

// Fit of a hit list given as up to 18 consecutive pieces (inner -> outer); crossing a
// piece boundary rotates the state into the inner piece's sector frame.
__device__ void fit_track(const GridView& G, const TrackletView& V, const FitView& F, int32_t kk,
                          const Consts& k) {
  // collect the piece chain (a head and at most kHalf absorbed pieces)
  int32_t pieces[kHalf + 1];
  int np = 0;
  const bool walk = F.chain_next && F.chain_prev[kk] < 0;
  for (int32_t p = kk; p >= 0 && np <= kHalf; p = walk ? F.chain_next[p] : -1) pieces[np++] = p;
  const int32_t last_piece = pieces[np - 1];
  State S;
  float x, chi2;
  int nh, cur_sec, pstart;
  bool ok = true;
  if (np >= 2 && F.ndf[last_piece] >= 0) {
    // A chain's fit starts on its outermost piece exactly as that piece's own fit did (its
    // outermost hit, its tracklet's direction and curvature, the same priors) and runs over
    // the same hits first, so it continues from that piece's stored record (state with its
    // compensation terms, chi2, hit count) instead of refitting them.
    load_fit(F, last_piece, S, x);
    chi2 = F.chi2[last_piece];
    nh = (F.ndf[last_piece] + 5) / 2;
    cur_sec = (G.gh[F.sel_hits[F.sel_off[last_piece]]].slot / kRows) % kSectors;
    pstart = np - 2;
  } else {
    const int32_t tl = F.sel_from[last_piece];
    const int32_t ho = F.sel_hits[F.sel_off[last_piece + 1] - 1];
    const GHit Ho = ldh(G.gh + ho);
    S.P[0] = Ho.y;
    S.P[1] = Ho.z;
    S.P[2] = V.state[(int64_t)tl * kStateStride + 2];
    S.P[3] = V.state[(int64_t)tl * kStateStride + 3];
    S.P[4] = V.state[(int64_t)tl * kStateStride + 4];
#pragma unroll
    for (int i = 0; i < 5; ++i) S.L[i] = 0.f;
    init_cov(S, k.prior1);
    x = k.x[Ho.slot % kRows];
    chi2 = 0.f;
    nh = 0;
    cur_sec = (Ho.slot / kRows) % kSectors;
    pstart = np - 1;
  }
  for (int pi = pstart; pi >= 0 && ok; --pi) {
    const int32_t p = pieces[pi];
    const int32_t a = F.sel_off[p], b = F.sel_off[p + 1];
    // the next hit's record is loaded while the current one is fitted, the index after it one
    // step earlier still
    int32_t hn = b - 2 >= a ? F.sel_hits[b - 2] : 0;
    GHit Hn;
    if (b - 1 >= a) Hn = ldh(G.gh + F.sel_hits[b - 1]);
    for (int32_t q = b - 1; q >= a; --q) {
      const GHit Hq = Hn;
      if (q - 1 >= a) Hn = ldh(G.gh + hn);
      if (q - 2 >= a) hn = F.sel_hits[q - 2];
      const int32_t sl = Hq.slot;
      const int sec = (sl / kRows) % kSectors;
      if (sec != cur_sec) {
        if ((sec < kHalf) != (cur_sec < kHalf)) {
          // across the central membrane into the inner piece's side: z moves by twice the
          // drift of the link's collision time
          const float d = (2.0f * k.v_drift) * F.link_t0[p];
          acc(S.P[1], S.L[1], sec < kHalf ? -d : d);
        } else if (!rotate(S, x, cur_sec, sec, k)) {
          ok = false;
          break;
        }
        cur_sec = sec;
      }
      const float xh = k.x[sl % kRows];
      if (!propagate(S, x, xh, k)) { ok = false; break; }
      x = xh;
      float c2;
      if (!kf_update(S, Hq.y, Hq.z, k, &c2)) { ok = false; break; }
      chi2 = chi2 + c2;
      ++nh;
    }
  }
  store_fit(F, kk, S, x, chi2, nh, ok);
}

__global__ __launch_bounds__(256) void k_fit(GridView G, TrackletView V, FitView F, Bound lo_b,
                                             Bound hi_b, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  fit_track(G, V, F, kk, k);
}

// Refit of the merged chain heads only.
__global__ __launch_bounds__(256) void k_fit_heads(GridView G, TrackletView V, FitView F,
                                                   const int32_t* head_list, const int32_t* n_heads,
                                                   Consts k) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_heads) return;
  fit_track(G, V, F, head_list[i], k);
}

// ------------------------------------------------------------------ downward extension
// A track's chain need not start at its first row (a cluster lost to inefficiency or a
// link lost in a dense neighbourhood breaks it), and the following visits only the rows
// above the chain (reading A13).  Every track whose fit succeeded therefore continues
// below its innermost hit: from the fitted state there, row by row inwards in its sector,
// with the following's window, minimum chi2 (ties: smaller input index), chi2 cut and
// miss limit, taking only clusters that no selected track owns.  A cluster found by
// several tracks goes to the one with more owned hits, then the smaller track id (a
// 32-bit max key, as for the tracklets: (owned hits << 24) | (2^24-1 - job-local track
// id)); a track keeps its found hits up to the first one it lost.  The kept hits go in
// front of the track's hits and its fit continues over them from the stored state, which
// equals a refit of the whole list (the fit runs outer -> inner, hit to hit).
struct ExtView {
  const int32_t* K_off;    // [J+1] first track of each job
  const int32_t* accf;     // [capT] 1 if the tracklet became a track
  const int32_t* ext_off;  // [capK+1] first slot of each track in ext_hits (scan of its rows below)
  int32_t* ext_hits;       // found clusters (grid order), rows descending, per track
  int32_t* ext_n;          // [capK] found, then kept
  uint32_t* claim;         // [N] grid order: max key of the tracks that found the cluster
  int32_t* xn;             // [capK+1] hits of the extended track
  int32_t capX;            // slots of ext_hits
};

// Rows below the innermost hit of every track whose fit succeeded: its slots in ext_hits.
__global__ void k_ext_rows(GridView G, FitView F, ExtView E, int32_t* rows, Bound lo_b, Bound hi_b) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  rows[kk] = F.ndf[kk] >= 0 ? G.gh[F.sel_hits[F.sel_off[kk]]].slot % kRows : 0;
}

__device__ __forceinline__ uint32_t ext_key(const FitView& F, const ExtView& E, int32_t kk, int32_t slot) {
  const int32_t local = kk - E.K_off[slot / kSlotsPerJob];
  const int32_t n = F.sel_off[kk + 1] - F.sel_off[kk];
  return ((uint32_t)n << 24) | (uint32_t)(kLocalIdMax - local);
}

// The search of one track as a step machine: ext_begin sets it up (false when there is
// nothing to search: a failed fit, the innermost hit on row 0, or no room in ext_hits),
// ext_step searches one row (true when the search has ended) and claims what it finds.
// The search of one track as a step machine: ext_begin sets it up (false when there is
// nothing to search: a failed fit, or the innermost hit on row 0), ext_step searches one
// row (true when the search has ended).  A track's found clusters go to its slots in
// ext_hits, one per row below its innermost hit, allocated in track order; a track whose
// slots would pass the end of ext_hits (its rows below outnumber the clusters, which only
// inputs cut short of their inner rows reach) keeps no list: the later kernels replay its
// search, which takes the same steps (it reads only the grid, the ownership and its own
// state), instead of reading the list.
struct ExtLane {
  State S;
  float x;
  int32_t kk, base, slot_base, last;
  uint32_t key;
  int r, misses, m;
  bool store, claim;
};

__device__ __forceinline__ bool ext_begin(const GridView& G, const FitView& F, const ExtView& E, ExtLane& T,
                                          int32_t kk, bool replay) {
  T.kk = kk;
  T.m = 0;
  if (F.ndf[kk] < 0) return false;
  const int32_t hs = G.gh[F.sel_hits[F.sel_off[kk]]].slot;
  const int r_in = hs % kRows;
  if (r_in == 0) return false;
  T.slot_base = hs - r_in;
  T.base = E.ext_off[kk];
  T.store = !replay && (int64_t)T.base + r_in <= (int64_t)E.capX;
  T.claim = !replay;
  T.key = ext_key(F, E, kk, hs);
  load_fit(F, kk, T.S, T.x);
  T.r = r_in - 1;
  T.misses = 0;
  return true;
}

__device__ __forceinline__ bool ext_step(const GridView& G, const TrackletView& V, const ExtView& E, ExtLane& T,
                                         const Consts& k) {
  const SlotGrid g = G.sg[T.slot_base + T.r];  // loaded before the transport (latency)
  const float xr = k.x[T.r];
  if (!propagate(T.S, T.x, xr, k)) return true;
  T.x = xr;
  const SInv si = s_inverse(T.S.C, k.vy, k.vz);
  if (!si.ok) return true;
  const float wy = k.nwin * sqrt_rn(T.S.C[0] + k.vy);
  const float wz = k.nwin * sqrt_rn(T.S.C[2] + k.vz);
  int32_t cand = -1;
  float bchi = 0.f, cy = 0.f, cz = 0.f;
  // clusters owned by a selected track are not candidates
  window_best(G, g, T.S, si, wy, wz,
              [&](int32_t c) {
                const uint32_t w = V.hitw[c];
                if (w == 0u) return true;
                const int32_t t = key_tracklet(w, V.T_off, T.slot_base);
                return !((uint32_t)t < (uint32_t)V.capT && E.accf[t]);
              },
              cand, bchi, cy, cz);
  if (cand >= 0 && bchi <= k.chi2_follow) {
    if (!kf_update(T.S, cy, cz, k, nullptr)) return true;
    if (T.store) E.ext_hits[T.base + T.m] = cand;
    if (T.claim) atomicMax(&E.claim[cand], T.key);
    T.last = cand;
    ++T.m;
    T.misses = 0;
  } else if (++T.misses >= k.max_miss) {
    return true;
  }
  return --T.r < 0;
}

// The next found cluster of a replayed search (-1 when the search ends first).
__device__ __forceinline__ int32_t ext_next(const GridView& G, const TrackletView& V, const ExtView& E,
                                            ExtLane& T, bool& ended, const Consts& k) {
  while (!ended) {
    const int m0 = T.m;
    ended = ext_step(G, V, E, T, k);
    if (T.m > m0) return T.last;
  }
  return -1;
}

// One lane per track: the search, claiming every cluster it finds.  ext_n: the number found,
// or -1 - that number for a track that kept no list.
__global__ __launch_bounds__(128) void k_ext_search(GridView G, TrackletView V, FitView F, ExtView E,
                                                    Bound lo_b, Bound hi_b, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  ExtLane T;
  bool listed = true;
  if (ext_begin(G, F, E, T, kk, false)) {
    listed = T.store;
    while (!ext_step(G, V, E, T, k)) {
    }
  }
  E.ext_n[kk] = listed ? T.m : -1 - T.m;
}

// The fit of track kk continued over its kept clusters from the stored state (hit to hit,
// as the fit runs), stored in its record.
template <class Next>
__device__ __forceinline__ void ext_continue(const GridView& G, const FitView& F, int32_t kk, int n0, int kept,
                                             Next next, const Consts& k) {
  State S;
  float x;
  load_fit(F, kk, S, x);
  float chi2 = F.chi2[kk];
  bool ok = true;
  for (int q = 0; q < kept && ok; ++q) {
    const GHit Hq = ldh(G.gh + next(q));
    const float xh = k.x[Hq.slot % kRows];
    if (!propagate(S, x, xh, k)) { ok = false; break; }
    x = xh;
    float c2;
    if (!kf_update(S, Hq.y, Hq.z, k, &c2)) { ok = false; break; }
    chi2 = chi2 + c2;
  }
  store_fit(F, kk, S, x, chi2, n0 + kept, ok);
}

// One lane per track: the kept prefix of the found clusters (up to the first one another
// track won), the fit continued over them from the stored state, and the length of the
// extended hit list.  ext_n becomes the kept number (-1 - it without a list: such a track's
// fit is continued by k_ext_write, which replays its search from the stored state).
__global__ __launch_bounds__(128) void k_ext_keep(GridView G, TrackletView V, FitView F, ExtView E,
                                                  Bound lo_b, Bound hi_b, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  const int32_t n0 = F.sel_off[kk + 1] - F.sel_off[kk];
  const int32_t v = E.ext_n[kk];
  const bool listed = v >= 0;
  const int m = listed ? v : -1 - v;
  int kept = 0;
  if (m > 0) {
    const int32_t base = E.ext_off[kk];
    const int32_t hs = G.gh[F.sel_hits[F.sel_off[kk]]].slot;
    const uint32_t key = ext_key(F, E, kk, hs);
    if (listed) {
      while (kept < m && E.claim[E.ext_hits[base + kept]] == key) ++kept;
      if (kept > 0) ext_continue(G, F, kk, n0, kept, [&](int q) { return E.ext_hits[base + q]; }, k);
    } else {
      ExtLane R;
      bool ended = false;
      ext_begin(G, F, E, R, kk, true);
      for (int q = 0; q < m; ++q) {
        const int32_t c = ext_next(G, V, E, R, ended, k);
        if (c < 0 || E.claim[c] != key) break;
        ++kept;
      }
    }
  }
  E.ext_n[kk] = listed ? kept : -1 - kept;
  E.xn[kk] = n0 + kept;
}

// One wave per track: the extended hit list (kept clusters in ascending rows, then the
// owned hits) written at its offset in the new list; a track without a list replays its
// search on lane 0.
__global__ __launch_bounds__(256) void k_ext_write(GridView G, TrackletView V, FitView F, ExtView E,
                                                   const int32_t* xoff, int32_t* xhits, Bound lo_b, Bound hi_b,
                                                   int32_t capH, int32_t* counters, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w0 = lo + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6); w0 < hi; w0 += nw) {
    const int32_t kk = (int32_t)w0;
    const int32_t o = xoff[kk];
    const int32_t v = E.ext_n[kk];
    const bool listed = v >= 0;
    const int kept = listed ? v : -1 - v;
    const int32_t base = E.ext_off[kk];
    const int32_t q0 = F.sel_off[kk], q1 = F.sel_off[kk + 1];
    const int32_t n = kept + (q1 - q0);
    for (int32_t i = lane; i < n; i += 64) {
      if (i < kept && !listed) continue;
      const int32_t c = i < kept ? E.ext_hits[base + kept - 1 - i] : F.sel_hits[q0 + i - kept];
      if (o + i < capH) xhits[o + i] = c;
    }
    if (!listed && kept > 0 && lane == 0) {
      // the search replayed from the stored state, which k_ext_keep left unchanged; its kept
      // clusters written in ascending rows, then the fit continued over them
      ExtLane R;
      bool ended = false;
      ext_begin(G, F, E, R, kk, true);
      for (int j = 0; j < kept; ++j) {
        const int32_t c = ext_next(G, V, E, R, ended, k);
        if (o + kept - 1 - j < capH) xhits[o + kept - 1 - j] = c;
      }
      if (o + n <= capH)  // (past the capacity the run reports it and the lists are cut)
        ext_continue(G, F, kk, q1 - q0, kept, [&](int q) { return xhits[o + kept - 1 - q]; }, k);
    }
    if (lane == 0 && o + n > capH) atomicOr(&counters[kCntStatus], kStatusCapacity);
  }
}


// --- merge: candidate search.  Tracks are bucketed by (event, sector).
// Merge buckets: (event, sector, z bin of the track's innermost cluster); bins are
// merge_dz wide, clamped at the ends, so the candidates of A within merge_dz of its end
// z lie in 2-3 consecutive bins of one bucket.
struct MergeView {
  const int32_t* trk_event;   // [capK] event of each selected track
  int32_t* bucket_cnt;        // [n_events*36]
  int32_t* bucket_off;        // [n_events*36+1]
  int32_t* bucket_fill;       // [n_events*36]
  int32_t* bucket_trk;        // [capK]
  float* bucket_z;            // [capK] z of the innermost cluster of each bucketed track
  uint64_t* bestA;            // [capK] packed (chi2 bits, id) best partner of A
  uint64_t* bestB;            // [capK]
  int32_t* chain_next;        // [capK]
  int32_t* chain_prev;        // [capK]
  int32_t* head_list;         // [capK]
  int32_t* n_heads;           // [1]
  float* link_t0;             // [capK] collision time of a membrane link a -> chain_next[a]
  int32_t n_events;
  int32_t nz;                 // z bins per (event, sector)
  float dz;
};

__device__ __forceinline__ int merge_zbin(float z, float dz, int nz) {
  float b = floorf(z / dz) + (float)(nz / 2);
  b = fminf(fmaxf(b, 0.f), (float)(nz - 1));
  return (int)b;
}

// Event of every selected track; tracks that can be an outer piece are counted into the
// bucket of their (event, sector, side, z bin of the innermost cluster).  Side 0: across
// the -y sector edge (fitted, innermost cluster within merge_edge of the edge, y < 0), side
// 1: the +y edge; side 2: across the central membrane (fitted, tan lambda pointing away from
// it: > 0 on side A, < 0 on side C), when that merge is on.
__device__ __forceinline__ int merge_bkey(int ev, int sec, int side, float z, float dz, int nz) {
  return ((ev * kSectors + sec) * 3 + side) * nz + merge_zbin(z, dz, nz);
}
__device__ __forceinline__ bool outer_piece(const GHit& Hb, const int32_t* ndf, int32_t kk, const Consts& k) {
  const float eb = k.x[Hb.slot % kRows] * k.tan10 - fabsf(Hb.y);
  return ndf[kk] >= 0 && eb <= k.merge_edge;
}
__device__ __forceinline__ bool membrane_outer_piece(const int32_t* ndf, const float* fitrow, int32_t kk,
                                                     int sec, const Consts& k) {
  if (!k.membrane || ndf[kk] < 0) return false;
  const float t = fitrow[(int64_t)kk * kFitStride + 3];
  return sec < kHalf ? t > 0.f : t < 0.f;
}

__global__ void k_track_event(const int32_t* sel_from, const int32_t* start, const int32_t* sel_off,
                              const int32_t* sel_hits, const GHit* gh, const int32_t* job_event,
                              const int32_t* ndf, const float* fitrow, int32_t* trk_event,
                              int32_t* bucket_cnt, Bound lo_b,
                              Bound hi_b, int32_t capK, int32_t n_events, int32_t nz, Consts k,
                              int32_t* counters) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  const int32_t h = start[sel_from[kk]];
  const int32_t sl = gh[h].slot;
  const int job = sl / (kSectors * kRows);
  const int sec = (sl / kRows) % kSectors;
  int ev = job_event ? job_event[job] : job;
  if (ev < 0 || ev >= n_events) {  // events must be numbered 0..n_jobs-1
    atomicOr(&counters[kCntStatus], kStatusRange);
    ev = job;
  }
  trk_event[kk] = ev;
  const GHit Hb = ldh(gh + sel_hits[sel_off[kk]]);
  if (outer_piece(Hb, ndf, kk, k))
    atomicAdd(&bucket_cnt[merge_bkey(ev, sec, Hb.y < 0.f ? 0 : 1, Hb.z, k.merge_dz, nz)], 1);
  if (membrane_outer_piece(ndf, fitrow, kk, sec, k))
    atomicAdd(&bucket_cnt[merge_bkey(ev, sec, 2, Hb.z, k.merge_dz, nz)], 1);
}

__global__ void k_track_bucket(const int32_t* sel_from, const int32_t* start, const int32_t* sel_off,
                               const int32_t* sel_hits, const GHit* gh, const int32_t* ndf, const float* fitrow,
                               MergeView M, Bound lo_b, Bound hi_b, int32_t capK, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  const int32_t sl = gh[start[sel_from[kk]]].slot;
  const int sec = (sl / kRows) % kSectors;
  const GHit Hb = ldh(gh + sel_hits[sel_off[kk]]);
  if (outer_piece(Hb, ndf, kk, k)) {
    const int b = merge_bkey(M.trk_event[kk], sec, Hb.y < 0.f ? 0 : 1, Hb.z, k.merge_dz, M.nz);
    const int32_t q = M.bucket_off[b] + atomicAdd(&M.bucket_fill[b], 1);
    M.bucket_trk[q] = kk;
    M.bucket_z[q] = Hb.z;
  }
  if (membrane_outer_piece(ndf, fitrow, kk, sec, k)) {
    const int b = merge_bkey(M.trk_event[kk], sec, 2, Hb.z, k.merge_dz, M.nz);
    const int32_t q = M.bucket_off[b] + atomicAdd(&M.bucket_fill[b], 1);
    M.bucket_trk[q] = kk;
    M.bucket_z[q] = Hb.z;
  }
}

// packed (chi2, id): chi2 >= 0 so its bits order like the value; smaller wins.
__device__ __forceinline__ uint64_t pack_best(float c, int32_t id) {
  return ((uint64_t)__float_as_uint(c) << 32) | (uint32_t)id;
}

// A's tracklet end state carried to plane x (same sector frame: the other side of the
// membrane); false when the transport fails.
__device__ __forceinline__ bool membrane_transport(const TrackletView& V, int32_t ta, float x_to, State& S,
                                                   const Consts& k) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    S.P[i] = V.state[(int64_t)ta * kStateStride + i];
    S.L[i] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < 15; ++i) S.C[i] = V.state[(int64_t)ta * kStateStride + 5 + i];
  float x = V.state[(int64_t)ta * kStateStride + 20];
  return propagate(S, x, x_to, k);
}

__device__ __forceinline__ void load_fit_pc(const FitView& F, int32_t b, float* P, float* C, float& x) {
  float rb[kFitStride];
  const float* src = F.row + (int64_t)b * kFitStride;
#pragma unroll
  for (int i = 0; i < 24; i += 4) {
    const float4 v = *reinterpret_cast<const float4*>(src + i);
    rb[i] = v.x;
    rb[i + 1] = v.y;
    rb[i + 2] = v.z;
    rb[i + 3] = v.w;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) P[i] = rb[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = rb[5 + i];
  x = rb[20];
}

// Candidates across the central membrane: A's end heads for it (tan lambda < 0 on side A,
// > 0 on side C); B (bucket side 2 of the same sector on the other side) starts beyond A's
// end, its innermost measured z mirrors A's end (|z_A + z_B| <= merge_dz), the true z at B's
// plane (the mean of the two measured z) lies within merge_edge of the membrane, and the
// chi2 over y, sin phi, tan lambda and q/pT is at most chi2_merge.
__device__ void membrane_candidates(const TrackletView& V, const FitView& F, const MergeView& M, int32_t a,
                                    int32_t ta, int seca, float za, float xa, const Consts& k) {
  const bool a_side = seca < kHalf;
  const float tA = V.state[(int64_t)ta * kStateStride + 3];
  if (!(a_side ? tA < 0.f : tA > 0.f)) return;
  const int sb = (seca + kHalf) % kSectors;
  const float zlo = -za - k.merge_dz - 1.f, zhi = -za + k.merge_dz + 1.f;
  const int32_t b0 = M.bucket_off[merge_bkey(M.trk_event[a], sb, 2, zlo, k.merge_dz, M.nz)];
  const int32_t b1 = M.bucket_off[merge_bkey(M.trk_event[a], sb, 2, zhi, k.merge_dz, M.nz) + 1];
  for (int32_t q = b0; q < b1; ++q) {
    if (!(fabsf(za + M.bucket_z[q]) <= k.merge_dz)) continue;
    const int32_t b = M.bucket_trk[q];
    float PB[5], CB[15], xb;
    load_fit_pc(F, b, PB, CB, xb);
    if (!(xb > xa)) continue;
    State S;
    if (!membrane_transport(V, ta, xb, S, k)) continue;
    if (!(fabsf((S.P[1] + PB[1]) * 0.5f) <= k.merge_edge)) continue;
    const float c = membrane_chi2(S.P, S.C, PB, CB);
    if (!(c <= k.chi2_merge)) continue;
    atomicMin((unsigned long long*)&M.bestA[a], (unsigned long long)pack_best(c, b));
    atomicMin((unsigned long long*)&M.bestB[b], (unsigned long long)pack_best(c, a));
  }
}

__global__ __launch_bounds__(256) void k_merge_candidates(GridView G, TrackletView V, FitView F,
                                                          MergeView M, Bound lo_b, Bound hi_b,
                                                          Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int32_t a = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= hi) return;
  if (F.ndf[a] < 0) return;
  const int32_t ta = F.sel_from[a];
  const float ya = V.state[(int64_t)ta * kStateStride + 0];
  const float za = V.state[(int64_t)ta * kStateStride + 1];
  const float xa = V.state[(int64_t)ta * kStateStride + 20];
  const int32_t sla = G.gh[V.start[ta]].slot;
  const int seca = (sla / kRows) % kSectors;
  if (k.membrane) membrane_candidates(V, F, M, a, ta, seca, za, xa, k);
  const float edge = xa * k.tan10 - fabsf(ya);
  if (!(edge <= k.merge_edge)) return;
  const int dir = ya > 0.f ? 1 : kHalf - 1;
  const int sb = (seca / kHalf) * kHalf + (seca % kHalf + dir) % kHalf;
  // outer pieces start at the edge shared with A's sector: their -y edge if A leaves
  // through its +y edge (side 0), else their +y edge (side 1)
  // (the bin range is padded by 1 cm so that rounding of za -/+ merge_dz never drops a
  // track the exact gate below accepts)
  const int side = dir == 1 ? 0 : 1;
  const float zlo = za - k.merge_dz - 1.f, zhi = za + k.merge_dz + 1.f;
  const int32_t b0 = M.bucket_off[merge_bkey(M.trk_event[a], sb, side, zlo, k.merge_dz, M.nz)];
  const int32_t b1 = M.bucket_off[merge_bkey(M.trk_event[a], sb, side, zhi, k.merge_dz, M.nz) + 1];
  if (b0 >= b1) return;
  // A's end state in B's frame: the same for every candidate
  State R;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    R.P[i] = V.state[(int64_t)ta * kStateStride + i];
    R.L[i] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < 15; ++i) R.C[i] = V.state[(int64_t)ta * kStateStride + 5 + i];
  float xr = xa;
  if (!rotate(R, xr, seca, sb, k)) return;
  for (int32_t q = b0; q < b1; ++q) {
    if (!(fabsf(za - M.bucket_z[q]) <= k.merge_dz)) continue;
    const int32_t b = M.bucket_trk[q];
    State S = R;
    float x = xr;
    // B's fitted record: 21 consecutive floats
    float rb[kFitStride];
    const float* src = F.row + (int64_t)b * kFitStride;
#pragma unroll
    for (int i = 0; i < kFitStride; i += 4) {
      const float4 v = *reinterpret_cast<const float4*>(src + i);
      rb[i] = v.x;
      rb[i + 1] = v.y;
      rb[i + 2] = v.z;
      rb[i + 3] = v.w;
    }
    if (!propagate(S, x, rb[20], k)) continue;
    float PB[5], CB[15];
#pragma unroll
    for (int i = 0; i < 5; ++i) PB[i] = rb[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) CB[i] = rb[5 + i];
    const float c = merge_chi2(S.P, S.C, PB, CB);
    if (!(c <= k.chi2_merge)) continue;
    atomicMin((unsigned long long*)&M.bestA[a], (unsigned long long)pack_best(c, b));
    atomicMin((unsigned long long*)&M.bestB[b], (unsigned long long)pack_best(c, a));
  }
}

// Mutual best pairs -> chain links; a link across the membrane gets its collision time.
__global__ void k_merge_links(GridView G, TrackletView V, FitView F, MergeView M, Bound lo_b, Bound hi_b,
                              int32_t capK, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), capK);
  const int32_t a = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= hi) return;
  const uint64_t ba = M.bestA[a];
  if (ba == ~0ull) return;
  const int32_t b = (int32_t)(uint32_t)ba;
  const uint64_t bb = M.bestB[b];
  if ((int32_t)(uint32_t)bb != a) return;
  M.chain_next[a] = b;
  M.chain_prev[b] = a;
  const int32_t ta = F.sel_from[a];
  const int seca = (G.gh[V.start[ta]].slot / kRows) % kSectors;
  const int secb = (G.gh[V.start[F.sel_from[b]]].slot / kRows) % kSectors;
  if ((seca < kHalf) != (secb < kHalf)) {
    float PB[5], CB[15], xb;
    load_fit_pc(F, b, PB, CB, xb);
    State S;
    membrane_transport(V, ta, xb, S, k);
    M.link_t0[a] = membrane_t0(seca < kHalf, S.P[1], PB[1], k);
  }
}

// Chain heads (no inner partner, an outer partner) are listed for the refit; every
// track gets its output flag: absorbed pieces are dropped.
__global__ void k_merge_heads(MergeView M, Bound lo_b, Bound hi_b, int32_t capK, int32_t* keep) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), capK);
  const int32_t a = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= hi) return;
  // a piece is absorbed if a head reaches it within kHalf steps (pure cycles stay apart)
  bool absorbed = false;
  if (M.chain_prev[a] >= 0) {
    int32_t p = a;
    int steps = 0;
    while (M.chain_prev[p] >= 0 && steps < kHalf) {
      p = M.chain_prev[p];
      ++steps;
    }
    absorbed = M.chain_prev[p] < 0;
  }
  keep[a] = absorbed ? 0 : 1;
  if (M.chain_prev[a] < 0 && M.chain_next[a] >= 0) {
    const int32_t i = atomicAdd(M.n_heads, 1);
    M.head_list[i] = a;
  }
}

// ------------------------------------------------------------------ output
struct OutView {
  int32_t cap_tracks, cap_hits;
  int32_t* n_tracks;
  int32_t* hit_off;
  int32_t* hits;
  float* param;
  float* cov;
  float* x_ref;
  float* chi2;
  int32_t* ndf;
  int32_t* sector;
  int32_t* job;
  int32_t* tracklet;
  float* t0;
};

__global__ void k_out_count(FitView F, const int32_t* keep, int32_t* outn, Bound lo_b, Bound hi_b) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int32_t kk = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= hi) return;
  int n = 0;
  if (keep[kk]) {
    const bool walk = F.chain_next && F.chain_prev[kk] < 0;
    int np = 0;
    for (int32_t p = kk; p >= 0 && np <= kHalf; p = walk ? F.chain_next[p] : -1, ++np)
      n += F.sel_off[p + 1] - F.sel_off[p];
  }
  outn[kk] = n;
}

// One wave per output track: the hit lists of its pieces copied with the lanes striding
// over them (coalesced), the per-track fields written by lanes 0..23 (the collision time by
// k_out_t0).
__global__ __launch_bounds__(256) void k_out_write(GridView G, TrackletView V, FitView F, OutView O,
                                                   const int32_t* keep, const int32_t* oid, const int32_t* ooff,
                                                   Bound lo_b, Bound hi_b, int32_t* counters, Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w0 = lo + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6); w0 < hi; w0 += nw) {
    const int32_t kk = (int32_t)w0;
    if (!keep[kk]) continue;
    const int32_t o = oid[kk];
    const int32_t h0 = ooff[kk];
    if (o >= O.cap_tracks) {
      if (lane == 0) atomicOr(&counters[kCntStatus], kStatusCapacity);
      continue;
    }
    int w = 0;
    const bool walk = F.chain_next && F.chain_prev[kk] < 0;
    int np = 0;
    for (int32_t p = kk; p >= 0 && np <= kHalf; p = walk ? F.chain_next[p] : -1, ++np) {
      const int32_t q0 = F.sel_off[p], q1 = F.sel_off[p + 1];
      for (int32_t q = q0 + lane; q < q1; q += 64) {
        const int32_t pos = h0 + w + (q - q0);
        if (pos < O.cap_hits) O.hits[pos] = G.gh[F.sel_hits[q]].idx;
      }
      w += q1 - q0;
    }
    if (lane == 0) {
      O.hit_off[o] = h0;
      if (h0 + w > O.cap_hits) atomicOr(&counters[kCntStatus], kStatusCapacity);
    }
    if (lane < 5) {
      O.param[(int64_t)o * 5 + lane] = F.row[(int64_t)kk * kFitStride + lane];
    } else if (lane < 20) {
      O.cov[(int64_t)o * 15 + (lane - 5)] = F.row[(int64_t)kk * kFitStride + lane];
    } else if (lane == 20) {
      O.x_ref[o] = F.row[(int64_t)kk * kFitStride + 20];
    } else if (lane == 21) {
      O.chi2[o] = F.chi2[kk];
    } else if (lane == 22) {
      O.ndf[o] = F.ndf[kk];
    } else if (lane == 23) {
      const int32_t t = F.sel_from[kk];
      const int32_t sl = G.gh[V.start[t]].slot;
      O.sector[o] = (sl / kRows) % kSectors;
      O.job[o] = sl / (kSectors * kRows);
      O.tracklet[o] = t;
    }
  }
}

// The collision time of each output track, one lane per track: the transport of the fitted
// state to the beam line is the longest per-track computation of the output, and a wave per
// track would run it on one lane.
__global__ __launch_bounds__(256) void k_out_t0(GridView G, TrackletView V, FitView F, OutView O,
                                                const int32_t* keep, const int32_t* oid, Bound lo_b, Bound hi_b,
                                                Consts k) {
  const int32_t lo = lo_b.get();
  const int32_t hi = min(hi_b.get(), F.capK);
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t kk = (int32_t)i;
    if (!keep[kk]) continue;
    const int32_t o = oid[kk];
    if (o >= O.cap_tracks) continue;
    const bool walk = F.chain_next && F.chain_prev[kk] < 0;
    const int32_t sec = (G.gh[V.start[F.sel_from[kk]]].slot / kRows) % kSectors;
    const float* row = F.row + (int64_t)kk * kFitStride;
    // a chain across the central membrane: its innermost membrane link's time
    bool memb = false;
    float tm = 0.f;
    if (walk) {
      int32_t p = kk;
      int ps = sec;
      for (int n = 0; n < kHalf && F.chain_next[p] >= 0; ++n) {
        const int32_t q = F.chain_next[p];
        const int qs = (G.gh[V.start[F.sel_from[q]]].slot / kRows) % kSectors;
        if ((ps < kHalf) != (qs < kHalf)) {
          memb = true;
          tm = F.link_t0[p];
          break;
        }
        p = q;
        ps = qs;
      }
    }
    O.t0[o] = F.ndf[kk] < 0 ? __builtin_nanf("") : memb ? tm : collision_time(row, row[20], sec, k);
  }
}

__global__ void k_out_finish(const int32_t* oid, const int32_t* ooff, Bound hi_b, int32_t capK,
                             OutView O, int32_t* counters) {
  const int32_t hi = min(hi_b.get(), capK);
  const int32_t K = oid[hi], H = ooff[hi];
  counters[kCntOut] = K;
  counters[kCntOutHits] = H;
  if (O.n_tracks) *O.n_tracks = K;
  if (K <= O.cap_tracks) O.hit_off[K] = H;
}

// ------------------------------------------------------------------ track-model compression
// Clusters are stored as residuals to the fitted tracks (section 5): a record per cluster,
// rs = row | sector << 8 | absolute << 15 and two int16 codes in units of the quantisation
// steps.  Track hits come first, in track order, with residual codes against the track's
// predicted position where it exists and fits in 16 bits, else absolute codes; then the
// clusters in no track, in input order, with absolute codes.  0x7FFF marks an invalid
// cluster (or a hit index outside the cluster list).
constexpr uint32_t kRecInvalid = 0x7FFFu;
constexpr float kCodeMax = 32767.f;

struct CmpClusters {
  const uint8_t* sector;
  const int16_t* row;
  const float* y;
  const float* z;
  int32_t n;
};
struct CmpTracks {
  const int32_t* n_tracks;
  int32_t cap_tracks, cap_hits;
  const int32_t* off;
  const int32_t* hits;
  const float* param;
  const float* x_ref;
  const int32_t* sector;
  const int32_t* ndf;
};
struct CmpCodes {
  int32_t cap;
  int32_t* n_codes;
  int32_t* n_attached;
  uint16_t* rs;
  int16_t* ey;
  int16_t* ez;
  int8_t* ezh;  // high byte of 24-bit absolute z codes, or null (16-bit codes)
};
struct CmpOut {
  uint8_t* sector;
  int16_t* row;
  float* y;
  float* z;
};

__device__ __forceinline__ int32_t cmp_tracks(const CmpTracks& T) {
  const int32_t k = *T.n_tracks;
  return k < 0 ? 0 : min(k, T.cap_tracks);
}
__device__ __forceinline__ bool cmp_cluster_ok(int s, int r, float y, float z) {
  return s < kSectors && r >= 0 && r < kRows && finite_f(y) && finite_f(z);
}
__device__ __forceinline__ int16_t abs_code(float v, float iq, int32_t& st) {
  float e = rintf(v * iq);
  if (e > kCodeMax) {
    e = kCodeMax;
    st |= kStatusRange;
  }
  if (e < -kCodeMax) {
    e = -kCodeMax;
    st |= kStatusRange;
  }
  return (int16_t)e;
}
// Packed copy of the clusters, written in one coalesced pass: (y, z, record word) in 16
// bytes, so that a track hit costs one gather.  The record word is row | sector << 8, or
// the invalid record.  The one-byte marks (1 = in no track) are set in the same pass and
// cleared by the track hits: a byte array small enough to stay in the last-level cache
// while the hits scatter into it.
__global__ __launch_bounds__(256) void k_cmp_pack(CmpClusters in, int4* rec, uint8_t* free_mark) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= in.n) return;
  const int s = in.sector[i], r = in.row[i];
  const float yv = in.y[i], zv = in.z[i];
  const uint32_t w = cmp_cluster_ok(s, r, yv, zv) ? ((uint32_t)r | ((uint32_t)s << 8)) : kRecInvalid;
  rec[i] = make_int4(__float_as_int(yv), __float_as_int(zv), (int32_t)w, 0);
  free_mark[i] = 1;
}

// Time frames: a 24-bit absolute z code, its low 16 bits and its signed high byte
// (e = hi * 2^16 + lo as unsigned), saturated at +-(2^23 - 1).
constexpr float kWideMax = 8388607.f;
__device__ __forceinline__ void abs_code_wide(float v, float iq, int16_t& lo, int8_t& hi, int32_t& st) {
  float e = rintf(v * iq);
  if (e > kWideMax) {
    e = kWideMax;
    st |= kStatusRange;
  }
  if (e < -kWideMax) {
    e = -kWideMax;
    st |= kStatusRange;
  }
  const int32_t c = (int32_t)e;
  lo = (int16_t)(uint16_t)(c & 0xFFFF);
  hi = (int8_t)(c >> 16);
}

// Absolute record of a packed cluster (or the invalid record); ezh: the high byte of the
// z code when wide, else untouched.
__device__ __forceinline__ void encode_abs(const int4& R, float iqy, float iqz, bool wide, uint32_t& rs,
                                           int16_t& ey, int16_t& ez, int8_t& ezh, int32_t& st) {
  const uint32_t w = (uint32_t)R.z;
  if (w == kRecInvalid) {
    rs = kRecInvalid;
    ey = ez = 0;
    st |= kStatusRange;
    return;
  }
  rs = w | (1u << 15);
  ey = abs_code(__int_as_float(R.x), iqy, st);
  if (wide)
    abs_code_wide(__int_as_float(R.y), iqz, ez, ezh, st);
  else
    ez = abs_code(__int_as_float(R.y), iqz, st);
}

// Track hits: one wave per track (grid-stride), one lane per hit.
__global__ __launch_bounds__(256) void k_cmp_tracks(int32_t n, const int4* rec, uint8_t* free_mark, CmpTracks T,
                                                    CmpCodes O, Consts k, float iqy, float iqz,
                                                    int32_t* counters) {
  const int32_t K = cmp_tracks(T);
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w_first = xcd_tile(blockIdx.x, gridDim.x) * wpb + (threadIdx.x >> 6);
  int32_t st = 0;
  for (int64_t w = w_first; w < K; w += nw) {
    const int32_t i = (int32_t)w;
    const int32_t a = max(T.off[i], 0);
    int32_t b = T.off[i + 1];
    if (b > T.cap_hits) {
      b = T.cap_hits;
      st |= kStatusCapacity;
    }
    float P[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) P[q] = T.param[(int64_t)i * 5 + q];
    const float xr = T.x_ref[i];
    const int sref = T.sector[i];
    const bool fit_ok = T.ndf[i] >= 0;
    for (int32_t j = a + lane; j < b; j += 64) {
      const int32_t h = T.hits[j];
      const bool valid = (uint32_t)h < (uint32_t)n;
      int4 R = make_int4(0, 0, (int32_t)kRecInvalid, 0);
      if (valid) {
        R = rec[h];
        // every hit is marked, also beyond the record capacity: the count of records
        // needed must not depend on it
        free_mark[h] = 0;
      }
      if (j >= O.cap) {
        st |= kStatusCapacity;
        continue;
      }
      uint32_t rs;
      int16_t ey = 0, ez = 0;
      int8_t ezh = 0;
      const uint32_t wd = (uint32_t)R.z;
      if (!valid) {
        rs = kRecInvalid;
        st |= kStatusRange;
      } else {
        const int r = wd & 0xFF, s = (wd >> 8) & 0x7F;
        const float yv = __int_as_float(R.x), zv = __int_as_float(R.y);
        bool done = false;
        float py, pz;
        if (wd != kRecInvalid && fit_ok && predict_yz(P, xr, sref, s, r, k, py, pz)) {
          const float e1 = rintf((yv - py) * iqy);
          const float e2 = rintf((zv - pz) * iqz);
          if (fabsf(e1) <= kCodeMax && fabsf(e2) <= kCodeMax) {
            rs = wd;
            ey = (int16_t)e1;
            ez = (int16_t)e2;
            done = true;
          }
        }
        if (!done) encode_abs(R, iqy, iqz, O.ezh != nullptr, rs, ey, ez, ezh, st);
      }
      O.rs[j] = (uint16_t)rs;
      O.ey[j] = ey;
      O.ez[j] = ez;
      if (O.ezh) O.ezh[j] = ezh;
    }
  }
  if (st) atomicOr(&counters[kCntStatus], st);
}

// Clusters in no track (mark still set), counted per tile of kScanTile input indices; item q
// of thread t is index tile * kScanTile + q * kScanThreads + t, so that the loads coalesce.
__global__ __launch_bounds__(kScanThreads) void k_cmp_count(int32_t n, const uint8_t* free_mark, int32_t* bsum) {
  __shared__ int lds[40];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  int c = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t k = base + (int64_t)q * kScanThreads;
    if (k < n && free_mark[k]) ++c;
  }
  int total;
  block_excl_scan(c, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Their records: H + (rank among them in input order), absolute codes; bsum holds the
// exclusive tile offsets and *n_free their sum.
__global__ __launch_bounds__(kScanThreads) void k_cmp_free(int32_t n, const int4* rec, const uint8_t* free_mark,
                                                          CmpTracks T, CmpCodes O, const int32_t* bsum,
                                                          const int32_t* n_free, float iqy, float iqz,
                                                          int32_t* counters) {
  __shared__ int lds[40];
  const int32_t K = cmp_tracks(T);
  const int32_t H = K > 0 ? max(T.off[K], 0) : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *O.n_codes = H + *n_free;
    *O.n_attached = H;
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  int64_t rank = (int64_t)H + bsum[blockIdx.x];
  int32_t st = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t k = base + (int64_t)q * kScanThreads;
    const int m = (k < n && free_mark[k]) ? 1 : 0;
    int tot;
    const int r = block_excl_scan(m, lds, tot);
    if (m) {
      const int4 R = rec[k];
      const int64_t pos = rank + r;
      if (pos >= O.cap) {
        st |= kStatusCapacity;
      } else {
        uint32_t rs;
        int16_t ey, ez;
        int8_t ezh = 0;
        encode_abs(R, iqy, iqz, O.ezh != nullptr, rs, ey, ez, ezh, st);
        O.rs[pos] = (uint16_t)rs;
        O.ey[pos] = ey;
        O.ez[pos] = ez;
        if (O.ezh) O.ezh[pos] = ezh;
      }
    }
    rank += tot;
  }
  if (st) atomicOr(&counters[kCntStatus], st);
}

// One record back to (sector, row, y, z); P == nullptr: no track.
__device__ __forceinline__ void decode_one(const CmpCodes& C, const CmpOut& D, int32_t j, const float* P, float xr,
                                           int sref, bool fit_ok, float qy, float qz, const Consts& k, int32_t& st) {
  const uint32_t rs = C.rs[j];
  const int r = rs & 0xFF, s = (rs >> 8) & 0x7F;
  const bool absolute = (rs >> 15) != 0;
  const float nan = __builtin_nanf("");
  if (r >= kRows || s >= kSectors) {
    D.sector[j] = 255;
    D.row[j] = -1;
    D.y[j] = nan;
    D.z[j] = nan;
    return;
  }
  D.sector[j] = (uint8_t)s;
  D.row[j] = (int16_t)r;
  const int32_t cz = (absolute && C.ezh) ? (int32_t)C.ezh[j] * 65536 + (int32_t)(uint16_t)C.ez[j] : (int32_t)C.ez[j];
  const float dy = (float)C.ey[j] * qy, dz = (float)cz * qz;
  if (absolute) {
    D.y[j] = dy;
    D.z[j] = dz;
    return;
  }
  float py, pz;
  if (P && fit_ok && predict_yz(P, xr, sref, s, r, k, py, pz)) {
    D.y[j] = py + dy;
    D.z[j] = pz + dz;
  } else {
    D.y[j] = nan;
    D.z[j] = nan;
    st |= kStatusRange;
  }
}

__global__ __launch_bounds__(256) void k_dcmp_tracks(CmpTracks T, CmpCodes C, CmpOut D, Consts k, float qy,
                                                     float qz, int32_t* counters) {
  const int32_t K = cmp_tracks(T);
  const int32_t m = min(min(*C.n_codes, *C.n_attached), C.cap);
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w_first = xcd_tile(blockIdx.x, gridDim.x) * wpb + (threadIdx.x >> 6);
  int32_t st = 0;
  for (int64_t w = w_first; w < K; w += nw) {
    const int32_t i = (int32_t)w;
    const int32_t a = T.off[i], b = min(T.off[i + 1], m);
    float P[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) P[q] = T.param[(int64_t)i * 5 + q];
    const float xr = T.x_ref[i];
    const int sref = T.sector[i];
    const bool fit_ok = T.ndf[i] >= 0;
    for (int32_t j = max(a, 0) + lane; j < b; j += 64) decode_one(C, D, j, P, xr, sref, fit_ok, qy, qz, k, st);
  }
  if (st) atomicOr(&counters[kCntStatus], st);
}

__global__ __launch_bounds__(256) void k_dcmp_free(CmpCodes C, CmpOut D, Consts k, float qy, float qz,
                                                   int32_t* counters) {
  const int32_t m = min(*C.n_codes, C.cap);
  const int64_t j = (int64_t)max(*C.n_attached, 0) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  int32_t st = 0;
  decode_one(C, D, (int32_t)j, nullptr, 0.f, 0, false, qy, qz, k, st);
  if (st) atomicOr(&counters[kCntStatus], st);
}

// ------------------------------------------------------------------ rANS entropy coding
// Static range ANS (section 5: the common entropy coder after the TPC-specific steps) on
// streams of 16-bit symbols: a model of 2^16 slots per stream (every occurring symbol keeps
// a slot, the remainder to the most frequent), a 32-bit state with 16-bit renormalisation,
// and the stream cut into chunks of 64 lanes x 512 symbols, lane l of a chunk coding the
// chunk's symbols l, l + 64, ... with its own state, so that a wave codes a chunk with
// coalesced symbol loads and every lane is independent.
constexpr uint32_t kRansL = 1u << 16;

__host__ __device__ inline int64_t rans_chunk_first(int64_t l) {
  return (l / kRansLanesPerChunk) * (int64_t)kRansLanesPerChunk * kRansLaneSymbols + l % kRansLanesPerChunk;
}
__host__ __device__ inline int32_t rans_lane_count(int64_t n, int64_t l) {
  const int64_t first = rans_chunk_first(l);
  if (first >= n) return 0;
  const int64_t c = (n - first + kRansLanesPerChunk - 1) / kRansLanesPerChunk;
  return (int32_t)(c < kRansLaneSymbols ? c : kRansLaneSymbols);
}

// Symbol counts: the int16 window [-2048, 2048) (where residual codes live) in LDS, one
// global atomic per touched bin and block; other symbols straight to global memory.
constexpr int kRansHot = 4096;
__global__ __launch_bounds__(256) void k_rans_hist(const uint16_t* sym, int32_t n, uint32_t* cnt) {
  __shared__ uint32_t hot[kRansHot];
  for (int i = threadIdx.x; i < kRansHot; i += blockDim.x) hot[i] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = sym[i];
    const uint32_t b = (v + kRansHot / 2) & 0xFFFFu;
    if (b < (uint32_t)kRansHot)
      atomicAdd(&hot[b], 1u);
    else
      atomicAdd(&cnt[v], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kRansHot; i += blockDim.x)
    if (hot[i]) atomicAdd(&cnt[(i - kRansHot / 2) & 0xFFFF], hot[i]);
}

// Symbol counts with the whole alphabet privatised in LDS: two passes over the stream, each
// counting one half of the 16-bit range in 32768 LDS bins (128 KiB), then one global
// atomic per non-empty bin and workgroup.  Used where the device grants that much LDS.
constexpr int kRansHalf = 1 << 15;
__global__ __launch_bounds__(1024) void k_rans_hist_lds(const uint16_t* sym, int32_t n, uint32_t* cnt) {
  extern __shared__ uint32_t bins[];
  for (uint32_t half = 0; half < 2; ++half) {
    for (int i = threadIdx.x; i < kRansHalf; i += blockDim.x) bins[i] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const uint32_t v = sym[i];
      if ((v >> 15) == half) atomicAdd(&bins[v & (kRansHalf - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRansHalf; i += blockDim.x)
      if (bins[i]) atomicAdd(&cnt[(half << 15) | (uint32_t)i], bins[i]);
    __syncthreads();
  }
}

// Thread t of the one 1024-thread workgroup owns the 64 consecutive symbols 64 t .. 64 t + 63,
// read and written as 16 four-symbol (16-byte) groups.
__device__ __forceinline__ uint4 rans_group(const uint32_t* a, int g) {
  return reinterpret_cast<const uint4*>(a + threadIdx.x * 64)[g];
}

// cum[v] = sum of freq[u], u < v, over the 2^16 symbols; cum[2^16] = the total; with enc_tab
// also the encoder's (f_s, C_s) entries (one 8-byte gather per coded symbol).
__device__ __forceinline__ void rans_cumulate(const uint32_t* freq, uint32_t* cum, int* lds,
                                              uint64_t* enc_tab = nullptr) {
  const int t = threadIdx.x;
  uint32_t local = 0;
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    const uint4 q = rans_group(freq, g);
    local += q.x + q.y + q.z + q.w;
  }
  int total;
  uint32_t run = (uint32_t)block_excl_scan((int)local, lds, total);
  uint4* out = reinterpret_cast<uint4*>(cum + t * 64);
  ulonglong2* eo = reinterpret_cast<ulonglong2*>(enc_tab + t * 64);
  for (int g = 0; g < 16; ++g) {
    const uint4 q = rans_group(freq, g);
    const uint4 c = make_uint4(run, run + q.x, run + q.x + q.y, run + q.x + q.y + q.z);
    run = c.w + q.w;
    out[g] = c;
    if (enc_tab) {
      eo[2 * g] = make_ulonglong2((uint64_t)q.x | ((uint64_t)c.x << 32), (uint64_t)q.y | ((uint64_t)c.y << 32));
      eo[2 * g + 1] = make_ulonglong2((uint64_t)q.z | ((uint64_t)c.z << 32), (uint64_t)q.w | ((uint64_t)c.w << 32));
    }
  }
  if (t == 0) cum[kRansM] = (uint32_t)total;
}

// floor(c (2^16 - K) / n) for c > 0, at least 1: an estimate from a double reciprocal made
// exact by integer correction steps (c (2^16 - K) < 2^47: the products stay in 64 bits).
__device__ __forceinline__ uint32_t rans_norm(uint32_t c, uint64_t mk, int32_t n, double r) {
  if (!c) return 0u;
  const uint64_t num = (uint64_t)c * mk;
  uint64_t q = (uint64_t)((double)c * r);
  while (q > 0 && q * (uint64_t)n > num) --q;
  while ((q + 1) * (uint64_t)n <= num) ++q;
  return q > 0 ? (uint32_t)q : 1u;
}

// The model: f_s = max(1, floor(c_s (2^16 - K) / n)) for the K occurring symbols, the
// remainder to the most frequent one (ties: the smaller symbol); then the cumulative table
// and the encoder's entries.
__global__ __launch_bounds__(1024) void k_rans_model(const uint32_t* cnt, int32_t n, uint32_t* freq,
                                                     uint32_t* cum, uint64_t* enc_tab) {
  __shared__ int lds[40];
  __shared__ unsigned long long best[1024];
  __shared__ uint32_t ksum[1024];
  const int t = threadIdx.x;
  uint32_t k = 0;
  unsigned long long key = 0;
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    const uint4 q = rans_group(cnt, g);
    const uint32_t c4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t v = t * 64 + g * 4 + j;
      k += c4[j] ? 1u : 0u;
      const unsigned long long kv = ((unsigned long long)c4[j] << 16) | (0xFFFFu - v);
      if (c4[j] && kv > key) key = kv;
    }
  }
  ksum[t] = k;
  best[t] = key;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      ksum[t] += ksum[t + o];
      if (best[t + o] > best[t]) best[t] = best[t + o];
    }
    __syncthreads();
  }
  const uint64_t mk = (uint64_t)kRansM - ksum[0];
  const uint32_t top = 0xFFFFu - (uint32_t)(best[0] & 0xFFFFu);
  const double r = n > 0 ? (double)mk / (double)n : 0.0;
  __syncthreads();
  uint32_t local = 0;
  uint4* fo = reinterpret_cast<uint4*>(freq + t * 64);
  for (int g = 0; g < 16; ++g) {
    const uint4 q = rans_group(cnt, g);
    const uint4 f = make_uint4(rans_norm(q.x, mk, n, r), rans_norm(q.y, mk, n, r), rans_norm(q.z, mk, n, r),
                               rans_norm(q.w, mk, n, r));
    local += f.x + f.y + f.z + f.w;
    fo[g] = f;
  }
  ksum[t] = local;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) ksum[t] += ksum[t + o];
    __syncthreads();
  }
  if (t == 0 && n > 0) freq[top] += kRansM - ksum[0];
  __syncthreads();
  rans_cumulate(freq, cum, lds, enc_tab);
}

__global__ __launch_bounds__(1024) void k_rans_cum(const uint32_t* freq, uint32_t* cum) {
  __shared__ int lds[40];
  rans_cumulate(freq, cum, lds);
}

// One thread per lane: the lane's symbols last to first, words written backwards into the
// lane's own buffer of S + 2 words; len[l] = words written.  Symbols and their (f, C)
// entries are loaded kRansBatch at a time, so the memory latency is paid once per batch
// and not on the state's dependency chain.
constexpr int kRansBatch = 8;
__global__ __launch_bounds__(256) void k_rans_enc(const uint16_t* sym, int32_t n, int64_t lanes,
                                                  const uint64_t* enc_tab, uint16_t* buf, int32_t* len) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= lanes) return;
  const int32_t count = rans_lane_count(n, l);
  const int64_t first = rans_chunk_first(l);
  uint16_t* out = buf + l * (kRansLaneSymbols + 2);
  int p = kRansLaneSymbols + 2;
  uint32_t x = kRansL;
  for (int m0 = count - 1; m0 >= 0; m0 -= kRansBatch) {
    uint32_t sb[kRansBatch];
    uint64_t eb[kRansBatch];
#pragma unroll
    for (int u = 0; u < kRansBatch; ++u) {
      const int m = m0 - u;
      sb[u] = m >= 0 ? sym[first + (int64_t)kRansLanesPerChunk * m] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kRansBatch; ++u) eb[u] = m0 - u >= 0 ? enc_tab[sb[u]] : 1ull;
#pragma unroll
    for (int u = 0; u < kRansBatch; ++u) {
      if (m0 - u < 0) break;
      const uint32_t f = (uint32_t)eb[u];
      const uint32_t c = (uint32_t)(eb[u] >> 32);
      if ((uint64_t)x >= ((uint64_t)f << 16)) {
        out[--p] = (uint16_t)(x & 0xFFFFu);
        x >>= 16;
      }
      x = ((x / f) << 16) + (x % f) + c;
    }
  }
  if (count > 0) {
    out[--p] = (uint16_t)(x & 0xFFFFu);
    out[--p] = (uint16_t)(x >> 16);
  }
  len[l] = kRansLaneSymbols + 2 - p;
}

// One wave per lane: its words to words[lane_off[l] ...]; nothing beyond the capacity.
__global__ __launch_bounds__(256) void k_rans_copy(const uint16_t* buf, const int32_t* len,
                                                   const uint32_t* lane_off, int64_t lanes, uint16_t* words,
                                                   int32_t cap, int32_t* n_words, int32_t* counters) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_words = (int32_t)lane_off[lanes];
  int32_t st = 0;
  for (int64_t l = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; l < lanes; l += nw) {
    const int32_t k = len[l];
    const uint16_t* src = buf + l * (kRansLaneSymbols + 2) + (kRansLaneSymbols + 2 - k);
    const int64_t dst = lane_off[l];
    for (int32_t i = lane; i < k; i += 64) {
      if (dst + i < cap)
        words[dst + i] = src[i];
      else
        st |= kStatusCapacity;
    }
  }
  if (st) atomicOr(&counters[kCntStatus], st);
}

// slot -> (s, f_s, slot - C_s) with s the last symbol with C_s <= slot (the symbol whose
// interval holds the slot): one gather per decoded symbol.
__global__ __launch_bounds__(256) void k_rans_table(const uint32_t* freq, const uint32_t* cum, uint64_t* tab) {
  const uint32_t slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= kRansM) return;
  uint32_t lo = 0, hi = kRansM;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cum[mid] <= slot)
      lo = mid;
    else
      hi = mid;
  }
  tab[slot] = (uint64_t)lo | ((uint64_t)freq[lo] << 16) | ((uint64_t)(slot - cum[lo]) << 33);
}

// One thread per lane: reads the lane's words first to last, writes its symbols.
__global__ __launch_bounds__(256) void k_rans_dec(const uint64_t* tab, const uint32_t* lane_off,
                                                  const uint16_t* words, int32_t cap, int32_t n, int64_t lanes,
                                                  uint16_t* sym, int32_t* counters) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= lanes) return;
  const int32_t count = rans_lane_count(n, l);
  if (count == 0) return;
  const int64_t first = rans_chunk_first(l);
  int64_t p = lane_off[l];
  const int64_t end = min((int64_t)lane_off[l + 1], (int64_t)cap);
  int32_t st = 0;
  if (p < 0 || p + 2 > end) {
    st |= kStatusRange;
    p = end;
  }
  uint32_t x = kRansL;
  if (p + 2 <= end) {
    x = ((uint32_t)words[p] << 16) | words[p + 1];
    p += 2;
  }
  for (int m = 0; m < count; ++m) {
    const uint64_t e = tab[x & 0xFFFFu];
    sym[first + (int64_t)kRansLanesPerChunk * m] = (uint16_t)(e & 0xFFFFu);
    x = (uint32_t)((e >> 16) & 0x1FFFFu) * (x >> 16) + (uint32_t)(e >> 33);
    if (x < kRansL) {
      uint32_t w = 0;
      if (p < end)
        w = words[p++];
      else
        st |= kStatusRange;
      x = (x << 16) | w;
    }
  }
  if (st) atomicOr(&counters[kCntStatus], st);
}

// ------------------------------------------------------------------ cluster finding
// Clusters from zero-suppressed digits (section 5: cluster finding runs on the GPUs before
// the tracking).  The digits' charges are summed into a dense map of every (sector, row,
// pad, time) cell; a digit is a peak if its cell's charge reaches q_min and is a local
// maximum over the 8 neighbouring cells of its row (strictly above the neighbours that come
// earlier in (pad, time) order, at least equal to the later ones); its cluster is the
// charge-weighted centroid and width over the 3 x 3 cells.  Clusters come in the order of
// their peak digits.
struct CfGeo {
  int32_t pads[kRows];        // pads of each row
  int32_t rowoff[kRows + 1];  // first cell of each row within a sector (pads x n_time each)
  float half[kRows];          // half the row width, pads * pitch / 2
  int64_t per_sector;         // cells per sector
  int32_t n_time, q_min;
  float pitch, bin;
};
struct CfDigits {
  int32_t n;
  const uint8_t* sector;
  const int16_t* row;
  const int16_t* pad;
  const int16_t* time;
  const uint16_t* adc;
};
struct CfOut {
  int32_t cap;
  int32_t* n_clusters;
  int32_t* status;
  int32_t* digit;
  uint8_t* sector;
  int16_t* row;
  float *y, *z;
  uint32_t *q_tot, *q_max;
  float *sigma_pad, *sigma_time;
};

// cell index of digit i, or -1 if it lies outside the pad plane
__device__ __forceinline__ int64_t cf_cell(const CfGeo& G, const CfDigits& D, int64_t i, int& s, int& r, int& p,
                                           int& t) {
  s = D.sector[i];
  r = D.row[i];
  p = D.pad[i];
  t = D.time[i];
  if (s >= kSectors || r < 0 || r >= kRows || p < 0 || p >= G.pads[r] || t < 0 || t >= G.n_time) return -1;
  return (int64_t)s * G.per_sector + G.rowoff[r] + (int64_t)p * G.n_time + t;
}

__device__ __forceinline__ uint32_t cf_at(const uint32_t* map, const CfGeo& G, int64_t base, int r, int p, int t) {
  return (p >= 0 && p < G.pads[r] && t >= 0 && t < G.n_time) ? map[base + (int64_t)p * G.n_time + t] : 0u;
}

__device__ __forceinline__ bool cf_peak(const uint32_t* map, const CfGeo& G, int64_t base, int r, int p, int t) {
  const uint32_t q = cf_at(map, G, base, r, p, t);
  if (q < (uint32_t)G.q_min) return false;
#pragma unroll
  for (int dp = -1; dp <= 1; ++dp)
#pragma unroll
    for (int dt = -1; dt <= 1; ++dt) {
      if (dp == 0 && dt == 0) continue;
      const uint32_t qn = cf_at(map, G, base, r, p + dp, t + dt);
      const bool before = dp < 0 || (dp == 0 && dt < 0);
      if (before ? !(q > qn) : !(q >= qn)) return false;
    }
  return true;
}

// The cells the digits touched back to zero, so that the next call on the same workspace
// need not clear the whole map.
__global__ __launch_bounds__(256) void k_cf_clear(CfGeo G, CfDigits D, uint32_t* map) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  int s, r, p, t;
  const int64_t c = cf_cell(G, D, i, s, r, p, t);
  if (c >= 0) map[c] = 0u;
}

__global__ __launch_bounds__(256) void k_cf_fill(CfGeo G, CfDigits D, uint32_t* map, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  int s, r, p, t;
  const int64_t c = cf_cell(G, D, i, s, r, p, t);
  if (c < 0)
    atomicOr(status, kStatusRange);
  else
    atomicAdd(map + c, (uint32_t)D.adc[i]);
}

// Peaks per tile of kScanTile digits (item q of thread j: digit tile * kScanTile + q * 256 + j,
// so the digit loads coalesce); peak[i] = 1 marks them for the write pass.
__global__ __launch_bounds__(kScanThreads) void k_cf_count(CfGeo G, CfDigits D, const uint32_t* map,
                                                           uint8_t* peak, int32_t* bsum) {
  __shared__ int lds[40];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  int c = 0;
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t i = base + (int64_t)q * kScanThreads;
    if (i >= D.n) break;
    int s, r, p, t;
    const int64_t cell = cf_cell(G, D, i, s, r, p, t);
    const bool pk = cell >= 0 && cf_peak(map, G, cell - (int64_t)p * G.n_time - t, r, p, t);
    peak[i] = pk ? 1 : 0;
    c += pk ? 1 : 0;
  }
  int total;
  block_excl_scan(c, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// exclusive offsets of the tiles' peaks; *total = all peaks
__global__ __launch_bounds__(1024) void k_cf_tiles(int32_t* bsum, int32_t ntiles, int32_t* total) {
  __shared__ int lds[40];
  int carry = 0;
  for (int c = 0; c < ntiles; c += blockDim.x) {
    const int i = c + threadIdx.x;
    const int v = i < ntiles ? bsum[i] : 0;
    int tot;
    const int e = block_excl_scan(v, lds, tot);
    if (i < ntiles) bsum[i] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// The clusters of a tile's peaks: thread j takes the tile's digits 8 j .. 8 j + 7 (one block
// scan gives each thread the rank of its first peak) and writes a cluster per marked digit.
__global__ __launch_bounds__(kScanThreads) void k_cf_write(CfGeo G, CfDigits D, const uint32_t* map,
                                                           const uint8_t* peak, const int32_t* bsum,
                                                           const int32_t* total, CfOut O) {
  __shared__ int lds[40];
  if (blockIdx.x == 0 && threadIdx.x == 0) *O.n_clusters = *total;
  const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t mask = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q)
    if (first + q < D.n && peak[first + q]) mask |= 1u << q;
  int tot;
  int64_t pos = (int64_t)bsum[blockIdx.x] + block_excl_scan(__popc(mask), lds, tot);
  int32_t st = 0;
  for (; mask; mask &= mask - 1, ++pos) {
    const int64_t i = first + __ffs(mask) - 1;
    if (pos >= O.cap) {
      st |= kStatusCapacity;
      continue;
    }
    int s, r, p, t;
    const int64_t cell = cf_cell(G, D, i, s, r, p, t);
    const int64_t rb = cell - (int64_t)p * G.n_time - t;
    int64_t Q = 0, Sp = 0, St = 0, Spp = 0, Stt = 0;
#pragma unroll
    for (int dp = -1; dp <= 1; ++dp)
#pragma unroll
      for (int dt = -1; dt <= 1; ++dt) {
        const int64_t qn = cf_at(map, G, rb, r, p + dp, t + dt);
        Q += qn;
        Sp += qn * dp;
        St += qn * dt;
        Spp += qn * dp * dp;
        Stt += qn * dt * dt;
      }
    const float fq = (float)Q;
    const float mp = div_rn((float)Sp, fq), mt = div_rn((float)St, fq);
    const float vp = div_rn((float)Spp, fq) - mp * mp, vt = div_rn((float)Stt, fq) - mt * mt;
    const float az = ((float)t + mt + 0.5f) * G.bin;
    O.digit[pos] = (int32_t)i;
    O.sector[pos] = (uint8_t)s;
    O.row[pos] = (int16_t)r;
    O.y[pos] = ((float)p + mp + 0.5f) * G.pitch - G.half[r];
    O.z[pos] = s < kHalf ? az : -az;
    O.q_tot[pos] = (uint32_t)Q;
    O.q_max[pos] = cf_at(map, G, rb, r, p, t);
    O.sigma_pad[pos] = sqrt_rn(vp > 0.f ? vp : 0.f);
    O.sigma_time[pos] = sqrt_rn(vt > 0.f ? vt : 0.f);
  }
  if (st) atomicOr(O.status, st);
}

// ------------------------------------------------------------------ test hooks
__global__ void k_links_to_input(const int32_t* a, const int32_t* b, const GHit* gh, int32_t* oa,
                                 int32_t* ob, Bound hi_b) {
  const int32_t hi = hi_b.get();
  const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= hi) return;
  const int32_t i = gh[h].idx;
  if (oa) oa[i] = a[h] >= 0 ? gh[a[h]].idx : -1;
  if (ob) ob[i] = b[h] >= 0 ? gh[b[h]].idx : -1;
}

__global__ void k_copy_tracklets(TrackletView V, const GHit* gh, const int32_t* toff, int32_t T,
                                 int32_t* start, int32_t* hits, float* state) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  start[t] = gh[V.start[t]].idx;
  const int n = V.nhits[t];
  for (int q = 0; q < n; ++q) hits[toff[t] + q] = gh[V.hits[(int64_t)t * kHitStride + q]].idx;
  for (int i = 0; i < 21; ++i) state[(int64_t)t * 21 + i] = V.state[(int64_t)t * kStateStride + i];
}

// The weights in input order, as 64-bit keys (n_hits << 32) | (2^32-1 - global id).
__global__ void k_hitw_to_input(const uint32_t* w, const GHit* gh, const int32_t* T_off, uint64_t* out,
                                Bound hi_b) {
  const int32_t hi = hi_b.get();
  const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= hi) return;
  const GHit H = ldh(gh + h);
  const uint32_t k = w[h];
  uint64_t v = 0ull;
  if (k != 0u) {
    const int32_t t = key_tracklet(k, T_off, H.slot);
    v = ((uint64_t)(k >> 24) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)t);
  }
  out[H.idx] = v;
}

__global__ void k_copy_selected(const int32_t* sel_from, const int32_t* sel_off, const int32_t* sel_hits,
                                const GHit* gh, int32_t K, int32_t* tr, int32_t* off, int32_t* hits) {
  const int32_t kk = blockIdx.x * blockDim.x + threadIdx.x;
  if (kk > K) return;
  off[kk] = sel_off[kk];
  if (kk == K) return;
  tr[kk] = sel_from[kk];
  for (int32_t q = sel_off[kk]; q < sel_off[kk + 1]; ++q) hits[q] = gh[sel_hits[q]].idx;
}

__global__ void k_debug_propagate(const float* in, float* out, int32_t n, Consts k) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* a = in + (int64_t)i * 22;
  State S;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    S.P[q] = a[q];
    S.L[q] = 0.f;
  }
#pragma unroll
  for (int q = 0; q < 15; ++q) S.C[q] = a[5 + q];
  const bool ok = propagate(S, a[20], a[21], k);
  float* o = out + (int64_t)i * 26;
  o[0] = ok ? 1.f : 0.f;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    o[1 + q] = S.P[q];
    o[6 + q] = S.L[q];
  }
#pragma unroll
  for (int q = 0; q < 15; ++q) o[11 + q] = S.C[q];
}

__global__ void k_debug_update(const float* in, float* out, int32_t n, Consts k) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* a = in + (int64_t)i * 27;
  State S;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    S.P[q] = a[q];
    S.L[q] = a[5 + q];
  }
#pragma unroll
  for (int q = 0; q < 15; ++q) S.C[q] = a[10 + q];
  float chi2 = 0.f;
  const bool ok = kf_update(S, a[25], a[26], k, &chi2);
  float* o = out + (int64_t)i * 27;
  o[0] = ok ? 1.f : 0.f;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    o[1 + q] = S.P[q];
    o[6 + q] = S.L[q];
  }
#pragma unroll
  for (int q = 0; q < 15; ++q) o[11 + q] = S.C[q];
  o[26] = chi2;
}

// Plain streaming copy (16-byte vectors, grid-stride): measures achievable HBM bandwidth
// and calibrates the hardware traffic counters.
__global__ __launch_bounds__(256) void k_copy_probe(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_members(const GHit* gh, int32_t* out, Bound hi_b) {
  const int32_t hi = hi_b.get();
  const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < hi) out[h] = gh[h].idx;
}

}  // namespace

// ==================================================================== host runtime
namespace {

struct Layout {
  // capacities
  int64_t N = 0;
  int32_t J = 0, S = 0;
  int64_t capCells = 0;
  int32_t capT = 0, capK = 0, capH = 0, capE = 0, nzb = 1;
  int64_t bsumN = 0;
  size_t bytes = 0;
  // arrays
  // grid build: slot of each input cluster and its rank there, the non-empty slots
  // (count first), the clusters in slot order
  int32_t *ckey, *srank, *slot_list, *slot_cnt, *slot_off, *ncell, *cell_base, *cell_off;
  int4* srec;
  uint32_t *zmin, *zmax;
  SlotGrid* sg;
  GHit* gh;
  float2* gyz;
  int32_t *up_raw, *dn_raw, *up, *dn, *fid, *start, *posg, *order;
  uint8_t *flag, *flagg;  // chain starts in input and grid order
  int32_t *trk_hits, *trk_n;
  float* trk_state;
  uint32_t* hitw;
  int32_t *own, *accf, *kid, *hoff, *sel_off, *sel_hits, *sel_from;
  // downward extension: slots of the found hits, the hits, their counts, the claims, and the
  // extended hit lists (the tracks' lists from then on)
  int32_t capX = 0;
  int32_t *ext_off, *ext_hits, *ext_n, *xn, *xsel_off, *xsel_hits;
  uint32_t* claim;
  float *fitrow, *fitchi2;
  int32_t* fitndf;
  int32_t *T_off, *K_off, *counters, *bsum;
  int4* cmp;         // compression: (y, z, record word, unused) per cluster
  uint8_t* cmp_free;  // compression: 1 while no track holds the cluster
  // rANS: symbol counts, cumulative frequencies, slot -> symbol table, lane lengths and
  // the lanes' word buffers (each lane writes backwards into its own S + 2 words)
  uint32_t *rans_cnt, *rans_cum;
  uint64_t* rans_t64;  // encode: (f_s, C_s) per symbol; decode: (s, f_s, slot - C_s) per slot
  int32_t* rans_len;
  uint16_t* rans_buf;
  int64_t rans_lanesN = 0;
  // merge
  float *bucket_z, *link_t0;
  int32_t *trk_event, *bucket_cnt, *bucket_off, *bucket_fill, *bucket_trk, *chain_next, *chain_prev,
      *head_list, *keep, *outn, *oid, *ooff;
  uint64_t *bestA, *bestB;
};

template <class T> void carve(char*& p, T*& out, int64_t count, size_t& total, bool do_set) {
  const size_t b = ((size_t)std::max<int64_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
  if (do_set) out = (T*)p;
  p += b;
  total += b;
}

void layout(Layout& L, int64_t N, int32_t J, float cpc, char* base, bool set) {
  L.N = N;
  L.J = J;
  L.S = J * kSlotsPerJob;
  L.capCells = (int64_t)std::ceil((double)N * (double)cpc) + L.S + 2;
  L.capT = (int32_t)std::min<int64_t>(N / 8 + 1024, N + 1024);
  L.capK = L.capT;
  L.capH = (int32_t)(N + 1);
  L.nzb = std::max(1, std::min(2048, 4194304 / std::max(1, J * kSectors)));
  L.capE = J * kSectors * 3 * L.nzb;
  const int64_t big = std::max<int64_t>(
      {N + 1, L.capCells + 1, (int64_t)L.S + 1, (int64_t)L.capT + 1, (int64_t)L.capE + 1});
  L.bsumN = big / kScanTile + 4;
  char* p = base;
  size_t t = 0;
  carve(p, L.ckey, N, t, set);
  carve(p, L.srec, N, t, set);
  carve(p, L.slot_list, L.S + 1, t, set);
  carve(p, L.slot_cnt, L.S + 1, t, set);
  carve(p, L.slot_off, L.S + 1, t, set);
  carve(p, L.zmin, L.S, t, set);
  carve(p, L.zmax, L.S, t, set);
  carve(p, L.sg, L.S, t, set);
  carve(p, L.ncell, L.S + 1, t, set);
  carve(p, L.cell_base, L.S + 1, t, set);
  carve(p, L.cell_off, L.capCells + 1, t, set);
  carve(p, L.srank, N, t, set);
  carve(p, L.gh, N, t, set);
  carve(p, L.gyz, N, t, set);
  carve(p, L.up_raw, N, t, set);
  carve(p, L.dn_raw, N, t, set);
  carve(p, L.up, N, t, set);
  carve(p, L.dn, N, t, set);
  carve(p, L.flag, N + 1, t, set);
  carve(p, L.fid, N + 1, t, set);
  carve(p, L.start, L.capT, t, set);
  carve(p, L.flagg, N + 1, t, set);
  carve(p, L.posg, N + 1, t, set);
  carve(p, L.order, L.capT, t, set);
  carve(p, L.trk_hits, (int64_t)kHitStride * L.capT, t, set);
  carve(p, L.trk_n, L.capT, t, set);
  carve(p, L.trk_state, (int64_t)kStateStride * L.capT, t, set);
  carve(p, L.hitw, N, t, set);
  carve(p, L.own, L.capT + 1, t, set);
  carve(p, L.accf, L.capT + 1, t, set);
  carve(p, L.kid, L.capT + 1, t, set);
  carve(p, L.hoff, L.capT + 1, t, set);
  carve(p, L.sel_off, L.capK + 1, t, set);
  carve(p, L.sel_hits, L.capH, t, set);
  carve(p, L.sel_from, L.capK, t, set);
  L.capX = (int32_t)(N + 1);
  carve(p, L.ext_off, L.capK + 1, t, set);
  carve(p, L.ext_n, L.capK + 1, t, set);
  carve(p, L.ext_hits, L.capX, t, set);
  carve(p, L.claim, N, t, set);
  carve(p, L.xn, L.capK + 1, t, set);
  carve(p, L.xsel_off, L.capK + 1, t, set);
  carve(p, L.xsel_hits, L.capH, t, set);
  carve(p, L.fitrow, (int64_t)kFitStride * L.capK, t, set);
  carve(p, L.fitchi2, L.capK, t, set);
  carve(p, L.fitndf, L.capK, t, set);
  carve(p, L.T_off, J + 1, t, set);
  carve(p, L.K_off, J + 1, t, set);
  carve(p, L.counters, kNumCounters, t, set);
  carve(p, L.bsum, L.bsumN, t, set);
  carve(p, L.trk_event, L.capK, t, set);
  carve(p, L.bucket_cnt, L.capE + 1, t, set);
  carve(p, L.bucket_off, L.capE + 1, t, set);
  carve(p, L.bucket_fill, L.capE + 1, t, set);
  carve(p, L.bucket_trk, 2 * (int64_t)L.capK, t, set);  // a track may be in a sector and a membrane bucket
  carve(p, L.bucket_z, 2 * (int64_t)L.capK, t, set);
  carve(p, L.link_t0, L.capK, t, set);
  carve(p, L.chain_next, L.capK, t, set);
  carve(p, L.chain_prev, L.capK, t, set);
  carve(p, L.head_list, L.capK, t, set);
  carve(p, L.keep, L.capK + 1, t, set);
  carve(p, L.outn, L.capK + 1, t, set);
  carve(p, L.oid, L.capK + 1, t, set);
  carve(p, L.ooff, L.capK + 1, t, set);
  carve(p, L.bestA, L.capK, t, set);
  carve(p, L.bestB, L.capK, t, set);
  carve(p, L.cmp, N, t, set);
  carve(p, L.cmp_free, N, t, set);
  L.rans_lanesN = rans_lanes(N);
  carve(p, L.rans_cnt, kRansM, t, set);
  carve(p, L.rans_cum, kRansM + 1, t, set);
  carve(p, L.rans_t64, kRansM, t, set);
  carve(p, L.rans_len, L.rans_lanesN + 1, t, set);
  carve(p, L.rans_buf, L.rans_lanesN * (kRansLaneSymbols + 2), t, set);
  L.bytes = t + 256;
}

int blocks_for(int64_t n, int threads) {
  const int64_t b = (n + threads - 1) / threads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 30));
}

}  // namespace

struct tpc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  tpc_params p;
  tpc_tuning tune;
  Consts k;
  int mode = TPC_MODE_BATCHED;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  Layout L;
  bool laid_out = false;
  // bound inputs
  tpc_clusters in{};
  tpc_jobs jobs{};
  std::vector<int32_t> job_off_h;
  int stage = 0;  // last completed stage
  std::string err;
  int32_t* pinned = nullptr;  // host-pinned counters for tpc_sync
  bool lds_count_ok = false;  // the device grants the LDS of k_grid_count_lds
  bool lds_hist_ok = false;   // ... and the 128 KiB of k_rans_hist_lds
  bool static_pending = false;  // tpc_rans_encode_static ran since the last tpc_sync
  void* cf_clean_ws = nullptr;  // cluster-finding workspace whose charge map this context left zero
  int64_t cf_clean_cells = 0;
  // graph cache (batched modes): the chain is captured once per set of buffers
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<uintptr_t> gkey;
  bool capturing = false;
  // per-kernel timing with HIP events on the context's stream
  bool prof = false;
  struct Mark {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  double prof_ms[TPC_PROF_KERNELS] = {};
  int32_t prof_n[TPC_PROF_KERNELS] = {};
};

namespace {

hipEvent_t take_event(tpc_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
// Bracket the launches between prof_begin and prof_end with events on the stream.
int prof_begin(tpc_ctx* c, int id) {
  if (!c->prof || c->capturing) return -1;
  tpc_ctx::Mark m{id, take_event(c), take_event(c)};
  (void)hipEventRecord(m.a, c->stream);
  c->marks.push_back(m);
  return (int)c->marks.size() - 1;
}
void prof_end(tpc_ctx* c, int h) {
  if (h < 0) return;
  (void)hipEventRecord(c->marks[h].b, c->stream);
}

int fail(tpc_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                       \
      return TPC_E_HIP;                                                                     \
    }                                                                                       \
  } while (0)

void make_consts(const tpc_params& p, Consts& k) {
  for (int r = 0; r < kRows; ++r) k.x[r] = (float)(85.0 + (double)r * 160.0 / 151.0);
  k.cb = (float)(-0.299792458e-2 * (double)p.bz);
  const double a = 20.0 * 3.14159265358979323846 / 180.0;
  k.cos20 = (float)std::cos(a);
  k.sin20 = (float)std::sin(a);
  k.tan10 = (float)std::tan(a / 2.0);
  k.vy = p.sigma_y * p.sigma_y;
  k.vz = p.sigma_z * p.sigma_z;
  k.cut2 = p.link_cut * p.link_cut;
  k.cut2_above = std::nextafter(k.cut2, INFINITY);
  k.smax = p.smax;
  k.win_dy_slope = p.win_dy_slope;
  k.win_dy_const = p.win_dy_const;
  k.win_dz_slope = p.win_dz_slope;
  k.win_dz_const = p.win_dz_const;
  k.link_cut = p.link_cut;
  k.nwin = p.nwin;
  k.chi2_follow = p.chi2_follow;
  k.max_miss = p.max_miss;
  k.min_hits = p.min_hits;
  k.prior0[0] = p.cy0; k.prior0[1] = p.cz0; k.prior0[2] = p.cs0; k.prior0[3] = p.ct0; k.prior0[4] = p.ck0;
  k.prior1[0] = p.cy1; k.prior1[1] = p.cz1; k.prior1[2] = p.cs1; k.prior1[3] = p.ct1; k.prior1[4] = p.ck1;
  k.merge_edge = p.merge_edge;
  k.chi2_merge = p.chi2_merge;
  k.merge_dz = p.merge_dz;
  k.v_drift = p.v_drift;
  k.membrane = p.merge_membrane;
}

Bound hb(int32_t v) { return Bound{nullptr, v, INT32_MAX}; }
// Workgroups (of 4 waves) for a grid-stride loop with one wave per item: enough to fill
// the device 8 workgroups deep, no more than the items need.
int wave_grid(tpc_ctx* c, int64_t items) {
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  return (int)std::max<int64_t>(1, std::min<int64_t>((items + 3) / 4, (int64_t)ncu * 32));
}
Bound db(const int32_t* p) { return Bound{p, 0, INT32_MAX}; }
Bound dbc(const int32_t* p, int32_t cap) { return Bound{p, 0, cap}; }

void fill_i32(tpc_ctx* c, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return;
  const int b = blocks_for(n, 256);
  hipLaunchKernelGGL(k_fill_i32, dim3(std::min(b, 65536)), dim3(256), 0, c->stream, p, n, v);
}

// exclusive scan over [lo, hi) (bound <= host upper bound of hi-lo)
// base_from_out: continue from the total a previous scan left in out[lo]
// bsum: block sums, (bound / kScanTile + 1) entries (nullptr: the workspace's)
template <typename T>
void scan(tpc_ctx* c, const T* in, int32_t* out, Bound lo, Bound hi, int64_t bound, bool base_from_out,
          int32_t* bsum = nullptr) {
  if (!bsum) bsum = c->L.bsum;
  const int nb = (int)std::max<int64_t>(1, (bound + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kScanThreads), 0, c->stream, in, lo, hi, bsum);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, c->stream, bsum, lo, hi,
                     (int32_t)base_from_out, out);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3(nb), dim3(kScanThreads), 0, c->stream, in, out, lo, hi, bsum);
}

In make_in(tpc_ctx* c) {
  In in;
  in.sector = c->in.sector;
  in.row = c->in.row;
  in.y = c->in.y;
  in.z = c->in.z;
  in.job_off = c->jobs.job_off;
  in.n_jobs = c->jobs.n_jobs;
  return in;
}
GridView make_grid(tpc_ctx* c) {
  Layout& L = c->L;
  return GridView{L.gh, L.sg, L.cell_base, L.cell_off, L.gyz};
}
TrackletView make_tv(tpc_ctx* c) {
  Layout& L = c->L;
  return TrackletView{L.start, L.up_raw, L.dn_raw, L.up, L.trk_hits, L.trk_n, L.trk_state, L.hitw, L.T_off,
                      L.capT};
}
// The tracks' hit lists: the selection's, or after the downward extension (when enabled)
// the extended ones.
const int32_t* trk_off(tpc_ctx* c, bool extended) {
  return extended && c->p.ext_down ? c->L.xsel_off : c->L.sel_off;
}
const int32_t* trk_hits(tpc_ctx* c, bool extended) {
  return extended && c->p.ext_down ? c->L.xsel_hits : c->L.sel_hits;
}

FitView make_fv(tpc_ctx* c, bool with_chain, bool extended) {
  Layout& L = c->L;
  return FitView{L.sel_from, trk_off(c, extended), trk_hits(c, extended), with_chain ? L.chain_next : nullptr,
                 with_chain ? L.chain_prev : nullptr, L.link_t0, L.fitrow, L.fitchi2, L.fitndf, L.capK};
}

// ---- stage launch sequences over the job range [j0, j1)
void launch_grid(tpc_ctx* c, int j0, int j1) {
  Layout& L = c->L;
  const int32_t* jo = c->jobs.job_off;
  const int64_t nbound = c->job_off_h[j1] - c->job_off_h[j0];
  const int32_t s0 = j0 * kSlotsPerJob, s1 = j1 * kSlotsPerJob;
  In in = make_in(c);
  // clear per-slot counters
  hipLaunchKernelGGL(k_fill_range_i32, dim3(blocks_for(s1 - s0, 256)), dim3(256), 0, c->stream, L.slot_cnt,
                     hb(s0), hb(s1), 0);
  hipLaunchKernelGGL(k_fill_range_i32, dim3(blocks_for(s1 - s0, 256)), dim3(256), 0, c->stream,
                     (int32_t*)L.zmin, hb(s0), hb(s1), -1);
  hipLaunchKernelGGL(k_fill_range_i32, dim3(blocks_for(s1 - s0, 256)), dim3(256), 0, c->stream,
                     (int32_t*)L.zmax, hb(s0), hb(s1), 0);
  if (c->lds_count_ok) {
    hipLaunchKernelGGL(k_grid_count_lds, dim3(blocks_for(nbound, kCountTile)), dim3(kCountThreads),
                       3 * kSlotsPerJob * sizeof(uint32_t), c->stream, in, db(jo + j0), db(jo + j1), L.ckey,
                       L.srank, L.slot_cnt, L.zmin, L.zmax, L.counters);
  } else {
    hipLaunchKernelGGL(k_grid_count, dim3(blocks_for(nbound, 256)), dim3(256), 0, c->stream, in,
                       db(jo + j0), db(jo + j1), L.ckey, L.srank, L.slot_cnt, L.zmin, L.zmax, L.counters);
  }
  // slot offsets in grid order (base: clusters of earlier jobs)
  scan(c, L.slot_cnt, L.slot_off, hb(s0), hb(s1), s1 - s0, j0 != 0);
  hipLaunchKernelGGL(k_fill_range_i32, dim3(1), dim3(64), 0, c->stream, L.slot_list, hb(kListCount),
                     hb(kListCount + 1), 0);
  hipLaunchKernelGGL(k_slot_geometry, dim3(blocks_for(s1 - s0, 256)), dim3(256), 0, c->stream, L.slot_cnt,
                     L.zmin, L.zmax, L.sg, L.ncell, L.slot_list, s0, s1, c->k, c->tune.cells_per_cluster);
  scan(c, L.ncell, L.cell_base, hb(s0), hb(s1), s1 - s0, j0 != 0);
  hipLaunchKernelGGL(k_slot_cellbase, dim3(blocks_for(s1 - s0, 256)), dim3(256), 0, c->stream, L.sg, L.cell_base,
                     s0, s1);
  // clusters in slot order, then each slot sorted by cell
  hipLaunchKernelGGL(k_slot_scatter, dim3(blocks_for(nbound, kCountTile)), dim3(kCountThreads), 0, c->stream, in,
                     db(jo + j0), db(jo + j1), L.ckey, L.srank, L.slot_off, L.srec);
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  const SlotSort ss{L.srec, L.cell_off, L.gh, L.gyz};
  hipLaunchKernelGGL(k_cell_sort, dim3((int)std::max<int64_t>(1, std::min<int64_t>(s1 - s0, (int64_t)ncu * 4))),
                     dim3(kSortThreads), 0, c->stream, ss, L.slot_list, L.slot_cnt, L.slot_off, L.sg, L.cell_base,
                     s1);
}

void launch_links(tpc_ctx* c, int j0, int j1) {
  Layout& L = c->L;
  const int64_t nbound = c->job_off_h[j1] - c->job_off_h[j0];
  const int32_t s0 = j0 * kSlotsPerJob, s1 = j1 * kSlotsPerJob;
  const Bound lo = db(L.slot_off + s0), hi = db(L.slot_off + s1);
  const int bl = c->tune.block_links > 0 ? c->tune.block_links : 256;
  const int pm = prof_begin(c, TPC_PROF_LINKS);
  hipLaunchKernelGGL(k_links, dim3(blocks_for(nbound, bl)), dim3(bl), 0, c->stream, make_grid(c), lo, hi,
                     L.up_raw, L.dn_raw, c->k);
  prof_end(c, pm);
  // clean links, starts flagged in input order (-> ranked ids) and grid order, weights cleared
  const int32_t* jo = c->jobs.job_off;
  const bool grid_order = c->tune.tracklet_order == 1;
  hipLaunchKernelGGL(k_fill_range_u8, dim3(blocks_for(nbound, 256)), dim3(256), 0, c->stream, L.flag,
                     db(jo + j0), db(jo + j1), (uint8_t)0);
  hipLaunchKernelGGL(k_clean_starts, dim3(blocks_for(nbound, 256)), dim3(256), 0, c->stream, L.up_raw, L.dn_raw,
                     L.gh, L.up, L.dn, L.flag, grid_order ? L.flagg : nullptr, L.hitw, lo, hi);
  scan(c, L.flag, L.fid, db(jo + j0), db(jo + j1), nbound, j0 != 0);
  hipLaunchKernelGGL(k_job_offsets, dim3(blocks_for(j1 - j0, 256)), dim3(256), 0, c->stream, L.fid, jo,
                     L.T_off, j0, j1, (int32_t)L.N);
  if (grid_order) scan(c, L.flagg, L.posg, lo, hi, nbound, j0 != 0);
  hipLaunchKernelGGL(k_write_starts, dim3(blocks_for(nbound, 256)), dim3(256), 0, c->stream, L.up, L.dn,
                     grid_order ? L.flagg : nullptr, L.gh, L.fid, grid_order ? L.posg : nullptr, L.T_off, L.start,
                     grid_order ? L.order : nullptr, L.capT, lo, hi, db(L.T_off + j1), L.counters);
}

int64_t tbound(tpc_ctx* c, int j0, int j1) {
  const int64_t n = c->job_off_h[j1] - c->job_off_h[j0];
  return std::min<int64_t>(n / 3 + 1, c->L.capT);
}

void launch_tracklets(tpc_ctx* c, int j0, int j1) {
  Layout& L = c->L;
  const Bound lo = dbc(L.T_off + j0, L.capT), hi = dbc(L.T_off + j1, L.capT);
  const int bt = c->tune.block_tracklets > 0 ? c->tune.block_tracklets : 256;
  const int64_t tb = tbound(c, j0, j1);
  // tracklets that overflow the work list are never built: their lengths read as 0
  hipLaunchKernelGGL(k_fill_range_i32, dim3(blocks_for(tb, 256)), dim3(256), 0, c->stream, L.trk_n, lo, hi, 0);
  const size_t keep_bytes = (size_t)kLaneWords * bt * sizeof(float);
  const int pm = prof_begin(c, TPC_PROF_TRACKLETS);
  if (c->mode == TPC_MODE_PERSISTENT && c->tune.persistent_waves > 0) {
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    const int waves = ncu * c->tune.persistent_waves;
    const int blocks = std::max(kXcds, (waves * 64 / bt) / kXcds * kXcds);
    fill_i32(c, L.counters + kCntQueue, kXcds, 0);
    if (c->tune.persistent_refill)
      hipLaunchKernelGGL(k_tracklets_persistent, dim3(blocks), dim3(bt), keep_bytes, c->stream, make_grid(c),
                         make_tv(c), c->tune.tracklet_order ? L.order : nullptr, lo, hi, c->k,
                         L.counters + kCntQueue);
    else
      hipLaunchKernelGGL(k_tracklets_chunked, dim3(blocks), dim3(bt), keep_bytes, c->stream, make_grid(c),
                         make_tv(c), c->tune.tracklet_order ? L.order : nullptr, lo, hi, c->k,
                         L.counters + kCntQueue);
  } else {
    hipLaunchKernelGGL(k_tracklets, dim3(blocks_for(tb, bt)), dim3(bt), keep_bytes, c->stream,
                       make_grid(c), make_tv(c), c->tune.tracklet_order ? L.order : nullptr, lo, hi, c->k);
  }
  prof_end(c, pm);
}

void launch_select(tpc_ctx* c, int j0, int j1) {
  Layout& L = c->L;
  const Bound lo = dbc(L.T_off + j0, L.capT), hi = dbc(L.T_off + j1, L.capT);
  const int64_t tb = tbound(c, j0, j1);
  const int64_t nbound = c->job_off_h[j1] - c->job_off_h[j0];
  const int32_t s0 = j0 * kSlotsPerJob, s1 = j1 * kSlotsPerJob;
  hipLaunchKernelGGL(k_fill_range_i32, dim3(blocks_for(tb, 256)), dim3(256), 0, c->stream, L.own, lo, hi, 0);
  hipLaunchKernelGGL(k_own_count, dim3(blocks_for(nbound, kOwnChunk)), dim3(kOwnThreads), 0, c->stream, L.hitw,
                     L.gh, L.T_off, L.slot_off, L.own, j0, j1, db(L.slot_off + s0), db(L.slot_off + s1), L.capT);
  hipLaunchKernelGGL(k_select_count, dim3(blocks_for(tb, 256)), dim3(256), 0, c->stream, make_tv(c), lo, hi,
                     L.own, L.accf, c->k);
  // the scans run over [T_off[j0], min(T_off[j1], capT)); clamp via a copy of the bound
  scan(c, L.accf, L.kid, lo, hi, tb, j0 != 0);
  scan(c, L.own, L.hoff, lo, hi, tb, j0 != 0);
  hipLaunchKernelGGL(k_select_write, dim3(blocks_for(tb, 256)), dim3(256), 0, c->stream, make_tv(c), lo, hi,
                     L.accf, L.kid, L.hoff, L.sel_from, L.sel_off, L.capK, L.counters);
  hipLaunchKernelGGL(k_select_hits, dim3(wave_grid(c, tb)), dim3(256), 0, c->stream, make_tv(c), L.kid, j0, j1,
                     L.sel_from, L.sel_off, L.sel_hits, L.capK, L.capH, L.counters);
  hipLaunchKernelGGL(k_select_finish, dim3(1), dim3(1), 0, c->stream, L.kid, L.hoff, hi, L.capT, L.sel_off,
                     L.capK, L.counters);
}

}  // namespace

// ==================================================================== C ABI
extern "C" {

int tpc_params_default(tpc_params* p) {
  if (!p) return TPC_E_ARG;
  p->win_dy_slope = 1.0f;
  p->win_dy_const = 0.5f;
  p->win_dz_slope = 2.0f;
  p->win_dz_const = 0.5f;
  p->link_cut = 1.0f;
  p->cy0 = 1.0f; p->cz0 = 1.0f; p->cs0 = 0.25f; p->ct0 = 0.25f; p->ck0 = 100.0f;
  p->cy1 = 1.0f; p->cz1 = 1.0f; p->cs1 = 1e-3f; p->ct1 = 1e-3f; p->ck1 = 1.0f;
  p->sigma_y = 0.1f;
  p->sigma_z = 0.1f;
  p->nwin = 3.0f;
  p->chi2_follow = 15.0f;
  p->max_miss = 4;
  p->min_hits = 10;
  p->smax = 0.95f;
  p->bz = 0.5f;
  p->merge_edge = 5.0f;
  p->chi2_merge = 50.0f;
  p->merge_dz = 20.0f;
  p->v_drift = 2.58f;
  p->ext_down = 0;
  p->merge_membrane = 0;
  return TPC_OK;
}

int tpc_params_preset(tpc_params* p, int preset) {
  if (!p || (preset != TPC_PRESET_ASYNC && preset != TPC_PRESET_SYNC)) return TPC_E_ARG;
  tpc_params_default(p);
  if (preset == TPC_PRESET_SYNC) {
    p->merge_edge = -1.0f;
    p->ext_down = 1;
  } else {
    p->merge_membrane = 1;
  }
  return TPC_OK;
}

int tpc_tuning_default(tpc_tuning* t) {
  if (!t) return TPC_E_ARG;
  t->cells_per_cluster = 2.0f;
  t->block_links = 256;
  t->block_tracklets = 64;
  t->persistent_waves = 16;
  t->use_graph = 1;
  t->tracklet_order = 1;
  t->persistent_refill = 0;
  return TPC_OK;
}

static bool params_ok(const tpc_params& p) {
  const float f[] = {p.win_dy_slope, p.win_dy_const, p.win_dz_slope, p.win_dz_const, p.link_cut, p.cy0,
                     p.cz0, p.cs0, p.ct0, p.ck0, p.cy1, p.cz1, p.cs1, p.ct1, p.ck1, p.sigma_y, p.sigma_z,
                     p.nwin, p.chi2_follow, p.smax, p.bz, p.merge_edge, p.chi2_merge, p.merge_dz, p.v_drift};
  for (float v : f)
    if (!std::isfinite(v)) return false;
  return p.link_cut > 0.f && std::isnormal(p.link_cut * p.link_cut) && p.sigma_y > 0.f && p.sigma_z > 0.f &&
         p.nwin > 0.f && p.smax > 0.f && p.smax < 1.f &&
         p.min_hits >= 3 && p.max_miss >= 1 && p.merge_dz >= 0.f && p.v_drift > 0.f &&
         (p.ext_down == 0 || p.ext_down == 1) && (p.merge_membrane == 0 || p.merge_membrane == 1);
}

// the reason of the last failed tpc_ctx_create (read through tpc_last_error(NULL))
static thread_local char g_create_err[256] = "null context";

namespace {
void scratch_setup(int device);
}

int tpc_ctx_create(tpc_ctx** out, int device, void* stream, const tpc_params* p) {
  if (!out) return TPC_E_ARG;
  if (p && !params_ok(*p)) return TPC_E_ARG;
  tpc_ctx* c = new tpc_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (p) c->p = *p; else tpc_params_default(&c->p);
  tpc_tuning_default(&c->tune);
  make_consts(c->p, c->k);
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->pinned, 64 * sizeof(int32_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    std::snprintf(g_create_err, sizeof(g_create_err), "tpc_ctx_create on device %d: %s", device,
                  hipGetErrorString(e));
    delete c;
    return TPC_E_HIP;
  }
  {
    int lds_max = 0;
    const int need = 3 * kSlotsPerJob * (int)sizeof(uint32_t);
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        lds_max >= need) {
      c->lds_count_ok = hipFuncSetAttribute((const void*)k_grid_count_lds,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, need) == hipSuccess;
    }
    const int need_h = kRansHalf * (int)sizeof(uint32_t);
    if (lds_max >= need_h)
      c->lds_hist_ok = hipFuncSetAttribute((const void*)k_rans_hist_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           need_h) == hipSuccess;
    (void)hipGetLastError();
  }
  scratch_setup(device);
  *out = c;
  return TPC_OK;
}

void tpc_ctx_destroy(tpc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto& m : c->marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

int tpc_set_stream(tpc_ctx* c, void* s) {
  if (!c) return TPC_E_ARG;
  c->stream = (hipStream_t)s;
  return TPC_OK;
}

int tpc_set_mode(tpc_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 2) return TPC_E_ARG;
  c->mode = mode;
  return TPC_OK;
}

int tpc_set_tuning(tpc_ctx* c, const tpc_tuning* t) {
  if (!c || !t || !(t->cells_per_cluster > 0.f) || t->cells_per_cluster > 8.f) return TPC_E_ARG;
  if (t->block_links % 64 || t->block_links <= 0 || t->block_links > 256) return TPC_E_ARG;
  if (t->block_tracklets % 64 || t->block_tracklets <= 0 || t->block_tracklets > 256) return TPC_E_ARG;
  if (t->tracklet_order != 0 && t->tracklet_order != 1) return TPC_E_ARG;
  if (t->persistent_refill != 0 && t->persistent_refill != 1) return TPC_E_ARG;
  c->tune = *t;
  c->laid_out = false;
  return TPC_OK;
}

const char* tpc_last_error(const tpc_ctx* c) { return c ? c->err.c_str() : g_create_err; }

size_t tpc_workspace_size(const tpc_ctx* c, int64_t n, int32_t J) {
  if (!c || n < 0 || J <= 0) return 0;
  Layout L;
  layout(L, std::max<int64_t>(n, 1), J, c->tune.cells_per_cluster, nullptr, false);
  return L.bytes;
}

int tpc_bind_workspace(tpc_ctx* c, void* p, size_t bytes) {
  if (!c || !p) return TPC_E_ARG;
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  c->ws = p;
  c->ws_bytes = bytes;
  c->own_ws = false;
  c->laid_out = false;
  return TPC_OK;
}

int tpc_grid_build(tpc_ctx* c, const tpc_clusters* cl, const tpc_jobs* jb) {
  if (!c || !cl || !jb) return TPC_E_ARG;
  if (cl->n < 0 || jb->n_jobs <= 0 || !jb->job_off || !jb->job_off_host) return fail(c, TPC_E_ARG, "bad sizes");
  if (cl->n > 0 && (!cl->sector || !cl->row || !cl->y || !cl->z)) return fail(c, TPC_E_ARG, "null cluster array");
  if (jb->job_off_host[0] != 0 || jb->job_off_host[jb->n_jobs] != cl->n)
    return fail(c, TPC_E_ARG, "job_off must start at 0 and end at n");
  for (int j = 0; j < jb->n_jobs; ++j)
    if (jb->job_off_host[j + 1] < jb->job_off_host[j]) return fail(c, TPC_E_ARG, "job_off not ascending");
  if ((int64_t)jb->n_jobs * kSlotsPerJob > (int64_t)INT32_MAX / 2) return fail(c, TPC_E_ARG, "too many jobs");
  if (!c->capturing) HIPCHK(c, hipSetDevice(c->device));
  c->in = *cl;
  c->jobs = *jb;
  c->job_off_h.assign(jb->job_off_host, jb->job_off_host + jb->n_jobs + 1);
  const int64_t N = std::max<int32_t>(cl->n, 1);
  Layout L;
  layout(L, N, jb->n_jobs, c->tune.cells_per_cluster, nullptr, false);
  if (!c->ws || c->ws_bytes < L.bytes) {
    if (c->ws && !c->own_ws) return fail(c, TPC_E_CAPACITY, "bound workspace too small");
    if (c->ws) (void)hipFree(c->ws);
    c->ws = nullptr;
    HIPCHK(c, hipMalloc(&c->ws, L.bytes));
    c->ws_bytes = L.bytes;
    c->own_ws = true;
  }
  char* base = (char*)(((uintptr_t)c->ws + 255) & ~(uintptr_t)255);
  layout(c->L, N, jb->n_jobs, c->tune.cells_per_cluster, base, true);
  c->laid_out = true;
  fill_i32(c, c->L.counters, kNumCounters, 0);
  fill_i32(c, c->L.T_off, 1, 0);
  fill_i32(c, c->L.K_off, 1, 0);
  const int pm = prof_begin(c, TPC_PROF_GRID);
  if (c->mode == TPC_MODE_PLAIN) {
    for (int j = 0; j < jb->n_jobs; ++j) launch_grid(c, j, j + 1);
  } else {
    launch_grid(c, 0, jb->n_jobs);
  }
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  c->stage = 1;
  return TPC_OK;
}

int tpc_find_neighbours(tpc_ctx* c, int32_t* up, int32_t* down) {
  if (!c || c->stage < 1) return fail(c, TPC_E_ARG, "grid not built");
  const int J = c->jobs.n_jobs;
  if (c->mode == TPC_MODE_PLAIN) {
    for (int j = 0; j < J; ++j) launch_links(c, j, j + 1);
  } else {
    launch_links(c, 0, J);
  }
  if (up || down)
    hipLaunchKernelGGL(k_links_to_input, dim3(blocks_for(c->L.N, 256)), dim3(256), 0, c->stream, c->L.up,
                       c->L.dn, c->L.gh, up, down, db(c->L.slot_off + c->L.S));
  HIPCHK(c, hipGetLastError());
  c->stage = 2;
  return TPC_OK;
}

int tpc_construct_tracklets(tpc_ctx* c, int32_t* n_tracklets) {
  if (!c || c->stage < 2) return fail(c, TPC_E_ARG, "links not found");
  const int J = c->jobs.n_jobs;
  if (c->mode == TPC_MODE_PLAIN) {
    for (int j = 0; j < J; ++j) launch_tracklets(c, j, j + 1);
  } else {
    launch_tracklets(c, 0, J);
  }
  if (n_tracklets)
    HIPCHK(c, hipMemcpyAsync(n_tracklets, c->L.T_off + J, sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipGetLastError());
  c->stage = 3;
  return TPC_OK;
}

int tpc_select_tracks(tpc_ctx* c, int32_t* n_selected) {
  if (!c || c->stage < 3) return fail(c, TPC_E_ARG, "tracklets not built");
  const int J = c->jobs.n_jobs;
  const int pm = prof_begin(c, TPC_PROF_SELECT);
  if (c->mode == TPC_MODE_PLAIN) {
    for (int j = 0; j < J; ++j) {
      launch_select(c, j, j + 1);
      // K_off[j+1] = number of tracks after job j
      hipLaunchKernelGGL(k_job_offsets, dim3(1), dim3(64), 0, c->stream, c->L.kid, c->L.T_off, c->L.K_off,
                         j, j + 1, c->L.capT);
    }
  } else {
    launch_select(c, 0, J);
    hipLaunchKernelGGL(k_job_offsets, dim3(blocks_for(J, 256)), dim3(256), 0, c->stream, c->L.kid,
                       c->L.T_off, c->L.K_off, 0, J, c->L.capT);
  }
  prof_end(c, pm);
  if (n_selected)
    HIPCHK(c, hipMemcpyAsync(n_selected, c->L.counters + kCntSelected, sizeof(int32_t),
                             hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipGetLastError());
  c->stage = 4;
  return TPC_OK;
}

int tpc_fit_merge(tpc_ctx* c, tpc_tracks* out) {
  if (!c || c->stage < 4) return fail(c, TPC_E_ARG, "tracks not selected");
  if (!out || !out->hit_off || !out->hits || !out->param || !out->cov || !out->x_ref || !out->chi2 ||
      !out->ndf || !out->sector || !out->job || !out->tracklet || out->cap_tracks < 0 || out->cap_hits < 0)
    return fail(c, TPC_E_ARG, "bad output struct");
  Layout& L = c->L;
  const int J = c->jobs.n_jobs;
  const int64_t kb = std::min<int64_t>(c->L.N / 3 + 1, L.capK);
  const int pm = prof_begin(c, TPC_PROF_FIT_MERGE);
  // per-track fit (no merge yet): the track range is [K_off[j0], K_off[j1])
  auto fit_range = [&](int j0, int j1, int64_t bound) {
    hipLaunchKernelGGL(k_fit, dim3(blocks_for(bound, 128)), dim3(128), 0, c->stream, make_grid(c), make_tv(c),
                       make_fv(c, false, false), dbc(L.K_off + j0, L.capK), dbc(L.K_off + j1, L.capK), c->k);
  };
  if (c->mode == TPC_MODE_PLAIN) {
    for (int j = 0; j < J; ++j) fit_range(j, j + 1, std::min<int64_t>((c->job_off_h[j + 1] - c->job_off_h[j]) / 3 + 1, L.capK));
  } else {
    fit_range(0, J, kb);
  }
  const Bound klo = hb(0), khi = dbc(L.counters + kCntSelected, L.capK);
  // ---- downward extension below the innermost hits (all selected tracks at once)
  if (c->p.ext_down) {
    const ExtView E{L.K_off, L.accf, L.ext_off, L.ext_hits, L.ext_n, L.claim, L.xn, L.capX};
    const FitView F = make_fv(c, false, false);
    hipLaunchKernelGGL(k_ext_rows, dim3(blocks_for(kb, 256)), dim3(256), 0, c->stream, make_grid(c), F, E,
                       L.ext_n, klo, khi);
    scan(c, L.ext_n, L.ext_off, klo, khi, kb, false);
    fill_i32(c, (int32_t*)L.claim, L.N, 0);
    hipLaunchKernelGGL(k_ext_search, dim3(blocks_for(kb, 128)), dim3(128), 0, c->stream, make_grid(c),
                       make_tv(c), F, E, klo, khi, c->k);
    hipLaunchKernelGGL(k_ext_keep, dim3(blocks_for(kb, 128)), dim3(128), 0, c->stream, make_grid(c), make_tv(c),
                       F, E, klo, khi, c->k);
    scan(c, L.xn, L.xsel_off, klo, khi, kb, false);
    hipLaunchKernelGGL(k_ext_write, dim3(wave_grid(c, kb)), dim3(256), 0, c->stream, make_grid(c), make_tv(c), F,
                       E, L.xsel_off, L.xsel_hits, klo, khi, L.capH, L.counters, c->k);
  }
  // ---- merge across adjacent sectors of one event
  const int nev = J;
  const int64_t nbk = (int64_t)nev * kSectors * 3 * L.nzb;
  fill_i32(c, L.bucket_cnt, nbk + 1, 0);
  fill_i32(c, L.bucket_fill, nbk + 1, 0);
  fill_i32(c, L.chain_next, L.capK, -1);
  fill_i32(c, L.chain_prev, L.capK, -1);
  fill_i32(c, (int32_t*)L.bestA, 2 * (int64_t)L.capK, -1);
  fill_i32(c, (int32_t*)L.bestB, 2 * (int64_t)L.capK, -1);
  fill_i32(c, L.counters + kCntMergeCand, 1, 0);
  hipLaunchKernelGGL(k_track_event, dim3(blocks_for(kb, 256)), dim3(256), 0, c->stream, L.sel_from, L.start,
                     trk_off(c, true), trk_hits(c, true), L.gh, c->jobs.job_event, L.fitndf, L.fitrow, L.trk_event,
                     L.bucket_cnt, klo,
                     khi, L.capK, nev, L.nzb, c->k, L.counters);
  scan(c, L.bucket_cnt, L.bucket_off, hb(0), hb((int32_t)nbk), nbk, false);
  MergeView M{L.trk_event, L.bucket_cnt, L.bucket_off, L.bucket_fill, L.bucket_trk, L.bucket_z, L.bestA,
              L.bestB, L.chain_next, L.chain_prev, L.head_list, L.counters + kCntMergeCand, L.link_t0, nev,
              L.nzb, c->p.merge_dz};
  hipLaunchKernelGGL(k_track_bucket, dim3(blocks_for(kb, 256)), dim3(256), 0, c->stream, L.sel_from, L.start,
                     trk_off(c, true), trk_hits(c, true), L.gh, L.fitndf, L.fitrow, M, klo, khi, L.capK, c->k);
  hipLaunchKernelGGL(k_merge_candidates, dim3(blocks_for(kb, 128)), dim3(128), 0, c->stream, make_grid(c),
                     make_tv(c), make_fv(c, false, true), M, klo, khi, c->k);
  hipLaunchKernelGGL(k_merge_links, dim3(blocks_for(kb, 256)), dim3(256), 0, c->stream, make_grid(c), make_tv(c),
                     make_fv(c, false, true), M, klo, khi, L.capK, c->k);
  hipLaunchKernelGGL(k_merge_heads, dim3(blocks_for(kb, 256)), dim3(256), 0, c->stream, M, klo, khi, L.capK,
                     L.keep);
  hipLaunchKernelGGL(k_fit_heads, dim3(blocks_for(kb, 128)), dim3(128), 0, c->stream, make_grid(c),
                     make_tv(c), make_fv(c, true, true), L.head_list, L.counters + kCntMergeCand, c->k);
  // ---- output compaction in track-id order
  hipLaunchKernelGGL(k_out_count, dim3(blocks_for(kb, 256)), dim3(256), 0, c->stream, make_fv(c, true, true),
                     L.keep, L.outn, klo, khi);
  scan(c, L.keep, L.oid, klo, khi, kb, false);
  scan(c, L.outn, L.ooff, klo, khi, kb, false);
  OutView O{out->cap_tracks, out->cap_hits, out->n_tracks, out->hit_off, out->hits, out->param, out->cov,
            out->x_ref, out->chi2, out->ndf, out->sector, out->job, out->tracklet, out->t0};
  hipLaunchKernelGGL(k_out_write, dim3(wave_grid(c, kb)), dim3(256), 0, c->stream, make_grid(c), make_tv(c),
                     make_fv(c, true, true), O, L.keep, L.oid, L.ooff, klo, khi, L.counters, c->k);
  if (O.t0)
    hipLaunchKernelGGL(k_out_t0, dim3(std::min(blocks_for(kb, 256), 65536)), dim3(256), 0, c->stream, make_grid(c),
                       make_tv(c), make_fv(c, true, true), O, L.keep, L.oid, klo, khi, c->k);
  hipLaunchKernelGGL(k_out_finish, dim3(1), dim3(1), 0, c->stream, L.oid, L.ooff, khi, L.capK, O, L.counters);
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  c->stage = 5;
  return TPC_OK;
}

static int run_chain(tpc_ctx* c, const tpc_clusters* cl, const tpc_jobs* jb, tpc_tracks* out) {
  int rc = tpc_grid_build(c, cl, jb);
  if (rc) return rc;
  if ((rc = tpc_find_neighbours(c, nullptr, nullptr))) return rc;
  if ((rc = tpc_construct_tracklets(c, nullptr))) return rc;
  if ((rc = tpc_select_tracks(c, nullptr))) return rc;
  return tpc_fit_merge(c, out);
}

int tpc_run(tpc_ctx* c, const tpc_clusters* cl, const tpc_jobs* jb, tpc_tracks* out) {
  if (!c || !cl || !jb || !out) return TPC_E_ARG;
  const bool graph = c->tune.use_graph && c->mode != TPC_MODE_PLAIN && !c->prof;
  if (!graph) return run_chain(c, cl, jb, out);
  // The captured chain depends on every pointer and size it was built with.
  std::vector<uintptr_t> key = {(uintptr_t)c->stream, (uintptr_t)cl->n, (uintptr_t)cl->sector,
                                (uintptr_t)cl->row, (uintptr_t)cl->y, (uintptr_t)cl->z,
                                (uintptr_t)jb->n_jobs, (uintptr_t)jb->job_off, (uintptr_t)jb->job_event,
                                (uintptr_t)c->ws, (uintptr_t)c->ws_bytes, (uintptr_t)c->mode,
                                (uintptr_t)out->cap_tracks, (uintptr_t)out->cap_hits,
                                (uintptr_t)out->n_tracks, (uintptr_t)out->hit_off, (uintptr_t)out->hits,
                                (uintptr_t)out->param, (uintptr_t)out->cov, (uintptr_t)out->x_ref,
                                (uintptr_t)out->chi2, (uintptr_t)out->ndf, (uintptr_t)out->sector,
                                (uintptr_t)out->job, (uintptr_t)out->tracklet, (uintptr_t)out->t0};
  for (int j = 0; j <= jb->n_jobs; ++j) key.push_back((uintptr_t)(uint32_t)jb->job_off_host[j]);
  // ... and on the launch shapes
  {
    uint32_t w[sizeof(tpc_tuning) / 4];
    std::memcpy(w, &c->tune, sizeof(w));
    for (uint32_t v : w) key.push_back(v);
  }
  if (!c->gexec || key != c->gkey) {
    if (c->gexec) {
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
    if (c->graph) {
      (void)hipGraphDestroy(c->graph);
      c->graph = nullptr;
    }
    HIPCHK(c, hipSetDevice(c->device));
    // workspace sizing happens outside the capture (it may allocate)
    if (c->own_ws || !c->ws) {
      Layout L;
      layout(L, std::max<int32_t>(cl->n, 1), jb->n_jobs, c->tune.cells_per_cluster, nullptr, false);
      if (!c->ws || c->ws_bytes < L.bytes) return run_chain(c, cl, jb, out);
    }
    if (c->stream == nullptr) return run_chain(c, cl, jb, out);  // the null stream cannot be captured
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    const int rc = run_chain(c, cl, jb, out);
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(c, TPC_E_HIP, "graph capture failed");
    c->graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->gkey = key;
  } else {
    // host-side state of the stages (bound inputs) as the capture left it
    c->in = *cl;
    c->jobs = *jb;
  }
  HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  c->stage = 5;
  return TPC_OK;
}

int tpc_profile(tpc_ctx* c, int enable) {
  if (!c) return TPC_E_ARG;
  c->prof = enable != 0;
  return TPC_OK;
}

int tpc_profile_read(tpc_ctx* c, double* ms, int32_t* launches, int32_t n, int32_t reset) {
  if (!c || n < 0) return TPC_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& m : c->marks) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) {
      c->prof_ms[m.id] += t;
      c->prof_n[m.id] += 1;
    }
    c->event_pool.push_back(m.a);
    c->event_pool.push_back(m.b);
  }
  c->marks.clear();
  for (int i = 0; i < n && i < TPC_PROF_KERNELS; ++i) {
    if (ms) ms[i] = c->prof_ms[i];
    if (launches) launches[i] = c->prof_n[i];
  }
  if (reset)
    for (int i = 0; i < TPC_PROF_KERNELS; ++i) {
      c->prof_ms[i] = 0.0;
      c->prof_n[i] = 0;
    }
  return TPC_OK;
}

namespace {
int32_t* scratch_status(int device);
}

int tpc_sync(tpc_ctx* c) {
  if (!c) return TPC_E_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  c->pinned[kNumCounters] = 0;
  if (c->static_pending) {
    // status of the last tpc_rans_encode_static on this device (the scratch's status word)
    c->static_pending = false;
    if (int32_t* s = scratch_status(c->device))
      HIPCHK(c, hipMemcpyAsync(c->pinned + kNumCounters, s, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  }
  if (!c->laid_out) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int32_t st = c->pinned[kNumCounters];
    if (st & kStatusCapacity) return fail(c, TPC_E_CAPACITY, "capacity exceeded");
    return TPC_OK;
  }
  HIPCHK(c, hipMemcpyAsync(c->pinned, c->L.counters, kNumCounters * sizeof(int32_t), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int32_t st = c->pinned[kCntStatus] | c->pinned[kNumCounters];
  if (st & kStatusCapacity) return fail(c, TPC_E_CAPACITY, "capacity exceeded");
  if (st & kStatusRange) return fail(c, TPC_E_RANGE, "cluster with sector/row out of range or non-finite y/z");
  return TPC_OK;
}

int tpc_counts(tpc_ctx* c, int32_t* dst) {
  if (!c || !dst) return fail(c, TPC_E_ARG, "null argument");
  if (!c->laid_out) return fail(c, TPC_E_ARG, "no tracking run");
  static_assert(kCntStatus == 0 && kCntTracklets == 1 && kCntSelected == 2 && kCntSelHits == 3 &&
                    kCntOut == 4 && kCntOutHits == 5,
                "tpc_counts copies the first six counters in the order tpc.h states");
  HIPCHK(c, hipMemcpyAsync(dst, c->L.counters, 6 * sizeof(int32_t), hipMemcpyDefault, c->stream));
  return TPC_OK;
}

int tpc_get_links_raw(tpc_ctx* c, int32_t* up_raw, int32_t* down_raw) {
  if (!c || c->stage < 2) return TPC_E_ARG;
  hipLaunchKernelGGL(k_links_to_input, dim3(blocks_for(c->L.N, 256)), dim3(256), 0, c->stream, c->L.up_raw,
                     c->L.dn_raw, c->L.gh, up_raw, down_raw, db(c->L.slot_off + c->L.S));
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int tpc_get_rows(tpc_ctx* c, int32_t* slot_off, int32_t* members) {
  if (!c || c->stage < 1) return TPC_E_ARG;
  HIPCHK(c, hipMemcpyAsync(slot_off, c->L.slot_off, ((size_t)c->L.S + 1) * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(k_members, dim3(blocks_for(c->L.N, 256)), dim3(256), 0, c->stream, c->L.gh, members,
                     db(c->L.slot_off + c->L.S));
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int tpc_get_tracklet_counts(tpc_ctx* c, int32_t* T, int64_t* H) {
  if (!c || c->stage < 3 || !T || !H) return TPC_E_ARG;
  int32_t t = 0;
  HIPCHK(c, hipMemcpyAsync(&t, c->L.T_off + c->jobs.n_jobs, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  t = std::min(t, c->L.capT);
  std::vector<int32_t> n(t);
  if (t) HIPCHK(c, hipMemcpy(n.data(), c->L.trk_n, (size_t)t * sizeof(int32_t), hipMemcpyDeviceToHost));
  int64_t s = 0;
  for (int32_t v : n) s += v;
  *T = t;
  *H = s;
  return TPC_OK;
}

int tpc_get_tracklets(tpc_ctx* c, int32_t* start, int32_t* off, int32_t* hits, float* state, uint64_t* w) {
  if (!c || c->stage < 3) return TPC_E_ARG;
  int32_t T;
  int64_t H;
  int rc = tpc_get_tracklet_counts(c, &T, &H);
  if (rc) return rc;
  std::vector<int32_t> n(T), o(T + 1, 0);
  if (T) HIPCHK(c, hipMemcpy(n.data(), c->L.trk_n, (size_t)T * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int i = 0; i < T; ++i) o[i + 1] = o[i] + n[i];
  HIPCHK(c, hipMemcpy(off, o.data(), (size_t)(T + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  if (T)
    hipLaunchKernelGGL(k_copy_tracklets, dim3(blocks_for(T, 256)), dim3(256), 0, c->stream, make_tv(c),
                       c->L.gh, off, T, start, hits, state);
  if (w)
    hipLaunchKernelGGL(k_hitw_to_input, dim3(blocks_for(c->L.N, 256)), dim3(256), 0, c->stream, c->L.hitw,
                       c->L.gh, c->L.T_off, w, db(c->L.slot_off + c->L.S));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TPC_OK;
}

int tpc_get_selected_counts(tpc_ctx* c, int32_t* K, int64_t* H) {
  if (!c || c->stage < 4 || !K || !H) return TPC_E_ARG;
  int32_t v[kNumCounters];
  HIPCHK(c, hipMemcpyAsync(v, c->L.counters, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *K = std::min(v[kCntSelected], c->L.capK);
  *H = v[kCntSelHits];
  return TPC_OK;
}

int tpc_get_selected(tpc_ctx* c, int32_t* tr, int32_t* off, int32_t* hits) {
  if (!c || c->stage < 4) return TPC_E_ARG;
  int32_t K;
  int64_t H;
  int rc = tpc_get_selected_counts(c, &K, &H);
  if (rc) return rc;
  hipLaunchKernelGGL(k_copy_selected, dim3(blocks_for(K + 1, 256)), dim3(256), 0, c->stream, c->L.sel_from,
                     c->L.sel_off, c->L.sel_hits, c->L.gh, K, tr, off, hits);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TPC_OK;
}

namespace {
// ---------------------------------------------------------------- looper leg pairs
// A particle whose circle turns back inside the chamber leaves two tracks: the outgoing
// leg and the return leg, which the tracking follows along increasing x like every track,
// i.e. against the particle's momentum.  Both describe one circle, with opposite signed
// curvature and opposite tan(lambda), and both end at the circle's point farthest from the
// beam line, where the particle turned.  Two fitted tracks of one event and one z side whose
// circles turn inside the chamber (2R < 245 cm / cos 10 deg) pair when those signs are
// opposite and their circle centres (global x, y) and their z carried along the helix to
// the turning point agree within kLegGate each; the score is the sum of the three squared
// differences and pairs are mutual best ones (ties: the smaller output index).
//
// One thread per track.  Loopers go into a hash table of 4-cm cells of the circle centre
// keyed by (event, side, cell), each cell holding a list of its tracks; each looper scans
// the 3 x 3 cells around its own centre.  The order in which the lists were built does not
// matter: the best partner is the smallest (score, index).
constexpr float kLegGate = 3.0f;
constexpr float kLegCell = 4.0f;   // > kLegGate: the 3 x 3 cells hold every candidate
constexpr int kLegSectorsPerSide = 18;
constexpr unsigned long long kLegEmpty = ~0ull;

struct LegConsts {
  float ca[kLegSectorsPerSide], sa[kLegSectorsPerSide];  // sector angle 10 + 20 s degrees
  float cmin;                                            // |C| of a circle with 2R = 245 / cos 10
  float cb;                                              // curvature per unit q/pT
};
struct LegWork {
  float4* geo;              // [cap] circle centre x, y, z at the turning point, signed curvature
  float* tl;                // [cap] tan(lambda)
  unsigned long long* grp;  // [cap] (event, side) of a looper, kLegEmpty otherwise
  int32_t* next;            // [cap] next track of the same cell
  int32_t* arg;             // [cap] best partner or -1
  unsigned long long* key;  // [hmask + 1] cell keys, kLegEmpty when free
  int32_t* head;            // [hmask + 1] first track of the cell
  uint32_t hmask;
};

__device__ __forceinline__ uint32_t leg_hash(unsigned long long k) {
  // the 64-bit finaliser of MurmurHash3
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)k;
}
__device__ __forceinline__ unsigned long long leg_cell(unsigned long long grp, int ix, int iy) {
  return (grp * 4096ull + (unsigned long long)(ix & 4095)) * 4096ull + (unsigned long long)(iy & 4095);
}

__global__ void k_leg_geometry(CmpTracks T, const int32_t* job, const int32_t* job_event, LegWork W, LegConsts LC) {
  const int n = min(*T.n_tracks, T.cap_tracks);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < T.cap_tracks; i += gridDim.x * blockDim.x) {
    W.grp[i] = kLegEmpty;
    W.arg[i] = -1;
    if (i >= n || T.ndf[i] < 0) continue;
    const float* P = T.param + 5 * (int64_t)i;
    const float C = P[4] * LC.cb;
    if (!(fabsf(C) > LC.cmin)) continue;
    const int sec = T.sector[i];
    const float ca = LC.ca[sec % kLegSectorsPerSide], sa = LC.sa[sec % kLegSectorsPerSide];
    const float x = T.x_ref[i], s = P[2];
    const float c = sqrt_rn((1.0f - s) * (1.0f + s));
    const float lx = x - div_rn(s, C), ly = P[0] + div_rn(c, C);
    const float cx = lx * ca - ly * sa, cy = lx * sa + ly * ca;
    if (!isfinite(cx) || !isfinite(cy)) continue;
    // the turning point: the centre moved by R away from the beam line
    const float R = div_rn(1.0f, fabsf(C));
    const float cn = sqrt_rn(cx * cx + cy * cy);
    const float tx = cx + R * div_rn(cx, cn), ty = cy + R * div_rn(cy, cn);
    const float px = x * ca - P[0] * sa, py = x * sa + P[0] * ca;
    const float dx = tx - px, dy = ty - py;
    const float chord = sqrt_rn(dx * dx + dy * dy);
    const float u = fminf(1.0f, chord * fabsf(C) * 0.5f);
    float A, B;
    asinc(u, A, B);
    W.geo[i] = make_float4(cx, cy, P[1] + P[3] * (chord * A), C);
    W.tl[i] = P[3];
    const int ev = job_event ? job_event[job[i]] : job[i];
    const unsigned long long g = (unsigned long long)(uint32_t)ev * 2ull + (sec >= kLegSectorsPerSide ? 1ull : 0ull);
    W.grp[i] = g;
    const unsigned long long k = leg_cell(g, (int)floorf(cx / kLegCell), (int)floorf(cy / kLegCell));
    // at most cap distinct keys in a table of >= 2 cap slots: a free or equal slot exists
    uint32_t h = leg_hash(k) & W.hmask;
    for (;;) {
      const unsigned long long prev = atomicCAS(&W.key[h], kLegEmpty, k);
      if (prev == kLegEmpty || prev == k) break;
      h = (h + 1) & W.hmask;
    }
    W.next[i] = atomicExch(&W.head[h], i);
  }
}

__global__ void k_leg_best(CmpTracks T, LegWork W) {
  const int n = min(*T.n_tracks, T.cap_tracks);
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
    const unsigned long long g = W.grp[a];
    if (g == kLegEmpty) continue;
    const float4 ga = W.geo[a];
    const float ta = W.tl[a];
    const int ix = (int)floorf(ga.x / kLegCell), iy = (int)floorf(ga.y / kLegCell);
    float best = 0.f;
    int arg = -1;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        const unsigned long long k = leg_cell(g, ix + dx, iy + dy);
        uint32_t h = leg_hash(k) & W.hmask;
        unsigned long long kh;
        while ((kh = W.key[h]) != kLegEmpty && kh != k) h = (h + 1) & W.hmask;
        if (kh == kLegEmpty) continue;
        for (int b = W.head[h]; b >= 0; b = W.next[b]) {
          if (b == a || W.grp[b] != g) continue;
          const float4 gb = W.geo[b];
          if (!(ga.w * gb.w < 0.f) || !(ta * W.tl[b] <= 0.f)) continue;
          const float ex = ga.x - gb.x, ey = ga.y - gb.y, ez = ga.z - gb.z;
          if (!(fabsf(ex) <= kLegGate) || !(fabsf(ey) <= kLegGate) || !(fabsf(ez) <= kLegGate)) continue;
          const float sc = (ex * ex + ey * ey) + ez * ez;
          if (arg < 0 || sc < best || (sc == best && b < arg)) {
            best = sc;
            arg = b;
          }
        }
      }
    W.arg[a] = arg;
  }
}

__global__ void k_leg_mutual(CmpTracks T, LegWork W, int32_t* leg) {
  const int n = min(*T.n_tracks, T.cap_tracks);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < T.cap_tracks; i += gridDim.x * blockDim.x) {
    const int b = i < n ? W.arg[i] : -1;
    leg[i] = (b >= 0 && W.arg[b] == i) ? b : -1;
  }
}

size_t leg_align(size_t b) { return (b + 255) & ~(size_t)255; }
uint32_t leg_slots(int32_t cap) {
  uint32_t h = 256;
  while (h < 2u * (uint32_t)cap) h <<= 1;
  return h;
}
bool cmp_tracks_ok(const tpc_tracks* t) {
  return t && t->cap_tracks >= 0 && t->cap_hits >= 0 && t->n_tracks && t->hit_off &&
         (t->cap_hits == 0 || t->hits) &&
         (t->cap_tracks == 0 || (t->param && t->x_ref && t->sector && t->ndf));
}
bool cmp_codes_ok(const tpc_codes* o) {
  return o && o->cap >= 0 && o->n_codes && o->n_attached && (o->cap == 0 || (o->rs && o->ey && o->ez));
}
bool steps_ok(float q_y, float q_z) {
  return q_y > 0.f && q_z > 0.f && std::isfinite(q_y) && std::isfinite(q_z) && std::isfinite(1.0f / q_y) &&
         std::isfinite(1.0f / q_z);
}
CmpTracks tracks_view(const tpc_tracks* t) {
  return CmpTracks{t->n_tracks, t->cap_tracks, t->cap_hits, t->hit_off, t->hits, t->param, t->x_ref, t->sector,
                   t->ndf};
}
CmpCodes codes_view(const tpc_codes* o) {
  return CmpCodes{o->cap, o->n_codes, o->n_attached, o->rs, o->ey, o->ez, o->ez_hi};
}
}  // namespace

int tpc_compress(tpc_ctx* c, const tpc_clusters* in, const tpc_tracks* t, float q_y, float q_z, tpc_codes* out) {
  if (!c) return TPC_E_ARG;
  if (!in || !cmp_tracks_ok(t) || !cmp_codes_ok(out)) return fail(c, TPC_E_ARG, "tpc_compress: null or negative argument");
  if (!steps_ok(q_y, q_z)) return fail(c, TPC_E_ARG, "tpc_compress: quantisation steps must be positive and finite");
  if (in->n < 0 || (in->n > 0 && (!in->sector || !in->row || !in->y || !in->z)))
    return fail(c, TPC_E_ARG, "tpc_compress: invalid cluster list");
  if (!c->laid_out || (int64_t)in->n > c->L.N)
    return fail(c, TPC_E_ARG, "tpc_compress: needs the workspace of a tracking run over at least n clusters");
  HIPCHK(c, hipSetDevice(c->device));
  Layout& L = c->L;
  const float iqy = 1.0f / q_y, iqz = 1.0f / q_z;
  const CmpClusters cl{in->sector, in->row, in->y, in->z, in->n};
  const CmpTracks T = tracks_view(t);
  const CmpCodes O = codes_view(out);
  const int pm = prof_begin(c, TPC_PROF_COMPRESS);
  const int nb = blocks_for(std::max(in->n, 1), 256);
  hipLaunchKernelGGL(k_cmp_pack, dim3(nb), dim3(256), 0, c->stream, cl, L.cmp, L.cmp_free);
  if (t->cap_tracks > 0)
    hipLaunchKernelGGL(k_cmp_tracks, dim3(wave_grid(c, t->cap_tracks)), dim3(256), 0, c->stream, in->n, L.cmp,
                       L.cmp_free, T, O, c->k, iqy, iqz, L.counters);
  // clusters in no track: counts per tile, tile offsets (their sum in fid[n]), records
  const int nt = blocks_for(std::max(in->n, 1), kScanTile);
  hipLaunchKernelGGL(k_cmp_count, dim3(nt), dim3(kScanThreads), 0, c->stream, in->n, L.cmp_free, L.bsum);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, c->stream, L.bsum, Bound{nullptr, 0, INT32_MAX},
                     Bound{nullptr, in->n, INT32_MAX}, 0, L.fid);
  hipLaunchKernelGGL(k_cmp_free, dim3(nt), dim3(kScanThreads), 0, c->stream, in->n, L.cmp, L.cmp_free, T, O,
                     L.bsum, L.fid + in->n, iqy, iqz, L.counters);
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int tpc_decompress(tpc_ctx* c, const tpc_tracks* t, const tpc_codes* in, float q_y, float q_z, uint8_t* sector,
                   int16_t* row, float* y, float* z) {
  if (!c) return TPC_E_ARG;
  if (!cmp_tracks_ok(t) || !cmp_codes_ok(in) || (in->cap > 0 && (!sector || !row || !y || !z)))
    return fail(c, TPC_E_ARG, "tpc_decompress: null or negative argument");
  if (!steps_ok(q_y, q_z)) return fail(c, TPC_E_ARG, "tpc_decompress: quantisation steps must be positive and finite");
  if (!c->laid_out) return fail(c, TPC_E_ARG, "tpc_decompress: needs a context that has run a tracking stage");
  HIPCHK(c, hipSetDevice(c->device));
  const CmpTracks T = tracks_view(t);
  const CmpCodes C = codes_view(in);
  const CmpOut D{sector, row, y, z};
  const int pm = prof_begin(c, TPC_PROF_DECOMPRESS);
  if (t->cap_tracks > 0 && in->cap > 0)
    hipLaunchKernelGGL(k_dcmp_tracks, dim3(wave_grid(c, t->cap_tracks)), dim3(256), 0, c->stream, T, C, D, c->k,
                       q_y, q_z, c->L.counters);
  if (in->cap > 0)
    hipLaunchKernelGGL(k_dcmp_free, dim3(blocks_for(in->cap, 256)), dim3(256), 0, c->stream, C, D, c->k, q_y, q_z,
                       c->L.counters);
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

size_t tpc_pair_legs_workspace_size(int32_t cap_tracks) {
  if (cap_tracks < 0 || cap_tracks > (1 << 28)) return 0;
  const size_t k = (size_t)std::max(cap_tracks, 1), h = leg_slots(cap_tracks);
  return leg_align(k * sizeof(float4)) + leg_align(k * sizeof(float)) + leg_align(k * sizeof(unsigned long long)) +
         2 * leg_align(k * sizeof(int32_t)) + leg_align(h * sizeof(unsigned long long)) + leg_align(h * sizeof(int32_t));
}

int tpc_pair_legs(tpc_ctx* c, const tpc_tracks* t, const int32_t* job_event, void* ws, size_t ws_bytes, int32_t* leg) {
  if (!c) return TPC_E_ARG;
  if (!cmp_tracks_ok(t) || (t->cap_tracks > 0 && (!t->job || !leg)))
    return fail(c, TPC_E_ARG, "tpc_pair_legs: null or negative argument");
  const size_t need = tpc_pair_legs_workspace_size(t->cap_tracks);
  if (need == 0) return fail(c, TPC_E_ARG, "tpc_pair_legs: more than 2^28 tracks");
  if (!ws || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(c, TPC_E_ARG, "tpc_pair_legs: workspace missing, unaligned or smaller than tpc_pair_legs_workspace_size");
  if (t->cap_tracks == 0) return TPC_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const size_t k = (size_t)t->cap_tracks, h = leg_slots(t->cap_tracks);
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += leg_align(bytes);
    return q;
  };
  LegWork W;
  W.geo = reinterpret_cast<float4*>(take(k * sizeof(float4)));
  W.tl = reinterpret_cast<float*>(take(k * sizeof(float)));
  W.grp = reinterpret_cast<unsigned long long*>(take(k * sizeof(unsigned long long)));
  W.next = reinterpret_cast<int32_t*>(take(k * sizeof(int32_t)));
  W.arg = reinterpret_cast<int32_t*>(take(k * sizeof(int32_t)));
  W.key = reinterpret_cast<unsigned long long*>(take(h * sizeof(unsigned long long)));
  W.head = reinterpret_cast<int32_t*>(take(h * sizeof(int32_t)));
  W.hmask = (uint32_t)h - 1;
  LegConsts LC;
  for (int s = 0; s < kLegSectorsPerSide; ++s) {
    const double al = (10.0 + 20.0 * s) * 3.14159265358979323846 / 180.0;
    LC.ca[s] = (float)std::cos(al);
    LC.sa[s] = (float)std::sin(al);
  }
  LC.cmin = (float)(2.0 / (245.0 / std::cos(10.0 * 3.14159265358979323846 / 180.0)));
  LC.cb = c->k.cb;
  const CmpTracks T = tracks_view(t);
  const int pm = prof_begin(c, TPC_PROF_LEGS);
  fill_i32(c, reinterpret_cast<int32_t*>(W.key), 2 * (int64_t)h, -1);
  fill_i32(c, W.head, (int64_t)h, -1);
  const int nb = std::min(blocks_for(t->cap_tracks, 256), 65536);
  hipLaunchKernelGGL(k_leg_geometry, dim3(nb), dim3(256), 0, c->stream, T, t->job, job_event, W, LC);
  hipLaunchKernelGGL(k_leg_best, dim3(nb), dim3(256), 0, c->stream, T, W);
  hipLaunchKernelGGL(k_leg_mutual, dim3(nb), dim3(256), 0, c->stream, T, W, leg);
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int64_t tpc_rans_lanes(int64_t n) { return n < 0 ? -1 : rans_lanes(n); }

int tpc_rans_encode(tpc_ctx* c, const uint16_t* sym, int32_t n, tpc_rans* out) {
  if (!c) return TPC_E_ARG;
  if (!out || n < 0 || (n > 0 && !sym) || out->cap_words < 0 || !out->n_words || !out->freq || !out->lane_off ||
      (out->cap_words > 0 && !out->words))
    return fail(c, TPC_E_ARG, "tpc_rans_encode: null or negative argument");
  if (reinterpret_cast<uintptr_t>(out->freq) % 16)
    return fail(c, TPC_E_ARG, "tpc_rans_encode: freq must be 16-byte aligned");
  if (!c->laid_out || (int64_t)n > c->L.N)
    return fail(c, TPC_E_ARG, "tpc_rans_encode: needs the workspace of a tracking run over at least n clusters");
  HIPCHK(c, hipSetDevice(c->device));
  Layout& L = c->L;
  const int64_t lanes = rans_lanes(n);
  const int pm = prof_begin(c, TPC_PROF_RANS_ENCODE);
  fill_i32(c, reinterpret_cast<int32_t*>(L.rans_cnt), kRansM, 0);
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (n > 0 && c->lds_hist_ok)
    hipLaunchKernelGGL(k_rans_hist_lds, dim3(std::min(blocks_for(n, 1024), ncu)), dim3(1024),
                       kRansHalf * sizeof(uint32_t), c->stream, sym, n, L.rans_cnt);
  else if (n > 0)
    hipLaunchKernelGGL(k_rans_hist, dim3(std::min(blocks_for(n, 256), ncu * 4)), dim3(256), 0, c->stream, sym, n,
                       L.rans_cnt);
  hipLaunchKernelGGL(k_rans_model, dim3(1), dim3(1024), 0, c->stream, L.rans_cnt, n, out->freq, L.rans_cum,
                     L.rans_t64);
  if (lanes > 0) {
    hipLaunchKernelGGL(k_rans_enc, dim3(blocks_for(lanes, 256)), dim3(256), 0, c->stream, sym, n, lanes,
                       L.rans_t64, L.rans_buf, L.rans_len);
    scan(c, L.rans_len, reinterpret_cast<int32_t*>(out->lane_off), Bound{nullptr, 0, INT32_MAX},
         Bound{nullptr, (int32_t)lanes, INT32_MAX}, lanes, false);
  } else {
    fill_i32(c, reinterpret_cast<int32_t*>(out->lane_off), 1, 0);
  }
  hipLaunchKernelGGL(k_rans_copy, dim3(std::max(1, wave_grid(c, lanes))), dim3(256), 0, c->stream, L.rans_buf,
                     L.rans_len, out->lane_off, lanes, out->words, out->cap_words, out->n_words, L.counters);
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int tpc_rans_decode(tpc_ctx* c, const tpc_rans* in, int32_t n, uint16_t* sym) {
  if (!c) return TPC_E_ARG;
  if (!in || n < 0 || (n > 0 && !sym) || in->cap_words < 0 || !in->freq || !in->lane_off ||
      (in->cap_words > 0 && !in->words))
    return fail(c, TPC_E_ARG, "tpc_rans_decode: null or negative argument");
  if (reinterpret_cast<uintptr_t>(in->freq) % 16)
    return fail(c, TPC_E_ARG, "tpc_rans_decode: freq must be 16-byte aligned");
  if (!c->laid_out) return fail(c, TPC_E_ARG, "tpc_rans_decode: needs a context that has run a tracking stage");
  HIPCHK(c, hipSetDevice(c->device));
  Layout& L = c->L;
  const int64_t lanes = rans_lanes(n);
  const int pm = prof_begin(c, TPC_PROF_RANS_DECODE);
  hipLaunchKernelGGL(k_rans_cum, dim3(1), dim3(1024), 0, c->stream, in->freq, L.rans_cum);
  hipLaunchKernelGGL(k_rans_table, dim3(kRansM / 256), dim3(256), 0, c->stream, in->freq, L.rans_cum,
                     L.rans_t64);
  if (lanes > 0)
    hipLaunchKernelGGL(k_rans_dec, dim3(blocks_for(lanes, 256)), dim3(256), 0, c->stream, L.rans_t64,
                       in->lane_off, in->words, in->cap_words, n, lanes, sym, L.counters);
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

// ---- rANS encoding without allocation
// A file-scope device array holds everything the encoder needs beyond its inputs and
// outputs, for streams of up to TPC_RANS_STATIC_MAX_SYMBOLS symbols.  Each device has its
// own copy; host code never uses the array's name as an address, only the pointer that
// hipGetSymbolAddress returned on that device (the name is a host-side stand-in).
constexpr size_t kStaticScratchBytes = size_t(10) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Once per device, with the device current (called from tpc_ctx_create).
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void* ptr = nullptr;
  g_scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (g_scratch_err[device] == hipSuccess) g_scratch[device] = ptr;
  (void)hipGetLastError();
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch[device];
}

struct StaticRans {
  uint32_t* cnt;
  uint32_t* cum;
  uint64_t* t64;
  int32_t* len;
  uint16_t* buf;
  int32_t* bsum;
  int32_t* counters;
};
constexpr int64_t kStaticLanes = (TPC_RANS_STATIC_MAX_SYMBOLS / (kRansLanesPerChunk * kRansLaneSymbols)) *
                                 kRansLanesPerChunk;
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kStaticCntOff = 0;
constexpr size_t kStaticCumOff = kStaticCntOff + al256(kRansM * 4);
constexpr size_t kStaticT64Off = kStaticCumOff + al256((kRansM + 1) * 4);
constexpr size_t kStaticLenOff = kStaticT64Off + al256(kRansM * 8);
constexpr size_t kStaticBufOff = kStaticLenOff + al256((kStaticLanes + 1) * 4);
constexpr size_t kStaticBsumOff = kStaticBufOff + al256(kStaticLanes * (kRansLaneSymbols + 2) * 2);
constexpr size_t kStaticCntrOff = kStaticBsumOff + al256((kStaticLanes / kScanTile + 4) * 4);
constexpr size_t kStaticEnd = kStaticCntrOff + al256(kNumCounters * 4);
static_assert(TPC_RANS_STATIC_MAX_SYMBOLS % (kRansLanesPerChunk * kRansLaneSymbols) == 0,
              "the limit is a whole number of chunks");
static_assert(kStaticEnd <= kStaticScratchBytes, "the encoder's scratch fits the static array");

StaticRans static_rans(void* base) {
  char* b = static_cast<char*>(base);
  return StaticRans{reinterpret_cast<uint32_t*>(b + kStaticCntOff), reinterpret_cast<uint32_t*>(b + kStaticCumOff),
                    reinterpret_cast<uint64_t*>(b + kStaticT64Off), reinterpret_cast<int32_t*>(b + kStaticLenOff),
                    reinterpret_cast<uint16_t*>(b + kStaticBufOff), reinterpret_cast<int32_t*>(b + kStaticBsumOff),
                    reinterpret_cast<int32_t*>(b + kStaticCntrOff)};
}

int32_t* scratch_status(int device) {
  void* p = scratch_ptr(device);
  return p ? static_rans(p).counters + kCntStatus : nullptr;
}
}  // namespace

int tpc_rans_encode_static(tpc_ctx* c, const uint16_t* sym, int32_t n, tpc_rans* out) {
  if (!c) return TPC_E_ARG;
  if (!out || n < 0 || (n > 0 && !sym) || out->cap_words < 0 || !out->n_words || !out->freq || !out->lane_off ||
      (out->cap_words > 0 && !out->words))
    return fail(c, TPC_E_ARG, "tpc_rans_encode_static: null or negative argument");
  if (reinterpret_cast<uintptr_t>(out->freq) % 16)
    return fail(c, TPC_E_ARG, "tpc_rans_encode_static: freq must be 16-byte aligned");
  if ((int64_t)n > TPC_RANS_STATIC_MAX_SYMBOLS)
    return fail(c, TPC_E_ARG, "tpc_rans_encode_static: n exceeds TPC_RANS_STATIC_MAX_SYMBOLS (4194304)");
  void* base = scratch_ptr(c->device);
  if (!base) {
    const hipError_t e = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_err[c->device] : hipErrorInvalidDevice;
    c->err = std::string("tpc_rans_encode_static: no scratch address on this device: ") + hipGetErrorString(e);
    return TPC_E_HIP;
  }
  HIPCHK(c, hipSetDevice(c->device));
  const StaticRans S = static_rans(base);
  const int64_t lanes = rans_lanes(n);
  // the scratch keeps the last call's contents: clear the counts and the status word
  fill_i32(c, reinterpret_cast<int32_t*>(S.cnt), kRansM, 0);
  fill_i32(c, S.counters, kNumCounters, 0);
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (n > 0 && c->lds_hist_ok)
    hipLaunchKernelGGL(k_rans_hist_lds, dim3(std::min(blocks_for(n, 1024), ncu)), dim3(1024),
                       kRansHalf * sizeof(uint32_t), c->stream, sym, n, S.cnt);
  else if (n > 0)
    hipLaunchKernelGGL(k_rans_hist, dim3(std::min(blocks_for(n, 256), ncu * 4)), dim3(256), 0, c->stream, sym, n,
                       S.cnt);
  hipLaunchKernelGGL(k_rans_model, dim3(1), dim3(1024), 0, c->stream, S.cnt, n, out->freq, S.cum, S.t64);
  if (lanes > 0) {
    hipLaunchKernelGGL(k_rans_enc, dim3(blocks_for(lanes, 256)), dim3(256), 0, c->stream, sym, n, lanes, S.t64,
                       S.buf, S.len);
    scan(c, S.len, reinterpret_cast<int32_t*>(out->lane_off), Bound{nullptr, 0, INT32_MAX},
         Bound{nullptr, (int32_t)lanes, INT32_MAX}, lanes, false, S.bsum);
  } else {
    fill_i32(c, reinterpret_cast<int32_t*>(out->lane_off), 1, 0);
  }
  hipLaunchKernelGGL(k_rans_copy, dim3(std::max(1, wave_grid(c, lanes))), dim3(256), 0, c->stream, S.buf, S.len,
                     out->lane_off, lanes, out->words, out->cap_words, out->n_words, S.counters);
  HIPCHK(c, hipGetLastError());
  c->static_pending = true;
  return TPC_OK;
}

int tpc_cf_params_default(tpc_cf_params* p) {
  if (!p) return TPC_E_ARG;
  p->pad_pitch = 0.5f;
  p->time_bin = 0.5f;
  p->n_time = 500;
  p->q_min = 10;
  return TPC_OK;
}

namespace {
bool cf_params_ok(const tpc_cf_params* p) {
  return p && p->pad_pitch > 0.f && p->time_bin > 0.f && std::isfinite(p->pad_pitch) &&
         std::isfinite(p->time_bin) && p->n_time >= 1 && p->n_time <= 32767 && p->q_min >= 1 &&
         p->pad_pitch >= 0.05f;
}
// F1: 2 ceil(x_r tan 10 deg / pitch) pads per row, x_r in double
CfGeo cf_geometry(const tpc_cf_params* p) {
  CfGeo G{};
  const double tan10 = std::tan(10.0 * 3.14159265358979323846 / 180.0);
  int64_t off = 0;
  for (int r = 0; r < kRows; ++r) {
    const double x = 85.0 + (double)r * 160.0 / 151.0;
    G.pads[r] = 2 * (int32_t)std::ceil(x * tan10 / (double)p->pad_pitch);
    G.half[r] = (float)((double)G.pads[r] * (double)p->pad_pitch / 2.0);
    G.rowoff[r] = (int32_t)std::min<int64_t>(off, INT32_MAX);
    off += (int64_t)G.pads[r] * p->n_time;
  }
  G.rowoff[kRows] = (int32_t)std::min<int64_t>(off, INT32_MAX);
  G.per_sector = off;
  G.n_time = p->n_time;
  G.q_min = p->q_min;
  G.pitch = p->pad_pitch;
  G.bin = p->time_bin;
  return G;
}
size_t cf_map_bytes(const CfGeo& G) { return ((size_t)G.per_sector * kSectors * sizeof(uint32_t) + 255) & ~(size_t)255; }
}  // namespace

size_t tpc_cf_workspace_size(const tpc_cf_params* p, int32_t n_digits) {
  if (!cf_params_ok(p) || n_digits < 0) return 0;
  const CfGeo G = cf_geometry(p);
  if (G.per_sector > INT32_MAX) return 0;  // the row offsets are 32-bit
  const int64_t tiles = ((int64_t)n_digits + kScanTile - 1) / kScanTile + 1;
  return cf_map_bytes(G) + (size_t)(tiles + 64) * sizeof(int32_t) + (size_t)n_digits;
}

int tpc_find_clusters(tpc_ctx* c, const tpc_cf_params* p, const tpc_digits* d, void* ws, size_t ws_bytes,
                      tpc_cf_clusters* out) {
  if (!c) return TPC_E_ARG;
  if (!cf_params_ok(p)) return fail(c, TPC_E_ARG, "tpc_find_clusters: invalid parameters");
  if (!d || d->n < 0 || (d->n > 0 && (!d->sector || !d->row || !d->pad || !d->time || !d->adc)))
    return fail(c, TPC_E_ARG, "tpc_find_clusters: invalid digit list");
  if (!out || out->cap < 0 || !out->n_clusters || !out->status ||
      (out->cap > 0 && (!out->digit || !out->sector || !out->row || !out->y || !out->z || !out->q_tot ||
                        !out->q_max || !out->sigma_pad || !out->sigma_time)))
    return fail(c, TPC_E_ARG, "tpc_find_clusters: invalid output");
  const size_t need = tpc_cf_workspace_size(p, d->n);
  if (need == 0) return fail(c, TPC_E_ARG, "tpc_find_clusters: pad plane too large for 32-bit row offsets");
  if (!ws || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(c, TPC_E_ARG, "tpc_find_clusters: workspace missing, unaligned or smaller than tpc_cf_workspace_size");
  HIPCHK(c, hipSetDevice(c->device));
  const CfGeo G = cf_geometry(p);
  uint32_t* map = static_cast<uint32_t*>(ws);
  int32_t* bsum = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + cf_map_bytes(G));
  const int32_t ntiles = (int32_t)(((int64_t)d->n + kScanTile - 1) / kScanTile);
  int32_t* total = bsum + ntiles + 1;
  uint8_t* peak = reinterpret_cast<uint8_t*>(bsum + ntiles + 64);
  const CfDigits D{d->n, d->sector, d->row, d->pad, d->time, d->adc};
  const CfOut O{out->cap, out->n_clusters, out->status, out->digit, out->sector, out->row, out->y, out->z,
                out->q_tot, out->q_max, out->sigma_pad, out->sigma_time};
  const int pm = prof_begin(c, TPC_PROF_CLUSTERS);
  // a workspace this context left clean (same pointer, same plane) needs no full clear
  const bool clean = c->cf_clean_ws == ws && c->cf_clean_cells == G.per_sector * kSectors;
  if (!clean) fill_i32(c, reinterpret_cast<int32_t*>(map), G.per_sector * kSectors, 0);
  fill_i32(c, out->status, 1, 0);
  fill_i32(c, total, 1, 0);
  if (d->n > 0) {
    hipLaunchKernelGGL(k_cf_fill, dim3(blocks_for(d->n, 256)), dim3(256), 0, c->stream, G, D, map, out->status);
    hipLaunchKernelGGL(k_cf_count, dim3(ntiles), dim3(kScanThreads), 0, c->stream, G, D, map, peak, bsum);
    hipLaunchKernelGGL(k_cf_tiles, dim3(1), dim3(1024), 0, c->stream, bsum, ntiles, total);
    hipLaunchKernelGGL(k_cf_write, dim3(ntiles), dim3(kScanThreads), 0, c->stream, G, D, map, peak, bsum, total,
                       O);
    hipLaunchKernelGGL(k_cf_clear, dim3(blocks_for(d->n, 256)), dim3(256), 0, c->stream, G, D, map);
  } else {
    fill_i32(c, out->n_clusters, 1, 0);
  }
  prof_end(c, pm);
  HIPCHK(c, hipGetLastError());
  c->cf_clean_ws = ws;
  c->cf_clean_cells = G.per_sector * kSectors;
  return TPC_OK;
}

int tpc_copy_probe(tpc_ctx* c, const void* src, void* dst, size_t bytes) {
  if (!c || !src || !dst || bytes % 16) return TPC_E_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  const int64_t n = (int64_t)(bytes / 16);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, (int64_t)ncu * 16);
  if (n) hipLaunchKernelGGL(k_copy_probe, dim3(std::max(blocks, 1)), dim3(256), 0, c->stream,
                            (const float4*)src, (float4*)dst, n);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int tpc_debug_propagate(tpc_ctx* c, const float* in, float* out, int32_t n) {
  if (!c || !in || !out || n < 0) return TPC_E_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  if (n) hipLaunchKernelGGL(k_debug_propagate, dim3(blocks_for(n, 64)), dim3(64), 0, c->stream, in, out, n, c->k);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

int tpc_debug_update(tpc_ctx* c, const float* in, float* out, int32_t n) {
  if (!c || !in || !out || n < 0) return TPC_E_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  if (n) hipLaunchKernelGGL(k_debug_update, dim3(blocks_for(n, 64)), dim3(64), 0, c->stream, in, out, n, c->k);
  HIPCHK(c, hipGetLastError());
  return TPC_OK;
}

}  // extern "C"

// Kernels of the TPC tracking path (gfx950).  All index spaces are int32.
//
// Data layout in HBM (all structure-of-arrays, one workspace):
//   input order   : the caller's cluster arrays; ckey/ccell per input cluster.
//   slots         : one per (job, sector, row) = (j*36 + s)*152 + r; slot_off is the
//                   start of each slot in grid order, sgrid its cell geometry.
//   grid order    : clusters sorted by (slot, cell); gy, gz, gidx (input index),
//                   gslot; every later stage works in this space.
//   tracklets     : ids ranked by the input index of their start cluster; hits are
//                   stored hit-major (k*capT + t) so that lanes of a wave write
//                   neighbouring words; state is [21][capT].
//   tracks        : CSR (sel_off, sel_hits) in tracklet-id order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpc_math.h"

namespace tpc {

// A range bound known either on the host (ptr == nullptr) or in device memory.
// The value is clamped to `max` (capacities of the arrays it indexes).
struct Bound {
  const int32_t* ptr;
  int32_t off;
  int32_t max;
  __device__ __forceinline__ int32_t get() const {
    const int32_t v = (ptr ? *ptr : 0) + off;
    return v < max ? v : max;
  }
};

// One cluster in grid order: position, slot and input index in one 16-byte record,
// read with a single 16-byte load.
struct __attribute__((aligned(16))) GHit {
  float y, z;
  int32_t slot, idx;
};
__device__ __forceinline__ GHit ldh(const GHit* p) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  GHit h;
  h.y = v.x;
  h.z = v.y;
  h.slot = __float_as_int(v.z);
  h.idx = __float_as_int(v.w);
  return h;
}
__device__ __forceinline__ void sth(GHit* p, float y, float z, int32_t slot, int32_t idx) {
  *reinterpret_cast<float4*>(p) = make_float4(y, z, __int_as_float(slot), __int_as_float(idx));
}

// Tracklet records: hit list rows of kHitStride ints (64-byte aligned, at least kRows),
// state rows of kStateStride floats (P[5], C[15], x; 32-byte aligned).
constexpr int kHitStride = 160;
// Largest job-local tracklet id that the 32-bit hit-weight key can hold.
constexpr int32_t kLocalIdMax = (1 << 24) - 1;
constexpr int kStateStride = 24;
// Fitted track records: P[5], C[15], x, the compensation terms L[5], padding (kFitStride
// floats, one 128-byte line).
constexpr int kFitStride = 32;

struct SlotGrid {
  float ylo, zlo, inv_by, inv_bz;
  int32_t ny, nz, ncell, cbase;  // cbase: global index of the slot's first cell
};

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// status bits
// rANS: slots of the model, symbols per lane, lanes per chunk (one wave)
constexpr uint32_t kRansM = 1u << 16;
constexpr int kRansLaneSymbols = 512;
constexpr int kRansLanesPerChunk = 64;
__host__ __device__ inline int64_t rans_lanes(int64_t n) {
  const int64_t chunk = (int64_t)kRansLanesPerChunk * kRansLaneSymbols;
  return (n + chunk - 1) / chunk * kRansLanesPerChunk;
}

constexpr int32_t kStatusRange = 1;
constexpr int32_t kStatusCapacity = 2;

// counters
enum Counter { kCntStatus = 0, kCntTracklets = 1, kCntSelected = 2, kCntSelHits = 3,
               kCntOut = 4, kCntOutHits = 5, kCntMergeCand = 6, kCntQueue = 8,  // 8 per-XCD tickets
               kNumCounters = 16 };

}  // namespace tpc

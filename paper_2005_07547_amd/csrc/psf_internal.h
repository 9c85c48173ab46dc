// Host-visible declarations shared between the C-ABI layer and the kernel
// translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psf_device.h"

namespace psf {

struct RecPtrs {
  const float *px, *py, *pz, *nx, *ny, *nz, *ox, *oy, *oz, *r, *g, *b, *rough;
};

struct QryPtrs {
  const float *px, *py, *pz, *nx, *ny, *nz, *ox, *oy, *oz, *rough;
};

// Partitioned-insert working buffers of one table.
struct PartView {
  unsigned long long* stage_key;  // staged sample keys, grouped per tile by partition
  float* stage_rgb;               // staged sample values (r, g, b triples), same order
  uint32_t* runs;                 // [tile][partition + 1]: exclusive offsets in the tile
  unsigned long long* rkeys;      // key of every record of the last binning, record order
  uint32_t tile;                  // records per binning tile
  uint32_t max_tiles;             // tiles per launch
  uint64_t capacity;              // records per launch
};

hipError_t launch_keys(const RecPtrs& rec, uint64_t n, const KeyParams& kp, unsigned long long* out,
                       hipStream_t s);
hipError_t launch_insert_direct(const RecPtrs& rec, uint64_t n, const KeyParams& kp,
                                const TableView& tv, hipStream_t s);
hipError_t launch_update(const TableView& tv, const BlendParams& bp, uint64_t nslots, hipStream_t s);
hipError_t launch_query(const QryPtrs& q, uint64_t n, const KeyParams& kp, const TableView& tv,
                        int32_t dtype, float* out, uint8_t* found, hipStream_t s);
hipError_t launch_clear(const TableView& tv, uint64_t nslots, hipStream_t s);
hipError_t launch_reset_counters(const TableView& tv, uint64_t nslots, hipStream_t s);
hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s);
hipError_t launch_count_occupied(const TableView& tv, uint64_t nslots, unsigned long long* out,
                                 hipStream_t s);
// Partitioned insertion of n <= pv.capacity records: bin, then merge.
// fuse != nullptr applies the temporal blend in the merge pass (the table
// must hold no pending samples).
hipError_t launch_bin(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                      const PartView& pv, hipStream_t s);
hipError_t launch_merge(uint64_t n, const TableView& tv, const PartView& pv, const BlendParams* fuse,
                        hipStream_t s);
// Lookup of the records binned last, by their cached keys.
hipError_t launch_query_cached(const unsigned long long* rkeys, uint64_t n, const TableView& tv,
                               int32_t dtype, float* out, uint8_t* found, hipStream_t s);
bool bin_per_ok(uint32_t per);          // supported records per thread of the binning pass
uint32_t bin_tile(uint32_t per);        // records per binning tile
uint32_t update_grid(uint64_t nslots);  // blocks of the streaming update

// One session of a batched iteration (device copy read by the batch kernels).
struct BatchSession {
  TableView tv;
  PartView pv;
  KeyParams kp;
  BlendParams bp;
  RecPtrs rec;
  QryPtrs q;
  uint64_t n, nq;
  float* out;
  uint8_t* found;
  uint32_t tile_begin, ntiles;  // binning blocks
  uint32_t part_begin, nparts;  // merge blocks (part_begin is a multiple of 8)
  uint32_t qblk_begin, nqblk;   // query blocks
  int32_t cached;               // queries are the binned records: use their keys
  int32_t pad;
};

// Launch the three batch kernels for k sessions (all partition-capable, no
// pending samples, the same binning width); d_sessions is device memory.
hipError_t launch_batch(const BatchSession* d_sessions, const BatchSession* h_sessions, uint32_t k,
                        hipStream_t s);
constexpr uint32_t kQueryBlock = 256;
hipError_t launch_compact(const TableView& tv, uint64_t nslots, int32_t dtype,
                          unsigned long long* cursor, uint64_t cap, unsigned long long* keys,
                          uint32_t* n_new, uint32_t* c_old, float* rgb, hipStream_t s);

}  // namespace psf

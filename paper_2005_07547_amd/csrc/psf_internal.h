// Host-visible declarations shared between the C-ABI layer and the kernel
// translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psf.h"
#include "psf_device.h"

namespace psf {

struct RecPtrs {
  const float *px, *py, *pz, *nx, *ny, *nz, *ox, *oy, *oz, *r, *g, *b, *rough, *footprint, *weight;
};

struct QryPtrs {
  const float *px, *py, *pz, *nx, *ny, *nz, *ox, *oy, *oz, *rough, *footprint;
};

// Partitioned-insert working buffers of one table.
struct PartView {
  unsigned long long* stage_key;  // staged entry keys, grouped per tile by partition
  float4* stage_v;                // staged entry values, same order: {r, g, b} sums
                                  // (w (r, g, b) with weights) and n, the records the
                                  // entry carries (with weights: the record's weight),
                                  // as a float; n = 0 marks an entry staged for lookup
                                  // only (a rejected sample).  The fused query writes
                                  // each entry's answer {r, g, b, 0} over it.
  float* stage_q;                 // per staged entry, the sum of its records' squared
                                  // luminances (tables that keep the variance; else null)
  uint32_t weights;               // this launch's records carry weights (n is then a
                                  // weight, one record per entry)
  uint32_t* runs;                 // [tile][partition + 1]: exclusive offsets in the tile
  uint32_t* runs_t;               // the same, transposed: [partition + 1][max_tiles]
                                  // (null: not transposed for this launch)
  // Staged position (in its tile) of every record of the binning, record
  // order; kNoPos for a skipped record.  Written only when non-null (the
  // fused query of an iteration whose queries are its records).
  uint16_t* perm;
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
// Two-field estimator (control variate or biased): the vertex keyed twice,
// on the outgoing direction (qo, table o) and on the incoming one (qi,
// table i); both share the position, normal and roughness arrays.
struct EstPtrs {
  QryPtrs qo, qi;
  const float *gr, *gg, *gb, *wp;
};
hipError_t launch_estimate(const EstPtrs& a, uint64_t n, const KeyParams& kp_o, const TableView& tv_o,
                           int32_t dt_o, const KeyParams& kp_i, const TableView& tv_i, int32_t dt_i,
                           int32_t mode, float param, float* out, uint8_t* applied, hipStream_t s);
// Progressive-solver samples: out = le + L~(next) * t per channel (le may be
// null pointers).
struct StepPtrs {
  QryPtrs next;
  const float *le_r, *le_g, *le_b, *t_r, *t_g, *t_b;
};
hipError_t launch_step_samples(const StepPtrs& a, uint64_t n, const KeyParams& kp, const TableView& tv,
                               int32_t dtype, float* out, hipStream_t s);
// Lookup falling back to up to `up` coarser levels; level_out[i] = 0 (no
// blended cell) or 1 + the number of levels above the query's own.
hipError_t launch_query_hier(const QryPtrs& q, uint64_t n, uint32_t up, const KeyParams& kp,
                             const TableView& tv, int32_t dtype, float* out, uint8_t* level_out,
                             hipStream_t s);
hipError_t launch_clear(const TableView& tv, uint64_t nslots, hipStream_t s);
hipError_t launch_reset_counters(const TableView& tv, uint64_t nslots, hipStream_t s);
// c_old = 0 for every cell whose box meets [lo, hi] (cells at e_min + level).
hipError_t launch_reset_region(const TableView& tv, uint64_t nslots, int32_t e_min, const float lo[3],
                               const float hi[3], hipStream_t s);
hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s);
hipError_t launch_count_occupied(const TableView& tv, uint64_t nslots, unsigned long long* out,
                                 hipStream_t s);
// Partitioned insertion of n <= pv.capacity records: bin, then merge.
// fuse != nullptr applies the temporal blend in the merge pass (the table
// must hold no pending samples); with results set as well, the merge pass
// also writes each staged entry's updated cell value over the entry (the
// bin pass must have written pv.perm), and launch_unstage then gathers them
// back into record order: the query of the records just inserted.
hipError_t launch_bin(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                      const PartView& pv, hipStream_t s);
hipError_t launch_merge(uint64_t n, const TableView& tv, const PartView& pv, const BlendParams* fuse,
                        bool results, hipStream_t s);
// runs -> runs_t for the first ntiles tiles (between bin and merge); a
// no-op when runs_t is null (the merge pass then reads runs in place).  The
// transpose pays once the table is large: from kTransposeMinWords entries.
constexpr uint64_t kTransposeMinWords = 1ull << 22;
bool transpose_pays(uint32_t ntiles, uint32_t nparts);
hipError_t launch_transpose_runs(const TableView& tv, const PartView& pv, uint32_t ntiles, hipStream_t s);
uint32_t transpose_blocks(uint32_t ntiles, uint32_t nparts);  // blocks of one transpose
hipError_t launch_unstage(uint64_t n, const TableView& tv, const PartView& pv, float* out,
                          uint8_t* found, hipStream_t s);
constexpr uint16_t kNoPos = 0xffffu;  // perm of a record without a valid key
// Result of a staged entry whose key has no blended cell: a NaN pattern in
// the red channel (real values are finite).
constexpr uint32_t kDroppedBits = 0xffffffffu;
// Staged key of a record with a valid key but a rejected (non-finite)
// sample: looked up, not inserted.  Valid keys never set bit 63.
constexpr unsigned long long kLookupOnlyBit = 1ull << 63;
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
  uint32_t trans_begin, ntrans;  // run-table transpose blocks
  uint32_t qblk_begin, nqblk;   // query blocks (one per tile when fused)
  int32_t fused_query;          // queries are the binned records: merge + unstage answer them
  int32_t pad;
};

// Launch the batch kernels for k sessions (all partition-capable, no
// pending samples, the same binning width); d_sessions is device memory.
// begins (device d_begins, host mirror h_begins) holds, per pass, each
// session's first block: [0, k) binning tiles, [stride, stride + k) merge
// partitions, [2 stride, ...) query blocks, [3 stride, ...) transpose blocks.
hipError_t launch_batch(const BatchSession* d_sessions, const uint32_t* d_begins, const uint32_t* h_begins,
                        uint32_t stride, const BatchSession* h_sessions, uint32_t k, hipStream_t s);
// Threads of a batch query block: the lookup of kQueryBlock queries, or the
// unstage of one fused session's tile (as wide as the single-table unstage).
constexpr uint32_t kQueryBlock = 512;
// Path sampler (the public structures, device copies in the kernels).
using PathPrim = psf_prim;
using PathCamera = psf_camera;
using PathParams = psf_path_params;
using PathOut = psf_path_out;
constexpr int32_t kPrimSphere = PSF_PRIM_SPHERE;
constexpr int32_t kOriginPoint = PSF_ORIGIN_POINT;
constexpr int32_t kPathsLo = PSF_PATHS_LO, kPathsLoe = PSF_PATHS_LOE;
hipError_t launch_sample_paths(const PathPrim* prims, uint32_t np, const PathCamera& cam, const PathParams& prm,
                               uint64_t n_paths, const PathOut& out, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint64_t n, uint32_t* out, hipStream_t s);

// SH payload tables (Sec. 2.6): direct insert into binary64 frame sums,
// streaming fit + blend, lookup evaluating the luminance at the normal.
hipError_t launch_insert_sh(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                            hipStream_t s);
hipError_t launch_update_sh(const TableView& tv, const BlendParams& bp, uint64_t nslots, hipStream_t s);
hipError_t launch_query_sh(const QryPtrs& q, uint64_t n, const KeyParams& kp, const TableView& tv, float* out,
                           uint8_t* found, hipStream_t s);
hipError_t launch_compact_var(const TableView& tv, uint64_t nslots, unsigned long long* cursor, uint64_t cap,
                              unsigned long long* keys, float* var, hipStream_t s);
hipError_t launch_compact_sh(const TableView& tv, uint64_t nslots, unsigned long long* cursor, uint64_t cap,
                             unsigned long long* keys, uint32_t* c_old, float* coeff, hipStream_t s);
hipError_t launch_clear_sh(const TableView& tv, uint64_t nslots, hipStream_t s);

hipError_t launch_compact(const TableView& tv, uint64_t nslots, int32_t dtype,
                          unsigned long long* cursor, uint64_t cap, unsigned long long* keys,
                          uint32_t* n_new, uint32_t* c_old, float* rgb, hipStream_t s);

}  // namespace psf

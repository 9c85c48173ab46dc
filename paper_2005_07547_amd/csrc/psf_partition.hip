// Partitioned insertion for gfx950.
//
// Global atomics on MI355X sustain only ~2e10 operations/s, far below what
// HBM streaming allows, so the fast insert path avoids them.  The table is
// split into partitions of 2^part_log2 consecutive slots (the partition of a
// key is the top bits of its hash, its probe sequence stays inside the
// partition).  Insertion then runs in two passes:
//
//   bin   -- one block per tile of records computes the keys, merges
//            records of one cell in neighbouring lanes into one entry,
//            counts entries per partition in LDS, sorts the tile by
//            partition in LDS and writes it out coalesced (keys, then
//            16-byte values {r, g, b, n}) to a staging area, plus the tile's
//            exclusive per-partition offsets (and, for the fused query, each
//            record's entry position in the tile);
//   (transpose -- for large launches, the offset table turned so that a
//            partition's offsets are one row);
//   merge -- one block per partition (512 threads, or 1024 where the
//            partition's LDS leaves room for one block per CU) loads the
//            partition's keys into LDS, gathers that partition's entries
//            from every tile, finds or claims each key's slot and
//            accumulates count (u32) and sums (binary64; also the weights
//            of a weighted table and the squared luminances of one that
//            keeps the variance) with LDS atomics, lists the touched
//            slots, then writes them back:
//            either adding into the global accumulators (plain insert) or,
//            when the whole frame is in this launch, applying the temporal
//            blend (Eq. 10-11) directly so the accumulators never touch HBM;
//            when the frame's queries are its records, it then writes each
//            staged entry's new cell value over the entry;
//   unstage -- one block per tile returns those values in record order.
//
// A partition is owned by exactly one block in the merge pass, so the
// write-back uses plain loads and stores.
#include <atomic>

#include "psf_device.h"
#include "psf_internal.h"

namespace psf {

constexpr int kBinThreads = 512;
constexpr int kMergeThreads = 512;
constexpr uint32_t kMaxPartLog2 = 12;

bool bin_per_ok(uint32_t per) { return per == 8 || per == 12 || per == 16; }

// LDS staging bytes per record of a binning tile: 16 (every tile's values
// in one float4 pass) where two blocks per CU still fit, else 12 (a tile
// with more than 3/4 of its records as entries stages its values in two
// halves).
__host__ __device__ constexpr size_t bin_lds_per_record(uint32_t per) { return per <= 8 ? 16 : 12; }
uint32_t bin_tile(uint32_t per) { return kBinThreads * per; }

// Exclusive prefix sum of cnt[0..m) in LDS, in place; returns the total.
// Called by all kThreads threads of the block.
template <int kThreads>
__device__ uint32_t block_exclusive_scan(uint32_t* cnt, uint32_t m, uint32_t* s_wave) {
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  const uint32_t chunk = (m + kThreads - 1) / kThreads;
  const uint32_t lo = tid * chunk;
  uint32_t local = 0;
  for (uint32_t c = 0; c < chunk; ++c)
    if (lo + c < m) local += cnt[lo + c];
  // inclusive scan across the wave
  uint32_t inc = local;
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(inc, off);
    if (lane >= off) inc += v;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      const uint32_t v = s_wave[w];
      s_wave[w] = run;
      run += v;
    }
    s_wave[kThreads / 64] = run;
  }
  __syncthreads();
  uint32_t run = s_wave[wave] + inc - local;
  for (uint32_t c = 0; c < chunk; ++c) {
    if (lo + c < m) {
      const uint32_t v = cnt[lo + c];
      cnt[lo + c] = run;
      run += v;
    }
  }
  const uint32_t total = s_wave[kThreads / 64];
  __syncthreads();
  return total;
}

// ------------------------------------------------------------------ bin
// Dynamic LDS holds first the partition histogram (P + 1 words), then, once
// every entry knows its place, the tile's staging buffers: keys, then the
// entries' values {r, g, b, n} (as float4 when they fit, else in two
// halves), so that every global write of the partition-sorted tile is
// coalesced.
//
// Pre-merge: unless the records carry weights, the records of one wave that
// fall in the same cell as the lane before them (neighbouring pixels of a
// scanline usually share a cell at the first bounce) leave a single staged
// entry: the first lane of each such run carries the run's record count and
// value sums (a segmented sum over lanes, in a fixed order), and the other
// records of the run only point at it for the fused query.
//
// kX: what the records carry beyond the common fields, kXFootprint (their
// level rule) and kXWeight (MIS weights: every sample is its own entry with
// value w (r, g, b) and n = w; a weight is read only after the sort, which
// also counts the samples it rejects); separate instantiations keep the
// extra loads and their registers out of the common case.
constexpr uint32_t kXFootprint = 1, kXWeight = 2;

__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long v, uint32_t d) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, d);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), d);
  return ((unsigned long long)hi << 32) | lo;
}

// Records carried by the entry of a run head in lane `lane` (1 + the
// continuation lanes that follow it); cont has bit l set where lane l
// continues lane l - 1's run.
__device__ __forceinline__ uint32_t run_records(unsigned long long cont, uint32_t lane) {
  const unsigned long long after = lane == 63 ? 0ull : cont >> (lane + 1);
  return 1u + (uint32_t)__builtin_ctzll(~after);
}

// Lane of the head of `lane`'s run (the last lane at or before it that does
// not continue its predecessor).
__device__ __forceinline__ uint32_t run_head(unsigned long long cont, uint32_t lane) {
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  return 63u - (uint32_t)__builtin_clzll(~cont & upto);
}

template <uint32_t kPer, uint32_t kX>
__device__ __forceinline__ void bin_body(const RecPtrs& rec, uint64_t n, const KeyParams& kp,
                                         const TableView& tv, const PartView& pv, uint32_t tile) {
  constexpr bool kFp = (kX & kXFootprint) != 0, kW = (kX & kXWeight) != 0;
  extern __shared__ uint32_t s_dyn_bin[];
  __shared__ uint32_t s_wave[kBinThreads / 64 + 1];
  __shared__ unsigned long long s_cont[kBinThreads / 64][kPer];  // per wave and record row: run continuations
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  uint32_t* s_hist = s_dyn_bin;
  unsigned long long* s_k = reinterpret_cast<unsigned long long*>(s_dyn_bin);
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  const uint64_t t0 = (uint64_t)tile * (kBinThreads * kPer);
  // records merge into runs only with integer counters and no weights; a
  // table that keeps the variance also sums each run's squared luminances
  // (in registers: with 8 records per thread; with more, its records stay
  // entries of their own)
  const bool var = tv.var != nullptr;
  constexpr bool kQRuns = kPer <= 8;
  const bool premerge = !kW && (kQRuns || !var);
  for (uint32_t p = tid; p <= P; p += kBinThreads) s_hist[p] = 0;
  __syncthreads();

  uint64_t key[kPer];
  // partition << 16 | rank, then the entry's position in the sorted tile
  // (for a merged record: its run head's); ~0 if the record has no entry
  uint32_t pos[kPer];
  float rgb[kPer][3];
  float qs[kQRuns ? kPer : 1];  // squared luminance (variance tables), summed over runs like rgb
  uint32_t n_skip = 0, n_ovf = 0;
  // flags riding in the top bits of a position (partition << 13 | rank, the
  // partition < 2^15 and the rank < 2^13, before the scan; the position in
  // the tile < 2^13 after it): merged into the previous lane's entry;
  // with weights, staged for lookup only and counted as a coordinate overflow
  constexpr uint32_t kPosTail = 1u << 29, kPosLookupOnly = 1u << 31, kPosOverflow = 1u << 30;
  constexpr uint32_t kPosBits = kPosTail - 1;
  const bool hr = rec.rough != nullptr;
  // Every load is unconditional (indices past the end are clamped, absent
  // arrays alias the positions) so that a batch of records is a single
  // memory round trip; validity is applied afterwards.  The records are read
  // once: non-temporal loads keep them from evicting what the merge pass
  // reads next from the caches (the staged entries, the key mirror, the
  // slots).
  const float* p_ox = hr ? rec.ox : rec.px;
  const float* p_oy = hr ? rec.oy : rec.px;
  const float* p_oz = hr ? rec.oz : rec.px;
  const float* p_ro = hr ? rec.rough : rec.px;
  constexpr uint32_t kLoad = kPer == 12 ? 3 : 4;  // records per load round trip (12: no spills)
#pragma unroll
  for (uint32_t j0 = 0; j0 < kPer; j0 += kLoad) {
    float f[kLoad][13];
    float fp[kLoad];
#pragma unroll
    for (uint32_t q = 0; q < kLoad; ++q) {
      const uint64_t i = t0 + (uint64_t)(j0 + q) * kBinThreads + tid;
      const uint64_t ic = i < n ? i : n - 1;
      f[q][0] = __builtin_nontemporal_load(rec.px + ic);
      f[q][1] = __builtin_nontemporal_load(rec.py + ic);
      f[q][2] = __builtin_nontemporal_load(rec.pz + ic);
      f[q][3] = __builtin_nontemporal_load(rec.nx + ic);
      f[q][4] = __builtin_nontemporal_load(rec.ny + ic);
      f[q][5] = __builtin_nontemporal_load(rec.nz + ic);
      f[q][6] = __builtin_nontemporal_load(p_ox + ic);
      f[q][7] = __builtin_nontemporal_load(p_oy + ic);
      f[q][8] = __builtin_nontemporal_load(p_oz + ic);
      f[q][9] = __builtin_nontemporal_load(rec.r + ic);
      f[q][10] = __builtin_nontemporal_load(rec.g + ic);
      f[q][11] = __builtin_nontemporal_load(rec.b + ic);
      f[q][12] = __builtin_nontemporal_load(p_ro + ic);
      fp[q] = kFp ? __builtin_nontemporal_load(rec.footprint + ic) : 0.0f;
    }
    // Every loaded value is used here, so the batch's loads all issue
    // before the first wait: left alone, the compiler sinks some of them
    // behind the key function's finiteness tests, each such group a
    // dependent round trip of its own.
#pragma unroll
    for (uint32_t q = 0; q < kLoad; ++q) {
#pragma unroll
      for (uint32_t k = 0; k < 13; ++k) asm volatile("" : : "v"(f[q][k]));
      if (kFp) asm volatile("" : : "v"(fp[q]));
    }
#pragma unroll
    for (uint32_t q = 0; q < kLoad; ++q) {
      const uint32_t j = j0 + q;
      const uint64_t i = t0 + (uint64_t)j * kBinThreads + tid;
      bool ovf = false;
      uint64_t k = 0;
      const bool kv = i < n && cell_key(kp, f[q][0], f[q][1], f[q][2], f[q][3], f[q][4], f[q][5], f[q][6],
                                        f[q][7], f[q][8], hr, f[q][12], kFp, fp[q], k, ovf);
      const bool sv = finite3(f[q][9], f[q][10], f[q][11]);
      key[j] = (kv && sv) ? k : k | kLookupOnlyBit;
      rgb[j][0] = f[q][9];
      rgb[j][1] = f[q][10];
      rgb[j][2] = f[q][11];
      if (i < n && !(kv && sv)) ++n_skip;
      n_ovf += (kv && sv && ovf) ? 1u : 0u;
      // a record whose sample is rejected but whose key is valid is still a
      // query vertex: with the fused query it is staged for lookup only
      const bool entry = kv && (sv || pv.perm);
      pos[j] = entry ? ((kv && sv) ? 0u : kPosLookupOnly) | ((ovf && sv) ? kPosOverflow : 0u) : ~0u;
    }
  }
  // entries per partition (ranks), after merging runs of one cell in
  // neighbouring lanes: only a run's head gets an entry
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const bool smp = pos[j] != ~0u && !(pos[j] & kPosLookupOnly);
    bool tail = false;
    if (kQRuns) {
      qs[kQRuns ? j : 0] = 0.0f;
      if (var) {
        const float y = luma32(rgb[j][0], rgb[j][1], rgb[j][2]);
        qs[kQRuns ? j : 0] = y * y;
      }
    }
    if (premerge) {
      // a sample whose key equals the previous lane's (also a sample)
      // continues that lane's run
      const unsigned long long kprev = shfl_up_u64(key[j], 1);
      const bool sprev = __shfl_up((int)smp, 1) != 0;
      tail = lane > 0 && smp && sprev && key[j] == kprev;
      const unsigned long long cont = __ballot(tail);
      if (lane == 0) s_cont[wave][j] = cont;
      if (cont) {
        // segmented suffix sums: after the step of offset d a lane holds
        // the sum over itself and the next 2d - 1 lanes of its run, so each
        // head ends with its run's total (fixed order: reproducible)
        unsigned long long live = cont;  // lanes ending runs of >= 2d
        for (uint32_t d = 1; live; d <<= 1) {
          const float vr = __shfl_down(rgb[j][0], d);
          const float vg = __shfl_down(rgb[j][1], d);
          const float vb = __shfl_down(rgb[j][2], d);
          const float vq = (kQRuns && var) ? __shfl_down(qs[kQRuns ? j : 0], d) : 0.0f;
          const bool same = lane + d < 64 &&
                            ((cont >> (lane + 1)) & ((1ull << d) - 1ull)) == ((1ull << d) - 1ull);
          if (same) {
            rgb[j][0] += vr;
            rgb[j][1] += vg;
            rgb[j][2] += vb;
            if (kQRuns) qs[kQRuns ? j : 0] += vq;
          }
          live &= live >> d;
        }
      }
    }
    if (pos[j] == ~0u) continue;
    if (tail) {
      pos[j] = kPosTail;
      continue;
    }
    const uint32_t p = partition_of(fmix64(key[j] & ~kLookupOnlyBit), tv.log2_slots, tv.part_log2);
    const uint32_t rank = atomicAdd(&s_hist[p], 1u);
    pos[j] |= (p << 13) | rank;
  }
  // rare-event counters: one atomic per wave when non-zero (with weights,
  // after the staging pass has judged them)
  auto count_events = [&]() {
    for (int off = 32; off > 0; off >>= 1) {
      n_skip += __shfl_xor(n_skip, off);
      n_ovf += __shfl_xor(n_ovf, off);
    }
    if (__lane_id() == 0) {
      if (n_skip) atomicAdd(stat_lane(tv.stats->skipped, tile), (unsigned long long)n_skip);
      if (n_ovf) atomicAdd(stat_lane(tv.stats->coord_overflow, tile), (unsigned long long)n_ovf);
    }
  };
  if (!kW) count_events();
  __syncthreads();
  const uint32_t count = block_exclusive_scan<kBinThreads>(s_hist, P + 1, s_wave);

  uint32_t* offs = pv.runs + (uint64_t)tile * (P + 1);
  for (uint32_t p = tid; p <= P; p += kBinThreads) offs[p] = s_hist[p];
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    if (pos[j] != ~0u && !(pos[j] & kPosTail)) {
      const uint32_t q = pos[j] & ((1u << 29) - 1u);
      pos[j] = (s_hist[q >> 13] + (q & 0x1fffu)) | (pos[j] & ~((1u << 29) - 1u));
    }
    if (premerge && pv.perm) {
      // a merged record is answered from its run head's entry
      const unsigned long long cont = s_cont[wave][j];
      if (cont) {
        const uint32_t hp = (uint32_t)__shfl((int)pos[j], (int)run_head(cont, lane));
        if (pos[j] == kPosTail) pos[j] = (hp & kPosBits) | kPosTail;
      }
    }
  }
  if (pv.perm) {
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint64_t i = t0 + (uint64_t)j * kBinThreads + tid;
      if (i < n) pv.perm[i] = pos[j] != ~0u ? (uint16_t)(pos[j] & kPosBits) : kNoPos;
    }
  }
  __syncthreads();  // the histogram is dead from here on; its LDS becomes staging

  auto own_entry = [&](uint32_t j) { return pos[j] != ~0u && !(pos[j] & kPosTail); };
  // n of each entry: the records it carries (with weights: the record's
  // weight); 0 marks an entry staged for lookup only
  auto entry_n = [&](uint32_t j) {
    uint32_t c = 1;
    if (premerge) {
      const unsigned long long cont = s_cont[wave][j];
      if (cont) c = run_records(cont, lane);
    }
    return (pos[j] & kPosLookupOnly) ? 0u : c;
  };
  if (var) {
    // each entry's squared-luminance sum, at its staged position (a record
    // of its own: its value's)
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      if (!own_entry(j)) continue;
      float q;
      if (kQRuns) {
        q = qs[kQRuns ? j : 0];
      } else {
        const float y = luma32(rgb[j][0], rgb[j][1], rgb[j][2]);
        q = y * y;
      }
      pv.stage_q[t0 + (pos[j] & kPosBits)] = q;
    }
  }
  float wn[kW ? kPer : 1];
  if (kW) {
    // The weights are first read here.  A sample whose weight is not finite
    // and > 0 is rejected: counted as skipped (not as a coordinate
    // overflow) and staged with n = 0, so the merge pass only looks it up
    // (with the fused query) or ignores it; an accepted one is staged as
    // w (r, g, b) with n = w.
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      wn[j] = 0.0f;
      if (!own_entry(j)) continue;
      const float w = rec.weight[t0 + (uint64_t)j * kBinThreads + tid];
      if (pos[j] & kPosLookupOnly) continue;
      if (__builtin_isfinite(w) && w > 0.0f) {
        rgb[j][0] *= w;
        rgb[j][1] *= w;
        rgb[j][2] *= w;
        wn[j] = w;
      } else {
        ++n_skip;
        n_ovf -= (pos[j] & kPosOverflow) ? 1u : 0u;
      }
    }
    count_events();
  }
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j)
    if (own_entry(j)) s_k[pos[j] & kPosBits] = key[j];
  __syncthreads();
  for (uint32_t i = tid; i < count; i += kBinThreads) pv.stage_key[t0 + i] = s_k[i];
  __syncthreads();
  // the entries' values {r, g, b, n}: as float4 when they fit in the LDS,
  // else in two halves, (r, g) then (b, n)
  auto entry_w = [&](uint32_t j) { return kW ? wn[kW ? j : 0] : (float)entry_n(j); };
  const size_t lds_bytes = (size_t)kBinThreads * kPer * bin_lds_per_record(kPer);  // the launch's dynamic LDS
  if ((size_t)count * 16 <= lds_bytes) {
    float4* s_v = reinterpret_cast<float4*>(s_dyn_bin);
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j)
      if (own_entry(j)) s_v[pos[j] & kPosBits] = make_float4(rgb[j][0], rgb[j][1], rgb[j][2], entry_w(j));
    __syncthreads();
    for (uint32_t i = tid; i < count; i += kBinThreads) pv.stage_v[t0 + i] = s_v[i];
  } else {
    float2* s_v = reinterpret_cast<float2*>(s_dyn_bin);
    float2* dst = reinterpret_cast<float2*>(pv.stage_v + t0);
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j)
      if (own_entry(j)) s_v[pos[j] & kPosBits] = make_float2(rgb[j][0], rgb[j][1]);
    __syncthreads();
    for (uint32_t i = tid; i < count; i += kBinThreads) dst[2 * i] = s_v[i];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j)
      if (own_entry(j)) s_v[pos[j] & kPosBits] = make_float2(rgb[j][2], entry_w(j));
    __syncthreads();
    for (uint32_t i = tid; i < count; i += kBinThreads) dst[2 * i + 1] = s_v[i];
  }
}

// Two 512-thread blocks per CU need at most 128 VGPRs (four waves per SIMD);
// the instantiations with footprints or weights would take a few more.
template <uint32_t kPer, uint32_t kX>
__global__ void __launch_bounds__(kBinThreads) __attribute__((amdgpu_waves_per_eu(kPer <= 12 ? 4 : 1)))
k_bin(RecPtrs rec, uint64_t n, KeyParams kp, TableView tv, PartView pv) {
  bin_body<kPer, kX>(rec, n, kp, tv, pv, blockIdx.x);
}

// ------------------------------------------------------------------ run table transpose
// The merge block of partition p needs the offsets of p and p + 1 in every
// tile: a column of the bin pass's [tile][P + 1] table.  A 64 x 64 LDS
// transpose turns the columns into rows, so the merge reads them coalesced.
constexpr uint32_t kTransposeDim = 64, kTransposeThreads = 256;

__device__ __forceinline__ void transpose_body(const PartView& pv, uint32_t P, uint32_t ntiles, uint32_t bx,
                                               uint32_t by) {
  __shared__ uint32_t s_t[kTransposeDim][kTransposeDim + 1];
  const uint32_t tid = threadIdx.x, c = tid % kTransposeDim, r0 = tid / kTransposeDim;
  constexpr uint32_t kRowsPerPass = kTransposeThreads / kTransposeDim;
  const uint32_t t0 = bx * kTransposeDim, p0 = by * kTransposeDim;
  const uint32_t stride = (pv.max_tiles + 3u) & ~3u;
  for (uint32_t r = r0; r < kTransposeDim; r += kRowsPerPass) {
    const uint32_t t = t0 + r, p = p0 + c;
    if (t < ntiles && p <= P) s_t[r][c] = pv.runs[(uint64_t)t * (P + 1) + p];
  }
  __syncthreads();
  for (uint32_t r = r0; r < kTransposeDim; r += kRowsPerPass) {
    const uint32_t p = p0 + r, t = t0 + c;
    if (t < ntiles && p <= P) pv.runs_t[(uint64_t)p * stride + t] = s_t[c][r];
  }
}

__global__ void __launch_bounds__(kTransposeThreads) k_transpose_runs(PartView pv, uint32_t P, uint32_t ntiles) {
  transpose_body(pv, P, ntiles, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------ merge
// Blocks are dispatched to the 8 XCDs round-robin; give each XCD a
// contiguous range of partitions so the offset rows they share stay in one
// L2.
__device__ __forceinline__ uint32_t xcd_partition(uint32_t b, uint32_t P) {
  if (P < 8 || (P & 7u)) return b;
  return (b & 7u) * (P >> 3) + (b >> 3);
}

constexpr uint32_t kRunsPerLane = 4;  // consecutive tile runs each lane keeps in registers
constexpr uint32_t kEntryBatch = 4;  // entries per lane loaded before processing
// Batches per wave whose (entry, slot) pairs stay in registers for the
// fused query; a wave with more batches finds the later entries' slots again.
constexpr uint32_t kKeepBatches = 2;
constexpr uint32_t kLookupLater = 0xfffffffeu;  // kept slot of a lookup-only entry

// Largest lane l with excl[l] <= e, where excl is a non-decreasing per-lane
// value (all lanes of the wave must call this).
__device__ __forceinline__ uint32_t wave_upper_bound(uint32_t excl, uint32_t e) {
  uint32_t a = 0;
#pragma unroll
  for (uint32_t step = 32; step > 0; step >>= 1) {
    const uint32_t v = (uint32_t)__shfl((int)excl, (int)(a + step));
    if (a + step < 64 && v <= e) a += step;
  }
  return a;
}

// One partition: blk is the block's index among the partition blocks of this
// table (the XCD-aware order maps it to a partition).  With results (fused
// mode only), every staged entry of the partition is overwritten with the
// value its cell holds after the blend (kDroppedBits in place of red when
// its key found no slot).
template <bool kFused, int kThreads = kMergeThreads>
__device__ __forceinline__ void merge_body(const TableView& tv, const PartView& pv, uint32_t ntiles,
                                           const BlendParams& bp, uint32_t blk, bool results) {
  // key[B] | cnt[B] | sum[3][B] (binary64: LDS f64 atomics are both faster
  // than f32 ones on gfx950 and exact enough to make the sum order
  // immaterial), then, in a table that keeps the luminance variance or has
  // weighted counters, sumx[B]: the squared luminances (staged per entry),
  // or the weights (binary64 like the value sums, rounded once to binary32
  // at the write-back, so the counters do not depend on the order of the
  // atomics; cnt then only marks the slots touched; every entry is one
  // record).  After the blend the sums hold the cells' new values.
  // Last, list[B] (16-bit): the touched slots, gathered for the write-back.
  extern __shared__ unsigned long long s_dyn[];
  __shared__ uint32_t s_dropped, s_nlist, s_sat;
  __shared__ uint32_t s_hist[16];
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  constexpr uint32_t kWaves = kThreads / 64;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t B = 1u << tv.part_log2;
  const uint32_t p = xcd_partition(blk, P);
  const uint64_t base = (uint64_t)p << tv.part_log2;
  const bool stats = (tv.flags & 1u) != 0;
  const bool wtd = weighted(tv);
  unsigned long long* s_key = s_dyn;
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_key + B);
  double* s_sum0 = reinterpret_cast<double*>(s_cnt + B);  // B >= 256: 8-byte aligned
  double* s_sum1 = s_sum0 + B;
  double* s_sum2 = s_sum1 + B;
  double* s_sumx = s_sum2 + B;  // only with tv.var or wtd
  const bool var = tv.var != nullptr;
  // the touched slots' indices (B entries), after the sums
  uint16_t* s_list = reinterpret_cast<uint16_t*>(s_sumx + ((var || wtd) ? B : 0u));
  const uint32_t tile = pv.tile;
  if (!kFused) results = false;

  // Each wave owns a contiguous slice of the tiles; it keeps up to
  // 64 * kRunsPerLane of this partition's runs (offsets) in registers.
  // (a multiple of 4 tiles, so that a lane's runs are one 16-byte load)
  const uint32_t per_wave = ((ntiles + kWaves - 1) / kWaves + 3u) & ~3u;
  const uint32_t w_lo = wave * per_wave;
  const uint32_t w_hi = (w_lo + per_wave < ntiles) ? w_lo + per_wave : ntiles;
  uint32_t r_lo[kRunsPerLane], r_hi[kRunsPerLane];
  uint32_t loaded = ~0u;  // chunk of runs held in registers
  const uint32_t stride = (pv.max_tiles + 3u) & ~3u;
  const uint32_t* row_lo = pv.runs_t + (uint64_t)p * stride;
  const uint32_t* row_hi = row_lo + stride;
  auto load_runs = [&](uint32_t c0) {
    const uint32_t t = c0 + lane * kRunsPerLane;  // a multiple of 4
    if (pv.runs_t) {
      // transposed table: two 16-byte loads (t + 3 < stride: inside the row)
      uint4 lo = make_uint4(0, 0, 0, 0), hi = make_uint4(0, 0, 0, 0);
      if (t < w_hi) {
        lo = *reinterpret_cast<const uint4*>(row_lo + t);
        hi = *reinterpret_cast<const uint4*>(row_hi + t);
      }
      const uint32_t l4[4] = {lo.x, lo.y, lo.z, lo.w}, h4[4] = {hi.x, hi.y, hi.z, hi.w};
#pragma unroll
      for (uint32_t j = 0; j < kRunsPerLane; ++j) {
        const bool in = t + j < w_hi;
        r_lo[j] = in ? l4[j] : 0u;
        r_hi[j] = in ? h4[j] : 0u;
      }
    } else {
      // the bin pass's table: one column, read in place (the lines are
      // shared by the neighbouring partitions an XCD runs at the same time)
#pragma unroll
      for (uint32_t j = 0; j < kRunsPerLane; ++j) {
        r_lo[j] = 0;
        r_hi[j] = 0;
        if (t + j < w_hi) {
          const uint32_t* offs = pv.runs + (uint64_t)(t + j) * (P + 1) + p;
          r_lo[j] = offs[0];
          r_hi[j] = offs[1];
        }
      }
    }
    loaded = c0;
  };
  // A chunk: the runs of up to 64 * kRunsPerLane consecutive tiles of the
  // wave's slice, lane l holding kRunsPerLane of them; pk[j] packs the start
  // of the lane's run j among the lane's entries (< 3 tiles) with the run's
  // offset in its tile (< 2^16); excl is the lane's first entry in the
  // chunk, total the chunk's entries.
  struct Chunk {
    uint32_t pk[kRunsPerLane];
    uint32_t excl, total;
    uint64_t cbase;
  };
  auto chunk_of = [&](uint32_t c0) {
    if (loaded != c0) load_runs(c0);
    Chunk ch;
    uint32_t lt = 0;
#pragma unroll
    for (uint32_t j = 0; j < kRunsPerLane; ++j) {
      ch.pk[j] = (lt << 16) | r_lo[j];
      lt += r_hi[j] - r_lo[j];
    }
    uint32_t inc = lt;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)inc, off);
      if (lane >= off) inc += v;
    }
    ch.excl = inc - lt;
    ch.total = (uint32_t)__shfl((int)inc, 63);
    ch.cbase = (uint64_t)c0 * tile;
    return ch;
  };
  // The batch at entry e0 of a chunk: at[q] is the staging index of the
  // lane's q-th entry, ev[q] whether it exists (absent entries point at a
  // tile's first entry, so that every load stays branch-free and in
  // bounds).  A batch takes the next 64 * kEntryBatch entries of the
  // chunk's concatenated runs.
  auto batch_of = [&](const Chunk& ch, uint32_t e0, uint64_t* at, bool* ev) {
#pragma unroll
    for (uint32_t q = 0; q < kEntryBatch; ++q) {
      const uint32_t e = e0 + q * 64 + lane;
      const uint32_t a = wave_upper_bound(ch.excl, e);
      const uint32_t r = e - (uint32_t)__shfl((int)ch.excl, (int)a);
      // the last of lane a's runs that starts at or before r holds it
      uint32_t js = 0, ps = (uint32_t)__shfl((int)ch.pk[0], (int)a);
#pragma unroll
      for (uint32_t j = 1; j < kRunsPerLane; ++j) {
        const uint32_t v = (uint32_t)__shfl((int)ch.pk[j], (int)a);
        if ((v >> 16) <= r) {
          js = j;
          ps = v;
        }
      }
      ev[q] = e < ch.total;
      at[q] = ch.cbase + (ev[q] ? (uint64_t)(a * kRunsPerLane + js) * tile + (ps & 0xffffu) + (r - (ps >> 16))
                                : 0ull);
    }
  };
  // Calls body(at, ev, nb) for every batch of the wave's entries, in order
  // (nb counts batches).
  auto for_each_batch = [&](auto&& body) {
    uint32_t nb = 0;
    for (uint32_t c0 = w_lo; c0 < w_hi; c0 += 64 * kRunsPerLane) {
      const Chunk ch = chunk_of(c0);
      for (uint32_t e0 = 0; e0 < ch.total; e0 += 64 * kEntryBatch, ++nb) {
        bool ev[kEntryBatch];
        uint64_t at[kEntryBatch];
        batch_of(ch, e0, at, ev);
        body(at, ev, nb);
      }
    }
    return nb;
  };

  // keys first, then the first runs, then the wave's first batch of entries:
  // all in flight together, before the key table is built
  constexpr uint32_t kKeysPerThread = (1u << kMaxPartLog2) / kThreads;
  unsigned long long kk[kKeysPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kKeysPerThread; ++j) {
    const uint32_t s = tid + j * kThreads;
    kk[j] = s < B ? tv.keys[base + s] : kEmpty;
  }
  Chunk ch0{};
  uint64_t at0[kEntryBatch];
  bool ev0[kEntryBatch];
  unsigned long long ek0[kEntryBatch];
  float4 v0[kEntryBatch];
  float q0[kEntryBatch];  // variance tables: the entries' squared-luminance sums
  if (w_lo < w_hi) {
    ch0 = chunk_of(w_lo);
    batch_of(ch0, 0, at0, ev0);
#pragma unroll
    for (uint32_t q = 0; q < kEntryBatch; ++q) {
      ek0[q] = pv.stage_key[at0[q]];
      v0[q] = pv.stage_v[at0[q]];
      q0[q] = var ? pv.stage_q[at0[q]] : 0.0f;
    }
  }
#pragma unroll
  for (uint32_t j = 0; j < kKeysPerThread; ++j) {
    const uint32_t s = tid + j * kThreads;
    if (s < B) {
      s_key[s] = kk[j];
      s_cnt[s] = 0;
      s_sum0[s] = s_sum1[s] = s_sum2[s] = 0.0;
      if (var || wtd) s_sumx[s] = 0.0;
    }
  }
  if (tid == 0) s_dropped = s_nlist = s_sat = 0;
  if (tid < 16) s_hist[tid] = 0;
  __syncthreads();

  // (staging index, slot) of the lane's entries of the first kKeepBatches
  // batches; ~0u marks an absent entry (index) or a dropped key (slot)
  uint32_t keep_at[kKeepBatches][kEntryBatch], keep_slot[kKeepBatches][kEntryBatch];
#pragma unroll
  for (uint32_t b = 0; b < kKeepBatches; ++b)
#pragma unroll
    for (uint32_t q = 0; q < kEntryBatch; ++q) keep_at[b][q] = keep_slot[b][q] = ~0u;

  auto accumulate = [&](const uint64_t* at, const bool* ev, const unsigned long long* ek, const float4* v,
                        const float* qv, uint32_t nb) {
#pragma unroll
    for (uint32_t q = 0; q < kEntryBatch; ++q) {
      uint32_t slot = ~0u;
      // n = 0: an entry staged for lookup only (a rejected sample); with the
      // fused query it is looked up after the blend, else it is ignored
      if (results && v[q].w == 0.0f) slot = kLookupLater;
      if (ev[q] && v[q].w != 0.0f) {
        // records behind the entry, for the drop and probe statistics
        const uint32_t recs = pv.weights ? 1u : (uint32_t)v[q].w;
        const unsigned long long key = ek[q];
        const uint32_t start = (uint32_t)fmix64(key) & (B - 1);
        uint32_t i = 0;
        for (; i < tv.max_probe; ++i) {
          const uint32_t s = (start + i) & (B - 1);
          unsigned long long cur = s_key[s];
          if (cur == kEmpty) cur = atomicCAS(&s_key[s], kEmpty, key);
          if (cur == kEmpty || cur == key) {
            slot = s;
            break;
          }
        }
        if (slot == ~0u) {
          atomicAdd(&s_dropped, recs);
        } else {
          if (stats) atomicAdd(&s_hist[i < 15 ? i : 15], recs);
          if (wtd) {
            atomicAdd(&s_sumx[slot], (double)v[q].w);
            s_cnt[slot] = 1u;
          } else {
            atomicAdd(&s_cnt[slot], (uint32_t)v[q].w);
          }
          atomicAdd(&s_sum0[slot], (double)v[q].x);
          atomicAdd(&s_sum1[slot], (double)v[q].y);
          atomicAdd(&s_sum2[slot], (double)v[q].z);
          if (var) atomicAdd(&s_sumx[slot], (double)qv[q]);
        }
      }
      if (results) {
        const uint32_t a = ev[q] ? (uint32_t)at[q] : ~0u;
#pragma unroll
        for (uint32_t b = 0; b < kKeepBatches; ++b) {
          if (nb == b) {
            keep_at[b][q] = a;
            keep_slot[b][q] = slot;
          }
        }
      }
    }
  };
  // the first batch was loaded above; every later one into the same registers
  uint32_t batches = 0;
  for (uint32_t c0 = w_lo; c0 < w_hi; c0 += 64 * kRunsPerLane) {
    const Chunk ch = c0 == w_lo ? ch0 : chunk_of(c0);
    for (uint32_t e0 = 0; e0 < ch.total; e0 += 64 * kEntryBatch, ++batches) {
      if (c0 != w_lo || e0 != 0) {
        batch_of(ch, e0, at0, ev0);
#pragma unroll
        for (uint32_t q = 0; q < kEntryBatch; ++q) {
          ek0[q] = pv.stage_key[at0[q]];
          v0[q] = pv.stage_v[at0[q]];
          q0[q] = var ? pv.stage_q[at0[q]] : 0.0f;
        }
      }
      accumulate(at0, ev0, ek0, v0, q0, batches);
    }
  }
  __syncthreads();

  // List the touched slots (about one in eight, scattered), so that the
  // write-back runs on full waves: each thread then blends at most kWb
  // cells, whose old slots are loaded together (one memory round trip).
  for (uint32_t s0 = 0; s0 < B; s0 += kThreads) {
    const uint32_t s = s0 + tid;
    const bool hit = s < B && s_cnt[s] != 0u;
    const unsigned long long m = __ballot(hit);
    uint32_t at = 0;
    if (lane == 0 && m) at = atomicAdd(&s_nlist, (uint32_t)__popcll(m));
    at = (uint32_t)__shfl((int)at, 0);
    if (hit)
      s_list[at + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
          (uint16_t)s;
  }
  __syncthreads();
  const uint32_t n_touched = s_nlist;
  bool sat = false;
  constexpr uint32_t kWb = 2;
  for (uint32_t i0 = 0; i0 < n_touched; i0 += kWb * kThreads) {
    uint32_t sl[kWb];
    Slot old[kWb];
    Acc acc_old[kWb];
    float var_old[kWb];  // fused: the variance
    double q_old[kWb];   // not fused: the pending squared-luminance sum
#pragma unroll
    for (uint32_t j = 0; j < kWb; ++j) {
      const uint32_t i = i0 + j * kThreads + tid;
      sl[j] = i < n_touched ? (uint32_t)s_list[i] : ~0u;
    }
    // absent entries read the partition's first slot, so that the group's
    // loads carry no branches and overlap
#pragma unroll
    for (uint32_t j = 0; j < kWb; ++j) {
      const uint64_t src = base + (sl[j] != ~0u ? sl[j] : 0u);
      old[j] = tv.slots[src];
      if (!kFused) acc_old[j] = tv.acc[src];
      if (var) {
        if (kFused)
          var_old[j] = tv.var[src];
        else
          q_old[j] = tv.acc_q[src];
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < kWb; ++j) {
      if (sl[j] == ~0u) continue;
      const uint32_t s = sl[j];
      const uint64_t g = base + s;
      // the frame's counter word (a weighted table's weight sum rounds once)
      const uint32_t c = wtd ? __float_as_uint((float)s_sumx[s]) : s_cnt[s];
      const unsigned long long k = s_key[s];
      if (kFused) {
        const float alpha = blend_alpha(bp, c, old[j].c_old, wtd);
        float L[3];
        load_blend_state(old[j], bp.dtype, L[0], L[1], L[2]);
        // the new sample mean, rounded once from binary64
        const double cd = wtd ? (double)__uint_as_float(c) : (double)c;
        const float means[3] = {(float)(s_sum0[s] / cd), (float)(s_sum1[s] / cd), (float)(s_sum2[s] / cd)};
        float out[3];
        for (int ch = 0; ch < 3; ++ch) {
          const float m = means[ch];
          out[ch] = alpha == 1.0f ? m : (1.0f - alpha) * L[ch] + alpha * m;
        }
        if (var) {
          double m, s2;
          frame_moments(s_sum0[s], s_sum1[s], s_sum2[s], s_sumx[s], cd, m, s2);
          tv.var[g] = blend_variance(var_old[j], alpha, luma32(L[0], L[1], L[2]), m, s2);
        }
        uint32_t enc[4], pad;
        encode_state(bp.dtype, out[0], out[1], out[2], enc, pad, sat);
        Slot nw;
        nw.key = k;
        nw.c_old = counter_add(old[j].c_old, c, wtd);
        nw.pad = pad;
        nw.L[0] = enc[0];
        nw.L[1] = enc[1];
        nw.L[2] = enc[2];
        nw.L[3] = enc[3];
        tv.slots[g] = nw;
        if (old[j].key != k) tv.keys[g] = k;
        if (results) {
          // what a lookup of the cell returns from now on
          float v[3];
          load_state(nw, bp.dtype, v[0], v[1], v[2]);
          s_sum0[s] = v[0];
          s_sum1[s] = v[1];
          s_sum2[s] = v[2];
        }
      } else {
        Acc a = acc_old[j];
        a.n = counter_add(a.n, c, wtd);
        a.s[0] += (float)s_sum0[s];
        a.s[1] += (float)s_sum1[s];
        a.s[2] += (float)s_sum2[s];
        tv.acc[g] = a;
        if (var) tv.acc_q[g] = q_old[j] + s_sumx[s];
        if (old[j].key != k) {
          tv.slots[g].key = k;
          tv.keys[g] = k;
        }
      }
    }
  }
  if (kFused && sat) atomicAdd(&s_sat, 1u);
  __syncthreads();

  if (results) {
    // slot of a key in the final LDS key table, or ~0u
    auto find = [&](unsigned long long key) {
      const uint32_t start = (uint32_t)fmix64(key) & (B - 1);
      for (uint32_t i = 0; i < tv.max_probe; ++i) {
        const uint32_t s = (start + i) & (B - 1);
        const unsigned long long cur = s_key[s];
        if (cur == key) return s;
        if (cur == kEmpty) break;
      }
      return ~0u;
    };
    // the value a lookup of the cell in slot returns (kDroppedBits if none),
    // written over the entry in one 16-byte store
    auto put = [&](uint64_t at, uint32_t slot) {
      float v[3] = {__uint_as_float(kDroppedBits), 0.0f, 0.0f};
      if (slot != ~0u && s_cnt[slot] > 0) {
        v[0] = (float)s_sum0[slot];
        v[1] = (float)s_sum1[slot];
        v[2] = (float)s_sum2[slot];
      } else if (slot != ~0u) {
        // a lookup-only entry whose cell this launch did not touch
        const Slot sl = tv.slots[base + slot];
        if (sl.c_old > 0) load_state(sl, bp.dtype, v[0], v[1], v[2]);
      }
      pv.stage_v[at] = make_float4(v[0], v[1], v[2], 0.0f);
    };
#pragma unroll
    for (uint32_t b = 0; b < kKeepBatches; ++b) {
#pragma unroll
      for (uint32_t q = 0; q < kEntryBatch; ++q) {
        if (keep_at[b][q] == ~0u) continue;
        uint32_t slot = keep_slot[b][q];
        if (slot == kLookupLater) slot = find(pv.stage_key[keep_at[b][q]] & ~kLookupOnlyBit);
        put(keep_at[b][q], slot);
      }
    }
    if (batches > kKeepBatches) {
      // later batches: read the keys again and find their (final) slots
      for_each_batch([&](const uint64_t* at, const bool* ev, uint32_t nb) {
        if (nb < kKeepBatches) return;
        unsigned long long ek[kEntryBatch];
#pragma unroll
        for (uint32_t q = 0; q < kEntryBatch; ++q) ek[q] = pv.stage_key[at[q]];
#pragma unroll
        for (uint32_t q = 0; q < kEntryBatch; ++q)
          if (ev[q]) put(at[q], find(ek[q] & ~kLookupOnlyBit));
      });
    }
  }

  if (tid == 0) {
    if (s_dropped) atomicAdd(&tv.stats->dropped, (unsigned long long)s_dropped);
    if (kFused) {
      if (s_sat) atomicAdd(&tv.stats->saturated, (unsigned long long)s_sat);
      BlockTouch* bt = &tv.touch[blk];
      bt->last = n_touched;
      bt->total += n_touched;
    }
  }
  if (stats && tid < 16 && s_hist[tid])
    atomicAdd(&tv.stats->probe_hist[tid], (unsigned long long)s_hist[tid]);
}

// 512 threads per partition block, 1024 where the partition's LDS allows
// one block per CU (4096 slots, or 2048 with a fifth sum per slot): 16
// waves per CU either way.
template <bool kFused, int kThreads>
__global__ void __launch_bounds__(kThreads) k_merge(TableView tv, PartView pv, uint32_t ntiles, BlendParams bp,
                                                    int32_t results) {
  merge_body<kFused, kThreads>(tv, pv, ntiles, bp, blockIdx.x, results != 0);
}

// ------------------------------------------------------------------ unstage
// The fused query: tile t's records take the values the merge pass left in
// the tile's staged entries (their positions in pv.perm).  The tile's staged
// values are read into LDS with 16-byte loads, then every thread answers
// four consecutive records at a time (8-byte perm loads, 16-byte stores when
// the output rows are 16-byte aligned; non-temporal, since no kernel of the
// iteration reads the answers again).
constexpr uint32_t kUnstageThreads = 512;

__device__ __forceinline__ void unstage_one(const float* s_res, uint32_t count, uint32_t pos, float& r,
                                            float& g, float& b, uint8_t& f) {
  r = g = b = 0.0f;
  f = 0;
  if (pos == kNoPos || pos >= count) return;
  const float x = s_res[3 * pos];
  if (__float_as_uint(x) == kDroppedBits) return;
  r = x;
  g = s_res[3 * pos + 1];
  b = s_res[3 * pos + 2];
  f = 1;
}

__device__ __forceinline__ void unstage_body(const PartView& pv, uint32_t P, uint64_t n, uint32_t t,
                                             float* out, uint8_t* found) {
  extern __shared__ float s_res[];  // tile * 3
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint64_t t0 = (uint64_t)t * pv.tile;
  const uint32_t count = pv.runs[(uint64_t)t * (P + 1) + P];
  // the answers (r, g, b of each 16-byte entry) packed into LDS
  const float4* src = pv.stage_v + t0;
  for (uint32_t i = tid; i < count; i += nt) {
    const float4 v = src[i];
    s_res[3 * i] = v.x;
    s_res[3 * i + 1] = v.y;
    s_res[3 * i + 2] = v.z;
  }
  __syncthreads();
  const uint64_t end = t0 + pv.tile < n ? t0 + pv.tile : n;
  const bool vec = (n & 3u) == 0 && ((uintptr_t)out & 15u) == 0 && ((uintptr_t)found & 3u) == 0;
  for (uint64_t i = t0 + 4ull * tid; i < end; i += 4ull * nt) {
    float r[4], g[4], b[4];
    uint8_t f[4];
    if (i + 4 <= end) {
      // i is a multiple of 4 and perm is 256-byte aligned
      const ushort4 pp = *reinterpret_cast<const ushort4*>(pv.perm + i);
      unstage_one(s_res, count, pp.x, r[0], g[0], b[0], f[0]);
      unstage_one(s_res, count, pp.y, r[1], g[1], b[1], f[1]);
      unstage_one(s_res, count, pp.z, r[2], g[2], b[2], f[2]);
      unstage_one(s_res, count, pp.w, r[3], g[3], b[3], f[3]);
    } else {
      for (int k = 0; k < 4; ++k) {
        const uint32_t pos = i + k < end ? pv.perm[i + k] : kNoPos;
        unstage_one(s_res, count, pos, r[k], g[k], b[k], f[k]);
      }
    }
    if (vec && i + 4 <= end) {
      typedef float v4f __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(v4f{r[0], r[1], r[2], r[3]}, reinterpret_cast<v4f*>(out + i));
      __builtin_nontemporal_store(v4f{g[0], g[1], g[2], g[3]}, reinterpret_cast<v4f*>(out + n + i));
      __builtin_nontemporal_store(v4f{b[0], b[1], b[2], b[3]}, reinterpret_cast<v4f*>(out + 2 * n + i));
      if (found) *reinterpret_cast<uchar4*>(found + i) = make_uchar4(f[0], f[1], f[2], f[3]);
    } else {
      for (int k = 0; k < 4; ++k) {
        if (i + k >= end) break;
        out[i + k] = r[k];
        out[n + i + k] = g[k];
        out[2 * n + i + k] = b[k];
        if (found) found[i + k] = f[k];
      }
    }
  }
}

__global__ void __launch_bounds__(kUnstageThreads) k_unstage(PartView pv, uint32_t P, uint64_t n, float* out,
                                                             uint8_t* found) {
  unstage_body(pv, P, n, blockIdx.x, out, found);
}

// ------------------------------------------------------------------ launchers
static size_t bin_lds(uint32_t P, uint32_t per) {
  const size_t hist = (size_t)(P + 1) * 4, stage = (size_t)kBinThreads * per * bin_lds_per_record(per);
  return hist > stage ? hist : stage;
}

// A merge block whose LDS leaves room for no second block on a CU (160 KB)
// takes 1024 threads, so that the CU still runs 16 waves.
static bool merge_wide(size_t lds) { return lds > 80 * 1024; }

static size_t merge_lds(const TableView& tv) {
  return (size_t)(1u << tv.part_log2) * (8 + 4 + 24 + ((tv.var || weighted(tv)) ? 8 : 0) + 2);
}

// Raise a kernel's dynamic-LDS limit only as far as the launch needs (and
// only when it exceeds the default 64 KiB).  The limit belongs to the
// function on the current device; the largest value set is remembered per
// device (devices past the table are set on every launch).
constexpr int kLdsDevices = 64;
struct LdsLimit {
  std::atomic<int> bytes[kLdsDevices];
};

static hipError_t lds_limit(const void* fn, size_t bytes, LdsLimit* cur) {
  if (bytes <= 65536) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const bool known = dev >= 0 && dev < kLdsDevices;
  if (known && (int)bytes <= cur->bytes[dev].load(std::memory_order_relaxed)) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess && known) {
    int prev = cur->bytes[dev].load(std::memory_order_relaxed);
    while ((int)bytes > prev && !cur->bytes[dev].compare_exchange_weak(prev, (int)bytes)) {
    }
  }
  return e;
}

static bool partition_ok(const TableView& tv, const PartView& pv, uint64_t n) {
  return n <= pv.capacity && tv.part_log2 <= kMaxPartLog2 && pv.tile % kBinThreads == 0 &&
         bin_per_ok(pv.tile / kBinThreads) && (1u << (tv.log2_slots - tv.part_log2)) <= kTouchEntries;
}

template <uint32_t kPer, uint32_t kX>
static hipError_t launch_bin_t(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                               const PartView& pv, size_t shm, uint32_t ntiles, hipStream_t s) {
  static LdsLimit lim;  // one per instantiation
  hipError_t e = lds_limit(reinterpret_cast<const void*>(&k_bin<kPer, kX>), shm, &lim);
  if (e != hipSuccess) return e;
  k_bin<kPer, kX><<<ntiles, kBinThreads, shm, s>>>(rec, n, kp, tv, pv);
  return hipGetLastError();
}

template <uint32_t kPer>
static hipError_t launch_bin_x(uint32_t x, const RecPtrs& rec, uint64_t n, const KeyParams& kp,
                               const TableView& tv, const PartView& pv, size_t shm, uint32_t ntiles,
                               hipStream_t s) {
  switch (x) {
    case 0: return launch_bin_t<kPer, 0>(rec, n, kp, tv, pv, shm, ntiles, s);
    case kXFootprint: return launch_bin_t<kPer, kXFootprint>(rec, n, kp, tv, pv, shm, ntiles, s);
    case kXWeight: return launch_bin_t<kPer, kXWeight>(rec, n, kp, tv, pv, shm, ntiles, s);
    default: return launch_bin_t<kPer, kXFootprint | kXWeight>(rec, n, kp, tv, pv, shm, ntiles, s);
  }
}

// What a launch's records carry (kX bits); weights need the staging array.
static uint32_t record_extras(const RecPtrs& rec) {
  return (rec.footprint ? kXFootprint : 0u) | (rec.weight ? kXWeight : 0u);
}

hipError_t launch_bin(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                      const PartView& pv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!partition_ok(tv, pv, n)) return hipErrorInvalidValue;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t per = pv.tile / kBinThreads;
  const uint32_t ntiles = (uint32_t)((n + pv.tile - 1) / pv.tile);
  const size_t shm = bin_lds(P, per);
  const uint32_t x = record_extras(rec);
  if ((x & kXWeight) && !weighted(tv)) return hipErrorInvalidValue;
  if (per == 8) return launch_bin_x<8>(x, rec, n, kp, tv, pv, shm, ntiles, s);
  if (per == 12) return launch_bin_x<12>(x, rec, n, kp, tv, pv, shm, ntiles, s);
  return launch_bin_x<16>(x, rec, n, kp, tv, pv, shm, ntiles, s);
}

hipError_t launch_merge(uint64_t n, const TableView& tv, const PartView& pv, const BlendParams* fuse,
                        bool results, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!partition_ok(tv, pv, n)) return hipErrorInvalidValue;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t ntiles = (uint32_t)((n + pv.tile - 1) / pv.tile);
  const size_t shm = merge_lds(tv);
  // staged lookup-only entries exist exactly when the bin pass wrote perm
  if (results != (pv.perm != nullptr) || (results && !fuse)) return hipErrorInvalidValue;
  static LdsLimit lim[4];
  const bool wide = merge_wide(shm);
  const void* fn = fuse ? (wide ? reinterpret_cast<const void*>(&k_merge<true, 1024>)
                                : reinterpret_cast<const void*>(&k_merge<true, kMergeThreads>))
                        : (wide ? reinterpret_cast<const void*>(&k_merge<false, 1024>)
                                : reinterpret_cast<const void*>(&k_merge<false, kMergeThreads>));
  hipError_t e = lds_limit(fn, shm, &lim[(fuse ? 2 : 0) + (wide ? 1 : 0)]);
  if (e != hipSuccess) return e;
  const int32_t res = results ? 1 : 0;
  if (fuse && wide)
    k_merge<true, 1024><<<P, 1024, shm, s>>>(tv, pv, ntiles, *fuse, res);
  else if (fuse)
    k_merge<true, kMergeThreads><<<P, kMergeThreads, shm, s>>>(tv, pv, ntiles, *fuse, res);
  else if (wide)
    k_merge<false, 1024><<<P, 1024, shm, s>>>(tv, pv, ntiles, BlendParams{}, 0);
  else
    k_merge<false, kMergeThreads><<<P, kMergeThreads, shm, s>>>(tv, pv, ntiles, BlendParams{}, 0);
  return hipGetLastError();
}

static size_t unstage_lds(uint32_t tile) { return (size_t)tile * 12; }

uint32_t transpose_blocks(uint32_t ntiles, uint32_t P) {
  return ((ntiles + kTransposeDim - 1) / kTransposeDim) * ((P + 1 + kTransposeDim - 1) / kTransposeDim);
}

bool transpose_pays(uint32_t ntiles, uint32_t P) { return (uint64_t)ntiles * (P + 1) >= kTransposeMinWords; }

hipError_t launch_transpose_runs(const TableView& tv, const PartView& pv, uint32_t ntiles, hipStream_t s) {
  if (ntiles == 0 || !pv.runs_t) return hipSuccess;
  if (ntiles > pv.max_tiles) return hipErrorInvalidValue;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const dim3 grid((ntiles + kTransposeDim - 1) / kTransposeDim, (P + 1 + kTransposeDim - 1) / kTransposeDim);
  k_transpose_runs<<<grid, kTransposeThreads, 0, s>>>(pv, P, ntiles);
  return hipGetLastError();
}

hipError_t launch_unstage(uint64_t n, const TableView& tv, const PartView& pv, float* out,
                          uint8_t* found, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!partition_ok(tv, pv, n) || !pv.perm) return hipErrorInvalidValue;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t ntiles = (uint32_t)((n + pv.tile - 1) / pv.tile);
  const size_t shm = unstage_lds(pv.tile);
  static LdsLimit lim;
  hipError_t e = lds_limit(reinterpret_cast<const void*>(&k_unstage), shm, &lim);
  if (e != hipSuccess) return e;
  k_unstage<<<ntiles, kUnstageThreads, shm, s>>>(pv, P, n, out, found);
  return hipGetLastError();
}


// ------------------------------------------------------------------ batched sessions
// One launch per pass covers every session: a block finds its session by
// its index among the sessions' block ranges and runs the single-table body
// with the session's views, copied out of the descriptor first (read in
// place, the descriptor is global memory the body's stores might alias, so
// its fields would be loaded again after every store: the batched merge ran
// 15 % slower than the single-table one that way).  begins[0..k) holds each session's first block
// of the pass (non-decreasing, begins[0] = 0); the block's session is the
// last one starting at or before it: one coalesced load and a ballot per 64
// sessions (a scan through the descriptors would cost a dependent load per
// session).  Called by whole waves; the result is wave-uniform.
__device__ __forceinline__ uint32_t find_session(const uint32_t* begins, uint32_t k, uint32_t b) {
  uint32_t count = 0;
  for (uint32_t c = 0; c < k; c += 64) {
    const uint32_t i = c + __lane_id();
    count += (uint32_t)__popcll(__ballot(i < k && begins[i] <= b));
  }
  return count - 1;
}

__global__ void __launch_bounds__(kTransposeThreads) k_transpose_batch(const BatchSession* ss, const uint32_t* bg,
                                                                       uint32_t k) {
  const BatchSession& S = ss[find_session(bg, k, blockIdx.x)];
  const uint32_t local = blockIdx.x - S.trans_begin;
  const PartView pv = S.pv;
  if (local >= S.ntrans || !pv.runs_t) return;
  const uint32_t P = 1u << (S.tv.log2_slots - S.tv.part_log2);
  const uint32_t ntiles = S.ntiles;
  const uint32_t gx = (ntiles + kTransposeDim - 1) / kTransposeDim;
  transpose_body(pv, P, ntiles, local % gx, local / gx);
}

// kX: the union of the sessions' record extras; each session runs the body
// of its own.
template <uint32_t kPer, uint32_t kW, uint32_t kFpAllowed>
__device__ __forceinline__ void bin_session(const BatchSession& S, uint32_t local) {
  const RecPtrs rec = S.rec;
  const KeyParams kp = S.kp;
  const TableView tv = S.tv;
  const PartView pv = S.pv;
  const uint64_t n = S.n;
  if (kFpAllowed && rec.footprint)
    bin_body<kPer, kW | kXFootprint>(rec, n, kp, tv, pv, local);
  else
    bin_body<kPer, kW>(rec, n, kp, tv, pv, local);
}

// (the batch instantiations that carry several bodies would spill heavily
// under the same cap)
template <uint32_t kPer, uint32_t kX>
__global__ void __launch_bounds__(kBinThreads) __attribute__((amdgpu_waves_per_eu(kPer <= 12 && kX == 0 ? 4 : 1)))
k_bin_batch(const BatchSession* ss, const uint32_t* bg, uint32_t k) {
  const BatchSession& S = ss[find_session(bg, k, blockIdx.x)];
  const uint32_t local = blockIdx.x - S.tile_begin;
  if (local >= S.ntiles) return;
  if constexpr ((kX & kXWeight) != 0) {
    if (S.rec.weight) {
      bin_session<kPer, kXWeight, kX & kXFootprint>(S, local);
      return;
    }
  }
  bin_session<kPer, 0, kX & kXFootprint>(S, local);
}

// 1024 threads per block when the widest session's partitions leave room
// for one block per CU, else 512.
template <int kThreads>
__global__ void __launch_bounds__(kThreads) k_merge_batch(const BatchSession* ss, const uint32_t* bg, uint32_t k) {
  const BatchSession& S = ss[find_session(bg, k, blockIdx.x)];
  const uint32_t local = blockIdx.x - S.part_begin;
  if (local >= S.nparts) return;
  const TableView tv = S.tv;
  const PartView pv = S.pv;
  const BlendParams bp = S.bp;
  merge_body<true, kThreads>(tv, pv, S.ntiles, bp, local, S.fused_query != 0);
}

// A session whose queries are its records takes one unstage block per tile;
// any other session one lookup block per kQueryBlock queries.
__global__ void __launch_bounds__(kQueryBlock) k_query_batch(const BatchSession* ss, const uint32_t* bg,
                                                              uint32_t k) {
  const BatchSession& S = ss[find_session(bg, k, blockIdx.x)];
  const uint32_t local = blockIdx.x - S.qblk_begin;
  float* out = S.out;
  uint8_t* found = S.found;
  if (S.fused_query) {
    const PartView pv = S.pv;
    if (local < S.ntiles)
      unstage_body(pv, 1u << (S.tv.log2_slots - S.tv.part_log2), S.n, local, out, found);
    return;
  }
  const uint64_t nq = S.nq;
  const uint64_t i = (uint64_t)local * kQueryBlock + threadIdx.x;
  if (i >= nq) return;
  const TableView tv = S.tv;
  const KeyParams kp = S.kp;
  const QryPtrs q = S.q;
  float rgb[3];
  const uint8_t hit = lookup_key(tv, S.bp.dtype, query_key(kp, q, i), rgb);
  out[i] = rgb[0];
  out[nq + i] = rgb[1];
  out[2 * nq + i] = rgb[2];
  if (found) found[i] = hit;
}

template <uint32_t kPer, uint32_t kX>
static hipError_t launch_bin_batch_t(const BatchSession* d_ss, const uint32_t* bg, uint32_t k, uint32_t tiles,
                                     size_t lds, hipStream_t s) {
  static LdsLimit lim;  // one per instantiation
  hipError_t e = lds_limit(reinterpret_cast<const void*>(&k_bin_batch<kPer, kX>), lds, &lim);
  if (e != hipSuccess) return e;
  k_bin_batch<kPer, kX><<<tiles, kBinThreads, lds, s>>>(d_ss, bg, k);
  return hipGetLastError();
}

template <uint32_t kPer>
static hipError_t launch_bin_batch_x(uint32_t x, const BatchSession* d_ss, const uint32_t* bg, uint32_t k,
                                     uint32_t tiles, size_t lds, hipStream_t s) {
  switch (x) {
    case 0: return launch_bin_batch_t<kPer, 0>(d_ss, bg, k, tiles, lds, s);
    case kXFootprint: return launch_bin_batch_t<kPer, kXFootprint>(d_ss, bg, k, tiles, lds, s);
    case kXWeight: return launch_bin_batch_t<kPer, kXWeight>(d_ss, bg, k, tiles, lds, s);
    default: return launch_bin_batch_t<kPer, kXFootprint | kXWeight>(d_ss, bg, k, tiles, lds, s);
  }
}

hipError_t launch_batch(const BatchSession* d_ss, const uint32_t* d_begins, const uint32_t* h_begins,
                        uint32_t stride, const BatchSession* h_ss, uint32_t k, hipStream_t s) {
  if (k == 0) return hipSuccess;
  if (k > stride) return hipErrorInvalidValue;
  uint32_t tiles = 0, parts = 0, qblks = 0, trans = 0;
  size_t lds_b = 0, lds_m = 0, lds_q = 0;
  uint32_t x = 0;  // what any session's records carry
  const uint32_t per = h_ss[0].pv.tile / kBinThreads;
  for (uint32_t i = 0; i < k; ++i) {
    const BatchSession& S = h_ss[i];
    if (h_begins[i] != S.tile_begin || h_begins[stride + i] != S.part_begin ||
        h_begins[2 * stride + i] != S.qblk_begin || h_begins[3 * stride + i] != S.trans_begin)
      return hipErrorInvalidValue;
    if (S.n == 0 || !partition_ok(S.tv, S.pv, S.n) || S.pv.tile != h_ss[0].pv.tile ||
        S.tile_begin != tiles || S.part_begin != parts || S.qblk_begin != qblks || (S.part_begin & 7u) ||
        S.trans_begin != trans ||
        S.ntrans != (S.pv.runs_t ? transpose_blocks(S.ntiles, 1u << (S.tv.log2_slots - S.tv.part_log2)) : 0u))
      return hipErrorInvalidValue;
    const uint32_t P = 1u << (S.tv.log2_slots - S.tv.part_log2);
    const size_t lb = bin_lds(P, per), lm = merge_lds(S.tv);
    lds_b = lb > lds_b ? lb : lds_b;
    lds_m = lm > lds_m ? lm : lds_m;
    if ((S.fused_query != 0) != (S.pv.perm != nullptr)) return hipErrorInvalidValue;
    if (S.fused_query) {
      if (S.nq != S.n || S.nqblk != S.ntiles) return hipErrorInvalidValue;
      lds_q = unstage_lds(S.pv.tile);
    }
    const uint32_t xs = record_extras(S.rec);
    if ((xs & kXWeight) && !weighted(S.tv)) return hipErrorInvalidValue;
    x |= xs;
    tiles += S.ntiles;
    parts += (S.nparts + 7u) & ~7u;
    qblks += S.nqblk;
    trans += S.ntrans;
  }
  static LdsLimit lim_m[2], lim_q;
  const bool wide = merge_wide(lds_m);
  const uint32_t* bg_tile = d_begins;
  const uint32_t* bg_part = d_begins + stride;
  const uint32_t* bg_qblk = d_begins + 2 * stride;
  const uint32_t* bg_trans = d_begins + 3 * stride;
  hipError_t e = per == 8    ? launch_bin_batch_x<8>(x, d_ss, bg_tile, k, tiles, lds_b, s)
                  : per == 12 ? launch_bin_batch_x<12>(x, d_ss, bg_tile, k, tiles, lds_b, s)
                              : launch_bin_batch_x<16>(x, d_ss, bg_tile, k, tiles, lds_b, s);
  if (e != hipSuccess) return e;
  e = wide ? lds_limit(reinterpret_cast<const void*>(&k_merge_batch<1024>), lds_m, &lim_m[1])
           : lds_limit(reinterpret_cast<const void*>(&k_merge_batch<kMergeThreads>), lds_m, &lim_m[0]);
  if (e == hipSuccess) e = lds_limit(reinterpret_cast<const void*>(&k_query_batch), lds_q, &lim_q);
  if (e != hipSuccess) return e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (trans) k_transpose_batch<<<trans, kTransposeThreads, 0, s>>>(d_ss, bg_trans, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (wide)
    k_merge_batch<1024><<<parts, 1024, lds_m, s>>>(d_ss, bg_part, k);
  else
    k_merge_batch<kMergeThreads><<<parts, kMergeThreads, lds_m, s>>>(d_ss, bg_part, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (qblks) k_query_batch<<<qblks, kQueryBlock, lds_q, s>>>(d_ss, bg_qblk, k);
  return hipGetLastError();
}

}  // namespace psf

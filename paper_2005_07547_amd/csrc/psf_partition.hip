// Partitioned insertion for gfx950.
//
// Global atomics on MI355X sustain only ~2e10 operations/s, far below what
// HBM streaming allows, so the fast insert path avoids them.  The table is
// split into partitions of 2^part_log2 consecutive slots (the partition of a
// key is the top bits of its hash, its probe sequence stays inside the
// partition).  Insertion then runs in two passes:
//
//   bin   -- one 1024-thread block per tile of records computes the keys,
//            counts records per partition in LDS and writes (key, rgb) to a
//            staging area grouped by partition inside the tile, plus the
//            tile's exclusive per-partition offsets;
//   merge -- one block per partition loads the partition's keys into LDS,
//            gathers that partition's staged entries from every tile, finds
//            or claims each key's slot and accumulates count and sums with
//            LDS atomics, then writes the partition back: either adding into
//            the global accumulators (plain insert) or, when the whole frame
//            is in this launch, applying the temporal blend (Eq. 10-11)
//            directly so the accumulators never touch HBM.
//
// A partition is owned by exactly one block in the merge pass, so the
// write-back uses plain loads and stores.
#include "psf_device.h"
#include "psf_internal.h"

namespace psf {

constexpr int kBinThreads = 1024;
constexpr uint32_t kBinPer = 8;  // records per thread; a tile is kBinThreads * kBinPer
constexpr int kMergeThreads = 512;
constexpr uint32_t kMaxPartLog2 = 12;

// ------------------------------------------------------------------ bin
__global__ void __launch_bounds__(kBinThreads) k_bin(RecPtrs rec, uint64_t n, KeyParams kp,
                                                     TableView tv, PartView pv) {
  extern __shared__ uint32_t s_hist[];  // P + 1 counters
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t tid = threadIdx.x;
  const uint32_t tile = blockIdx.x;
  const uint64_t t0 = (uint64_t)tile * pv.tile;
  for (uint32_t p = tid; p <= P; p += kBinThreads) s_hist[p] = 0;
  __syncthreads();

  uint64_t key[kBinPer];
  uint32_t part_rank[kBinPer];  // partition << 16 | rank, or ~0 if not staged
  float rgb[kBinPer][3];
  uint32_t n_skip = 0, n_ovf = 0;
#pragma unroll
  for (uint32_t j = 0; j < kBinPer; ++j) {
    part_rank[j] = ~0u;
    const uint64_t i = t0 + (uint64_t)j * kBinThreads + tid;
    if (i >= n) continue;
    const bool hr = rec.rough != nullptr;
    const float ro = hr ? rec.rough[i] : 0.0f;
    const bool gl = hr && ro < kp.rough_thr;
    const float r = rec.r[i], g = rec.g[i], b = rec.b[i];
    bool ovf = false;
    uint64_t k;
    bool ok = cell_key(kp, rec.px[i], rec.py[i], rec.pz[i], rec.nx[i], rec.ny[i], rec.nz[i],
                       gl ? rec.ox[i] : 0.0f, gl ? rec.oy[i] : 0.0f, gl ? rec.oz[i] : 0.0f, hr, ro,
                       k, ovf);
    ok = ok && finite3(r, g, b);
    if (!ok) {
      ++n_skip;
      continue;
    }
    n_ovf += ovf ? 1u : 0u;
    const uint32_t p = partition_of(fmix64(k), tv.log2_slots, tv.part_log2);
    const uint32_t rank = atomicAdd(&s_hist[p], 1u);
    key[j] = k;
    part_rank[j] = (p << 16) | rank;
    rgb[j][0] = r;
    rgb[j][1] = g;
    rgb[j][2] = b;
  }
  // rare-event counters: one atomic per wave when non-zero
  for (int off = 32; off > 0; off >>= 1) {
    n_skip += __shfl_xor(n_skip, off);
    n_ovf += __shfl_xor(n_ovf, off);
  }
  if (__lane_id() == 0) {
    if (n_skip) atomicAdd(&tv.stats->skipped, (unsigned long long)n_skip);
    if (n_ovf) atomicAdd(&tv.stats->coord_overflow, (unsigned long long)n_ovf);
  }
  __syncthreads();

  // exclusive scan of the P+1 counters (last one stays 0 -> becomes total)
  __shared__ uint32_t s_part[kBinThreads];
  const uint32_t cnt_total = P + 1;
  const uint32_t chunk = (cnt_total + kBinThreads - 1) / kBinThreads;
  const uint32_t lo = tid * chunk;
  uint32_t local = 0;
  for (uint32_t c = 0; c < chunk; ++c)
    if (lo + c < cnt_total) local += s_hist[lo + c];
  s_part[tid] = local;
  __syncthreads();
  for (uint32_t off = 1; off < kBinThreads; off <<= 1) {
    const uint32_t v = tid >= off ? s_part[tid - off] : 0u;
    __syncthreads();
    s_part[tid] += v;
    __syncthreads();
  }
  uint32_t run = s_part[tid] - local;  // exclusive prefix of this chunk
  for (uint32_t c = 0; c < chunk; ++c) {
    if (lo + c < cnt_total) {
      const uint32_t v = s_hist[lo + c];
      s_hist[lo + c] = run;
      run += v;
    }
  }
  __syncthreads();

  uint32_t* offs = pv.runs + (uint64_t)tile * (P + 1);
  for (uint32_t p = tid; p <= P; p += kBinThreads) offs[p] = s_hist[p];

#pragma unroll
  for (uint32_t j = 0; j < kBinPer; ++j) {
    if (part_rank[j] == ~0u) continue;
    const uint64_t pos = t0 + s_hist[part_rank[j] >> 16] + (part_rank[j] & 0xffffu);
    pv.stage_key[pos] = key[j];
    pv.stage_rgb[pos] = rgb[j][0];
    pv.stage_rgb[pv.capacity + pos] = rgb[j][1];
    pv.stage_rgb[2 * pv.capacity + pos] = rgb[j][2];
  }
}

// ------------------------------------------------------------------ merge
// bp == nullptr: add into the global accumulators; otherwise blend.
template <bool kFused>
__global__ void __launch_bounds__(kMergeThreads) k_merge(TableView tv, PartView pv, uint32_t ntiles,
                                                         BlendParams bp) {
  extern __shared__ unsigned long long s_dyn[];  // key[B] | cnt[B] | sum[3][B]
  __shared__ uint32_t s_scan[kMergeThreads];
  __shared__ uint32_t s_dropped, s_touched, s_sat;
  __shared__ uint32_t s_hist[16];
  const uint32_t tid = threadIdx.x;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t B = 1u << tv.part_log2;
  const uint32_t p = blockIdx.x;
  const uint64_t base = (uint64_t)p << tv.part_log2;
  const bool stats = (tv.flags & 1u) != 0;
  unsigned long long* s_key = s_dyn;
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_key + B);
  float* s_sum0 = reinterpret_cast<float*>(s_cnt + B);
  float* s_sum1 = s_sum0 + B;
  float* s_sum2 = s_sum1 + B;

  for (uint32_t s = tid; s < B; s += kMergeThreads) {
    s_key[s] = tv.slots[base + s].key;
    s_cnt[s] = 0;
    s_sum0[s] = s_sum1[s] = s_sum2[s] = 0.0f;
  }
  if (tid == 0) s_dropped = s_touched = s_sat = 0;
  if (tid < 16) s_hist[tid] = 0;

  // per-tile run lengths of this partition, scanned so entries can be
  // spread evenly over the block (tiles are processed kMergeThreads at a time)
  for (uint32_t t0 = 0; t0 < ntiles; t0 += kMergeThreads) {
    const uint32_t t = t0 + tid;
    uint32_t lo = 0, len = 0;
    if (t < ntiles) {
      const uint32_t* offs = pv.runs + (uint64_t)t * (P + 1);
      lo = offs[p];
      len = offs[p + 1] - lo;
    }
    __syncthreads();
    s_scan[tid] = len;
    __syncthreads();
    for (uint32_t off = 1; off < kMergeThreads; off <<= 1) {
      const uint32_t v = tid >= off ? s_scan[tid - off] : 0u;
      __syncthreads();
      s_scan[tid] += v;
      __syncthreads();
    }
    const uint32_t total = s_scan[kMergeThreads - 1];
    // entry e belongs to the tile whose inclusive prefix first exceeds e
    for (uint32_t e = tid; e < total; e += kMergeThreads) {
      uint32_t a = 0, b = kMergeThreads - 1;
      while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (s_scan[m] > e) b = m; else a = m + 1;
      }
      const uint32_t tt = t0 + a;
      const uint32_t before = a ? s_scan[a - 1] : 0u;
      const uint32_t* offs = pv.runs + (uint64_t)tt * (P + 1);
      const uint64_t pos = (uint64_t)tt * pv.tile + offs[p] + (e - before);
      const unsigned long long key = pv.stage_key[pos];
      const float r = pv.stage_rgb[pos];
      const float g = pv.stage_rgb[pv.capacity + pos];
      const float b2 = pv.stage_rgb[2 * pv.capacity + pos];
      const uint32_t start = (uint32_t)fmix64(key) & (B - 1);
      uint32_t slot = ~0u;
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
        atomicAdd(&s_dropped, 1u);
        continue;
      }
      if (stats) atomicAdd(&s_hist[i < 15 ? i : 15], 1u);
      atomicAdd(&s_cnt[slot], 1u);
      atomicAdd(&s_sum0[slot], r);
      atomicAdd(&s_sum1[slot], g);
      atomicAdd(&s_sum2[slot], b2);
    }
  }
  __syncthreads();

  // write the partition back
  bool sat = false;
  uint32_t touched = 0;
  for (uint32_t s = tid; s < B; s += kMergeThreads) {
    const uint32_t c = s_cnt[s];
    if (c == 0) continue;
    const uint64_t g = base + s;
    Slot* d = &tv.slots[g];
    if (kFused) {
      const uint32_t c_old = d->c_old;
      const float alpha = blend_alpha(bp, c, c_old);
      const float inv = 1.0f / (float)c;
      float L[3];
      load_state(*d, bp.dtype, L[0], L[1], L[2]);
      float out[3];
      const float sums[3] = {s_sum0[s], s_sum1[s], s_sum2[s]};
      for (int ch = 0; ch < 3; ++ch) {
        const float m = sums[ch] * inv;
        out[ch] = alpha == 1.0f ? m : (1.0f - alpha) * L[ch] + alpha * m;
      }
      uint32_t enc[4];
      encode_state(bp.dtype, out[0], out[1], out[2], enc, sat);
      d->key = s_key[s];
      d->c_old = c_old + c;
      *reinterpret_cast<uint4*>(d->L) = make_uint4(enc[0], enc[1], enc[2], enc[3]);
      ++touched;
    } else {
      Acc a = tv.acc[g];
      a.n += c;
      a.s[0] += s_sum0[s];
      a.s[1] += s_sum1[s];
      a.s[2] += s_sum2[s];
      tv.acc[g] = a;
      d->key = s_key[s];
    }
  }
  if (kFused) {
    for (int off = 32; off > 0; off >>= 1) touched += __shfl_xor(touched, off);
    if (__lane_id() == 0 && touched) atomicAdd(&s_touched, touched);
    if (sat) atomicAdd(&s_sat, 1u);
  }
  __syncthreads();
  if (tid == 0) {
    if (s_dropped) atomicAdd(&tv.stats->dropped, (unsigned long long)s_dropped);
    if (kFused) {
      if (s_sat) atomicAdd(&tv.stats->saturated, (unsigned long long)s_sat);
      if (s_touched) atomicAdd(&tv.stats->touched_count, s_touched);
      __threadfence();
      const uint32_t done = atomicAdd(&tv.stats->done_blocks, 1u);
      if (done == gridDim.x - 1) {
        const uint32_t cnt = __hip_atomic_load(&tv.stats->touched_count, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        tv.stats->touched_last = cnt;
        tv.stats->touched_total += cnt;
        tv.stats->updates += 1;
        tv.stats->touched_count = 0;
        tv.stats->done_blocks = 0;
        __threadfence();
      }
    }
  }
  if (stats && tid < 16 && s_hist[tid])
    atomicAdd(&tv.stats->probe_hist[tid], (unsigned long long)s_hist[tid]);
}

static hipError_t merge_attr() {
  static bool done = false;
  if (done) return hipSuccess;
  const int lim = (int)((size_t)(1u << kMaxPartLog2) * (8 + 4 + 12));
  hipError_t a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_merge<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (a == hipSuccess)
    a = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_merge<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (a == hipSuccess) done = true;
  return a;
}

bool partition_ok(const TableView& tv, const PartView& pv, uint64_t n) {
  return n <= pv.capacity && tv.part_log2 <= kMaxPartLog2 && pv.tile == kBinThreads * kBinPer;
}

hipError_t launch_bin(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                      const PartView& pv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!partition_ok(tv, pv, n)) return hipErrorInvalidValue;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t ntiles = (uint32_t)((n + pv.tile - 1) / pv.tile);
  k_bin<<<ntiles, kBinThreads, (size_t)(P + 1) * sizeof(uint32_t), s>>>(rec, n, kp, tv, pv);
  return hipGetLastError();
}

hipError_t launch_merge(uint64_t n, const TableView& tv, const PartView& pv, const BlendParams* fuse,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!partition_ok(tv, pv, n)) return hipErrorInvalidValue;
  hipError_t e = merge_attr();
  if (e != hipSuccess) return e;
  const uint32_t P = 1u << (tv.log2_slots - tv.part_log2);
  const uint32_t ntiles = (uint32_t)((n + pv.tile - 1) / pv.tile);
  const size_t shm = (size_t)(1u << tv.part_log2) * (8 + 4 + 12);
  if (fuse)
    k_merge<true><<<P, kMergeThreads, shm, s>>>(tv, pv, ntiles, *fuse);
  else
    k_merge<false><<<P, kMergeThreads, shm, s>>>(tv, pv, ntiles, BlendParams{});
  return hipGetLastError();
}

}  // namespace psf

// PSTF hash-filter kernels for gfx950: direct (wave-merged) insertion, the
// streaming temporal blend, lookups, key output, resets and
// export support.  The partitioned insertion lives in psf_partition.hip.
#include "psf_device.h"
#include "psf_internal.h"

namespace psf {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t lane) {
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, (int)lane);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)lane);
  return ((uint64_t)hi << 32) | lo;
}

// Add a per-wave count to a device counter with one atomic from lane 0.
__device__ __forceinline__ void wave_count(unsigned long long* ctr, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m && lane_id() == (uint32_t)__ffsll((unsigned long long)m) - 1)
    atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// Find or claim the slot of key along its probe sequence.  Returns the slot
// index or ~0 when max_probe slots were all taken by other keys.  *probes
// receives the number of slots examined.
__device__ __forceinline__ uint64_t find_or_claim(const TableView& tv, uint64_t key, uint32_t* probes) {
  const ProbeSeq ps = probe_seq(key, tv.log2_slots, tv.part_log2);
  for (uint32_t i = 0; i < tv.max_probe; ++i) {
    const uint64_t s = ps.at(i);
    unsigned long long* kp = &tv.slots[s].key;
    unsigned long long cur = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kEmpty) {
      cur = atomicCAS(kp, kEmpty, (unsigned long long)key);
      if (cur == kEmpty) tv.keys[s] = key;  // this lane claimed the slot
    }
    if (cur == kEmpty || cur == key) {
      *probes = i + 1;
      return s;
    }
  }
  *probes = tv.max_probe;
  return ~0ull;
}

__device__ __forceinline__ uint64_t find_slot(const TableView& tv, uint64_t key) {
  const ProbeSeq ps = probe_seq(key, tv.log2_slots, tv.part_log2);
  for (uint32_t i = 0; i < tv.max_probe; ++i) {
    const uint64_t s = ps.at(i);
    const unsigned long long cur = tv.slots[s].key;
    if (cur == key) return s;
    if (cur == kEmpty) return ~0ull;
  }
  return ~0ull;
}

// ------------------------------------------------------------------ keys
__global__ void __launch_bounds__(256) k_keys(RecPtrs rec, uint64_t n, KeyParams kp,
                                              unsigned long long* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t key;
  bool ovf;
  const bool hr = rec.rough != nullptr;
  const bool g = hr && rec.rough[i] < kp.rough_thr;
  const bool hf = rec.footprint != nullptr;
  const bool ok = cell_key(kp, rec.px[i], rec.py[i], rec.pz[i], rec.nx[i], rec.ny[i], rec.nz[i],
                           g ? rec.ox[i] : 0.0f, g ? rec.oy[i] : 0.0f, g ? rec.oz[i] : 0.0f, hr,
                           hr ? rec.rough[i] : 0.0f, hf, hf ? rec.footprint[i] : 0.0f, key, ovf);
  out[i] = ok ? key : kEmpty;
}

// ------------------------------------------------------------------ direct insert
// One record per lane.  Lanes of a wave holding the same key elect the lowest
// lane as leader; sums are merged in LDS; each leader claims its slot with a
// 64-bit CAS and adds the merged count and sums with global atomics.  In a
// weighted table the sums are of w * value and the counter adds the weights
// (binary32 atomics on the counter word).  A table that keeps the luminance
// variance also adds each sample's squared luminance (binary64) to acc_q.
constexpr int kInsBlock = 256;

__global__ void __launch_bounds__(kInsBlock) k_insert_direct(RecPtrs rec, uint64_t n, KeyParams kp,
                                                             TableView tv) {
  __shared__ float s_sum[kInsBlock][3];
  __shared__ uint32_t s_cnt[kInsBlock];
  __shared__ float s_w[kInsBlock];
  __shared__ double s_q[kInsBlock];
  __shared__ uint32_t s_hist[16];
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t wbase = tid & ~63u;
  const bool stats = (tv.flags & 1u) != 0;
  if (stats && tid < 16) s_hist[tid] = 0;
  s_sum[tid][0] = s_sum[tid][1] = s_sum[tid][2] = 0.0f;
  s_cnt[tid] = 0;
  s_w[tid] = 0.0f;
  s_q[tid] = 0.0;
  const bool wtd = weighted(tv);
  __syncthreads();

  const uint64_t i = (uint64_t)blockIdx.x * kInsBlock + tid;
  bool valid = false;
  bool skip = false;
  uint64_t key = kEmpty;
  bool ovf = false;
  float r = 0.0f, g = 0.0f, b = 0.0f, w = 1.0f;
  if (i < n) {
    const bool hr = rec.rough != nullptr;
    const float ro = hr ? ld_once(rec.rough + i) : 0.0f;
    const bool gl = hr && ro < kp.rough_thr;
    r = ld_once(rec.r + i);
    g = ld_once(rec.g + i);
    b = ld_once(rec.b + i);
    const bool hf = rec.footprint != nullptr;
    valid = cell_key(kp, ld_once(rec.px + i), ld_once(rec.py + i), ld_once(rec.pz + i), ld_once(rec.nx + i),
                     ld_once(rec.ny + i), ld_once(rec.nz + i), gl ? ld_once(rec.ox + i) : 0.0f,
                     gl ? ld_once(rec.oy + i) : 0.0f, gl ? ld_once(rec.oz + i) : 0.0f, hr, ro, hf,
                     hf ? ld_once(rec.footprint + i) : 0.0f, key, ovf);
    valid = valid && finite3(r, g, b);
    if (rec.weight) {
      w = ld_once(rec.weight + i);
      valid = valid && __builtin_isfinite(w) && w > 0.0f;
      r *= w;
      g *= w;
      b *= w;
    }
    skip = !valid;
  }
  wave_count(stat_lane(tv.stats->skipped, blockIdx.x), skip);
  wave_count(stat_lane(tv.stats->coord_overflow, blockIdx.x), valid && ovf);

  // elect a leader lane per distinct key
  uint64_t pending = __ballot(valid);
  uint32_t leader = 64;
  while (pending) {
    const uint32_t l = (uint32_t)__ffsll((unsigned long long)pending) - 1;
    const uint64_t lk = readlane64(key, l);
    const bool mine = valid && leader == 64 && key == lk;
    const uint64_t m = __ballot(mine);
    if (mine) leader = l;
    pending &= ~m;
  }
  if (valid) {
    atomicAdd(&s_cnt[wbase + leader], 1u);
    if (wtd) atomicAdd(&s_w[wbase + leader], w);
    atomicAdd(&s_sum[wbase + leader][0], r);
    atomicAdd(&s_sum[wbase + leader][1], g);
    atomicAdd(&s_sum[wbase + leader][2], b);
    if (tv.acc_q) {
      const double y = luma64(r, g, b);
      atomicAdd(&s_q[wbase + leader], y * y);
    }
  }
  __syncthreads();

  const bool lead = valid && leader == lane;
  uint64_t slot = ~0ull;
  uint32_t cnt = 0;
  if (lead) {
    cnt = s_cnt[tid];
    uint32_t probes;
    slot = find_or_claim(tv, key, &probes);
    if (slot != ~0ull) {
      Acc* a = &tv.acc[slot];
      if (wtd)
        atomicAdd(reinterpret_cast<float*>(&a->n), s_w[tid]);
      else
        atomicAdd(&a->n, cnt);
      atomicAdd(&a->s[0], s_sum[tid][0]);
      atomicAdd(&a->s[1], s_sum[tid][1]);
      atomicAdd(&a->s[2], s_sum[tid][2]);
      if (tv.acc_q) atomicAdd(&tv.acc_q[slot], s_q[tid]);
      if (stats) atomicAdd(&s_hist[probes - 1 < 15 ? probes - 1 : 15], 1u);
    } else {
      atomicAdd(&tv.stats->dropped, (unsigned long long)cnt);
    }
  }
  if (stats) {
    __syncthreads();
    if (tid < 16 && s_hist[tid]) atomicAdd(&tv.stats->probe_hist[tid], (unsigned long long)s_hist[tid]);
  }
}

// ------------------------------------------------------------------ temporal update
// Blend one slot's accumulated frame into its state (Eq. 10-11) and clear the
// accumulator.  Returns true if the slot had samples.
__device__ __forceinline__ bool blend_slot(const TableView& tv, const BlendParams& bp, uint64_t s,
                                           bool& sat) {
  const Acc a = tv.acc[s];
  if (a.n == 0) return false;
  const bool wtd = weighted(tv);
  Slot* d = &tv.slots[s];
  const uint32_t c_old = d->c_old;
  const float alpha = blend_alpha(bp, a.n, c_old, wtd);
  const float inv = 1.0f / counter_value(a.n, wtd);
  float L[3];
  load_blend_state(*d, bp.dtype, L[0], L[1], L[2]);
  float out[3];
  for (int c = 0; c < 3; ++c) {
    const float m = a.s[c] * inv;
    out[c] = alpha == 1.0f ? m : (1.0f - alpha) * L[c] + alpha * m;
  }
  uint32_t enc[4], pad;
  encode_state(bp.dtype, out[0], out[1], out[2], enc, pad, sat);
  if (tv.var) {
    double m, s2;
    frame_moments(a.s[0], a.s[1], a.s[2], tv.acc_q[s], (double)a.n, m, s2);
    tv.var[s] = blend_variance(tv.var[s], alpha, luma32(L[0], L[1], L[2]), m, s2);
    tv.acc_q[s] = 0.0;
  }
  d->c_old = counter_add(c_old, a.n, wtd);
  d->pad = pad;
  *reinterpret_cast<uint4*>(d->L) = make_uint4(enc[0], enc[1], enc[2], enc[3]);
  tv.acc[s] = Acc{0u, {0.0f, 0.0f, 0.0f}};
  return true;
}

// Streaming pass over every slot's accumulator; each block records how many
// cells it blended in its own BlockTouch entry.
__global__ void __launch_bounds__(256) k_update(TableView tv, BlendParams bp, uint64_t nslots) {
  __shared__ uint32_t s_touched, s_sat;
  if (threadIdx.x == 0) s_touched = s_sat = 0;
  __syncthreads();
  bool sat = false;
  uint32_t touched = 0;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x)
    touched += blend_slot(tv, bp, s, sat) ? 1u : 0u;
  for (int off = 32; off > 0; off >>= 1) touched += __shfl_xor(touched, off);
  if (lane_id() == 0 && touched) atomicAdd(&s_touched, touched);
  if (sat) atomicAdd(&s_sat, 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_sat) atomicAdd(&tv.stats->saturated, (unsigned long long)s_sat);
    BlockTouch* bt = &tv.touch[blockIdx.x];
    bt->last = s_touched;
    bt->total += s_touched;
  }
}

// ------------------------------------------------------------------ query
__global__ void __launch_bounds__(256) k_query(QryPtrs q, uint64_t n, KeyParams kp, TableView tv,
                                               int32_t dtype, float* out, uint8_t* found) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float rgb[3];
  const uint8_t hit = lookup_key(tv, dtype, query_key(kp, q, i), rgb);
  st_once(out + i, rgb[0]);
  st_once(out + n + i, rgb[1]);
  st_once(out + 2 * n + i, rgb[2]);
  if (found) found[i] = hit;
}

// ------------------------------------------------------------------ multi-level lookup
// Sec. 2.3: finite elements come in a hierarchy of levels.  A vertex whose
// own cell has no blended value is answered by the finest coarser cell
// (same normal and direction bins) that has one, at most `up` levels up.
__global__ void __launch_bounds__(256) k_query_hier(QryPtrs q, uint64_t n, uint32_t up, KeyParams kp,
                                                    TableView tv, int32_t dtype, float* out,
                                                    uint8_t* level_out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float rgb[3] = {0.0f, 0.0f, 0.0f};
  uint8_t lv = 0;
  for (uint32_t k = 0; k <= up; ++k) {
    const uint64_t key = query_key(kp, q, i, (int32_t)k);
    if (key == kEmpty) break;  // invalid vertex, or past the coarsest level
    if (lookup_key(tv, dtype, key, rgb)) {
      lv = (uint8_t)(k + 1);
      break;
    }
  }
  out[i] = rgb[0];
  out[n + i] = rgb[1];
  out[2 * n + i] = rgb[2];
  if (level_out) level_out[i] = lv;
}

// ------------------------------------------------------------------ two-field estimators
// Sec. 4.2 (Eq. 25) and Sec. 5 (Eq. 28): the control variate h = f~L_i(x,
// w_i) has the known integral L~o\e(x, w_o).  mode 0: wp (g - beta h) +
// beta L; mode 1: gamma wp (g - h) + L.  Either cell missing: wp g.
constexpr uint32_t kEstThreads = 256, kEstPerThread = 1;

__global__ void __launch_bounds__(kEstThreads) k_estimate(EstPtrs a, uint64_t n, KeyParams kp_o,
                                                          TableView tv_o, int32_t dt_o, KeyParams kp_i,
                                                          TableView tv_i, int32_t dt_i, int32_t mode,
                                                          float param, float* out, uint8_t* applied) {
  // kEstPerThread vertices per thread: all their first probes (two per
  // vertex) are in flight together; indices past the end read the last
  // vertex and write nothing
  const uint64_t i0 = (uint64_t)blockIdx.x * (kEstThreads * kEstPerThread) + threadIdx.x;
  PendingLookup lo[kEstPerThread], li[kEstPerThread];
#pragma unroll
  for (uint32_t v = 0; v < kEstPerThread; ++v) {
    const uint64_t i = i0 + (uint64_t)v * kEstThreads;
    const uint64_t ic = i < n ? i : n - 1;
    lo[v] = lookup_first(tv_o, query_key(kp_o, a.qo, ic));
    li[v] = lookup_first(tv_i, query_key(kp_i, a.qi, ic));
  }
#pragma unroll
  for (uint32_t v = 0; v < kEstPerThread; ++v) {
    const uint64_t i = i0 + (uint64_t)v * kEstThreads;
    if (i >= n) break;
    float L[3], h[3];
    const uint8_t fo = lookup_finish(tv_o, dt_o, lo[v], L);
    const uint8_t fi = lookup_finish(tv_i, dt_i, li[v], h);
    const float g[3] = {ld_once(a.gr + i), ld_once(a.gg + i), ld_once(a.gb + i)};
    const float w = ld_once(a.wp + i);
    const bool both = fo && fi;
    float e[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (!both) {
        e[c] = w * g[c];
      } else if (mode == 0) {
        const float corr = w * (g[c] - param * h[c]);
        e[c] = corr + param * L[c];
      } else {
        const float corr = param * (w * (g[c] - h[c]));
        e[c] = corr + L[c];
      }
    }
    st_once(out + i, e[0]);
    st_once(out + n + i, e[1]);
    st_once(out + 2 * n + i, e[2]);
    if (applied) applied[i] = both ? 1 : 0;
  }
}

// ------------------------------------------------------------------ progressive solver
// Sec. 2.2, Eq. 9: the new sample at x_i transports the current approximant
// at the next vertex once: Lbar = L_e + L~(x_{i+1}) * f G w / p.
__global__ void __launch_bounds__(256) k_step_samples(StepPtrs a, uint64_t n, KeyParams kp, TableView tv,
                                                      int32_t dtype, float* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float L[3];
  lookup_key(tv, dtype, query_key(kp, a.next, i), L);
  const bool le = a.le_r != nullptr;
  const float e[3] = {le ? ld_once(a.le_r + i) : 0.0f, le ? ld_once(a.le_g + i) : 0.0f,
                      le ? ld_once(a.le_b + i) : 0.0f};
  const float t[3] = {ld_once(a.t_r + i), ld_once(a.t_g + i), ld_once(a.t_b + i)};
#pragma unroll
  for (int c = 0; c < 3; ++c) out[(uint64_t)c * n + i] = e[c] + L[c] * t[c];
}

// ------------------------------------------------------------------ reset / init
__global__ void k_clear(TableView tv, uint64_t nslots) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    Slot z;
    z.key = kEmpty;
    z.c_old = 0;
    z.pad = 0;
    z.L[0] = z.L[1] = z.L[2] = z.L[3] = 0;
    tv.slots[s] = z;
    tv.keys[s] = kEmpty;
    if (tv.acc) tv.acc[s] = Acc{0u, {0.0f, 0.0f, 0.0f}};
    if (tv.var) tv.var[s] = 0.0f;
    if (tv.acc_q) tv.acc_q[s] = 0.0;
  }
}

__global__ void k_reset_counters(TableView tv, uint64_t nslots) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x)
    tv.slots[s].c_old = 0;
}

// Box of a key's cell along one axis meets [lo, hi]: the cell is
// [i s, (i + 1) s) with i the signed 16-bit coordinate at bit `shift`.
__device__ __forceinline__ bool cell_meets(uint64_t key, int32_t shift, float s, float lo, float hi) {
  const int32_t i = (int32_t)(int16_t)(uint16_t)((key >> shift) & 0xffffu);
  const float a = (float)i * s, b = (float)(i + 1) * s;
  return b > lo && a <= hi;
}

struct Box3 {
  float lo[3], hi[3];
};

__global__ void k_reset_region(TableView tv, uint64_t nslots, int32_t e_min, Box3 box) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = tv.keys[s];
    if (key == kEmpty) continue;
    const int32_t lvl = (int32_t)((key >> 59) & 15u);
    const float w = ldexpf(1.0f, e_min + lvl);
    if (cell_meets(key, 0, w, box.lo[0], box.hi[0]) && cell_meets(key, 16, w, box.lo[1], box.hi[1]) &&
        cell_meets(key, 32, w, box.lo[2], box.hi[2]))
      tv.slots[s].c_old = 0;
  }
}

__global__ void k_zero_words(uint32_t* p, uint64_t words) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ------------------------------------------------------------------ export support
__global__ void __launch_bounds__(256) k_count_occupied(TableView tv, uint64_t nslots,
                                                        unsigned long long* out) {
  __shared__ uint32_t s_c;
  if (threadIdx.x == 0) s_c = 0;
  __syncthreads();
  uint32_t c = 0;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x)
    c += tv.keys[s] != kEmpty;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane_id() == 0 && c) atomicAdd(&s_c, c);
  __syncthreads();
  if (threadIdx.x == 0 && s_c) atomicAdd(out, (unsigned long long)s_c);
}

__global__ void k_compact(TableView tv, uint64_t nslots, int32_t dtype, unsigned long long* cursor,
                          uint64_t cap, unsigned long long* keys, uint32_t* n_new, uint32_t* c_old,
                          float* rgb) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    const Slot sl = tv.slots[s];
    if (sl.key == kEmpty) continue;
    const unsigned long long at = atomicAdd(cursor, 1ull);
    if (at >= cap) continue;
    keys[at] = sl.key;
    n_new[at] = tv.acc ? tv.acc[s].n : 0u;
    c_old[at] = sl.c_old;
    float r, g, b;
    load_state(sl, dtype, r, g, b);
    rgb[at] = r;
    rgb[cap + at] = g;
    rgb[2 * cap + at] = b;
  }
}

// ------------------------------------------------------------------ SH payload (Sec. 2.6)
// Luminance as two real SH bands over the normal, chroma (Co, Cg) as means;
// per frame a ridge least-squares fit in binary64 (the reading is stated in
// psf.h at PSF_PAYLOAD_SH2_YCOCG).
__device__ __forceinline__ void sh_basis(double x, double y, double z, double b[4]) {
  const double k0 = 0.28209479177387814, k1 = 0.4886025119029199;
  b[0] = k0;
  b[1] = k1 * y;
  b[2] = k1 * z;
  b[3] = k1 * x;
}

// upper-triangle index of entry (i, j) of a symmetric 4 x 4 matrix
__device__ __forceinline__ int sh_tri(int i, int j) {
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  return lo == 0 ? hi : (lo == 1 ? 3 + hi : (lo == 2 ? 5 + hi : 9));
}

// (G + lambda diag(0, 1, 1, 1)) c = r, Cholesky in binary64
__device__ __forceinline__ void sh_solve(const double g[10], const double r[4], double lambda, double c[4]) {
  double a[4][4], l[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[i][j] = g[sh_tri(i, j)] + ((i == j && i > 0) ? lambda : 0.0);
      l[i][j] = 0.0;
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double d = a[j][j];
    for (int k = 0; k < j; ++k) d -= l[j][k] * l[j][k];
    l[j][j] = sqrt(d);
    for (int i = j + 1; i < 4; ++i) {
      double v = a[i][j];
      for (int k = 0; k < j; ++k) v -= l[i][k] * l[j][k];
      l[i][j] = v / l[j][j];
    }
  }
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = r[i];
    for (int k = 0; k < i; ++k) v -= l[i][k] * y[k];
    y[i] = v / l[i][i];
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 4; ++k) v -= l[k][i] * c[k];
    c[i] = v / l[i][i];
  }
}

// One record per thread: key, find or claim the slot, binary64 atomics on
// the cell's frame sums (weight, Gram matrix, basis-weighted luminance,
// chroma).
__global__ void __launch_bounds__(256) k_insert_sh(RecPtrs rec, uint64_t n, KeyParams kp, TableView tv) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = false, ovf = false;
  uint64_t key = kEmpty;
  float r = 0.0f, g = 0.0f, b = 0.0f, w = 1.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
  if (i < n) {
    const bool hr = rec.rough != nullptr;
    const float ro = hr ? rec.rough[i] : 0.0f;
    const bool gl = hr && ro < kp.rough_thr;
    const bool hf = rec.footprint != nullptr;
    nx = rec.nx[i];
    ny = rec.ny[i];
    nz = rec.nz[i];
    r = rec.r[i];
    g = rec.g[i];
    b = rec.b[i];
    valid = cell_key(kp, rec.px[i], rec.py[i], rec.pz[i], nx, ny, nz, gl ? rec.ox[i] : 0.0f,
                     gl ? rec.oy[i] : 0.0f, gl ? rec.oz[i] : 0.0f, hr, ro, hf, hf ? rec.footprint[i] : 0.0f, key,
                     ovf);
    valid = valid && finite3(r, g, b);
    if (rec.weight) {
      w = rec.weight[i];
      valid = valid && __builtin_isfinite(w) && w > 0.0f;
    }
  }
  wave_count(stat_lane(tv.stats->skipped, blockIdx.x), i < n && !valid);
  wave_count(stat_lane(tv.stats->coord_overflow, blockIdx.x), valid && ovf);
  if (!valid) return;
  uint32_t probes;
  const uint64_t slot = find_or_claim(tv, key, &probes);
  if (slot == ~0ull) {
    atomicAdd(&tv.stats->dropped, 1ull);
    return;
  }
  ShAcc* a = &tv.sh_acc[slot];
  const double wd = w;
  const double y = 0.25 * (double)r + 0.5 * (double)g + 0.25 * (double)b;
  const double co = 0.5 * (double)r - 0.5 * (double)b;
  const double cg = -0.25 * (double)r + 0.5 * (double)g - 0.25 * (double)b;
  double bs[4];
  sh_basis(nx, ny, nz, bs);
  atomicAdd(&a->n, wd);
#pragma unroll
  for (int p = 0; p < 4; ++p) {
#pragma unroll
    for (int q = p; q < 4; ++q) atomicAdd(&a->g[sh_tri(p, q)], wd * bs[p] * bs[q]);
    atomicAdd(&a->r[p], wd * y * bs[p]);
  }
  atomicAdd(&a->co, wd * co);
  atomicAdd(&a->cg, wd * cg);
}

// Streaming pass: every cell with frame sums gets its fit blended in
// (Eq. 10-11 on the counters, FP32 blend of the six numbers) and its sums
// cleared; per-block touch counts as in the RGB update.
__global__ void __launch_bounds__(256) k_update_sh(TableView tv, BlendParams bp, uint64_t nslots) {
  __shared__ uint32_t s_touched;
  if (threadIdx.x == 0) s_touched = 0;
  __syncthreads();
  const bool wtd = weighted(tv);
  uint32_t touched = 0;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    ShAcc a = tv.sh_acc[s];
    if (a.n == 0.0) continue;
    double fit[4];
    sh_solve(a.g, a.r, 1e-7 * a.n, fit);
    const uint32_t c_old = tv.slots[s].c_old;
    const uint32_t nw = wtd ? __float_as_uint((float)a.n) : (uint32_t)a.n;
    const float alpha = blend_alpha(bp, nw, c_old, wtd);
    ShState st = tv.sh[s];
    const float v[6] = {(float)fit[0], (float)fit[1], (float)fit[2], (float)fit[3], (float)(a.co / a.n),
                        (float)(a.cg / a.n)};
    float* sv[6] = {&st.c[0], &st.c[1], &st.c[2], &st.c[3], &st.co, &st.cg};
#pragma unroll
    for (int k = 0; k < 6; ++k) *sv[k] = alpha == 1.0f ? v[k] : (1.0f - alpha) * *sv[k] + alpha * v[k];
    tv.sh[s] = st;
    tv.slots[s].c_old = counter_add(c_old, nw, wtd);
    tv.sh_acc[s] = ShAcc{};
    ++touched;
  }
  for (int off = 32; off > 0; off >>= 1) touched += __shfl_xor(touched, off);
  if (lane_id() == 0 && touched) atomicAdd(&s_touched, touched);
  __syncthreads();
  if (threadIdx.x == 0) {
    BlockTouch* bt = &tv.touch[blockIdx.x];
    bt->last = s_touched;
    bt->total += s_touched;
  }
}

// Lookup: the luminance at the query's normal and the chroma, as RGB.
__global__ void __launch_bounds__(256) k_query_sh(QryPtrs q, uint64_t n, KeyParams kp, TableView tv, float* out,
                                                  uint8_t* found) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = query_key(kp, q, i);
  float rgb[3] = {0.0f, 0.0f, 0.0f};
  uint8_t hit = 0;
  if (key != kEmpty) {
    const uint64_t s = find_slot(tv, key);
    if (s != ~0ull && tv.slots[s].c_old != 0) {
      const ShState st = tv.sh[s];
      const float k0 = 0.28209479177387814f, k1 = 0.4886025119029199f;
      const float y = ((st.c[0] * k0 + st.c[1] * (k1 * q.ny[i])) + st.c[2] * (k1 * q.nz[i])) +
                      st.c[3] * (k1 * q.nx[i]);
      rgb[0] = (y + st.co) - st.cg;
      rgb[1] = y + st.cg;
      rgb[2] = (y - st.co) - st.cg;
      hit = 1;
    }
  }
  out[i] = rgb[0];
  out[n + i] = rgb[1];
  out[2 * n + i] = rgb[2];
  if (found) found[i] = hit;
}

__global__ void k_compact_sh(TableView tv, uint64_t nslots, unsigned long long* cursor, uint64_t cap,
                             unsigned long long* keys, uint32_t* c_old, float* coeff) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    const Slot sl = tv.slots[s];
    if (sl.key == kEmpty) continue;
    const unsigned long long at = atomicAdd(cursor, 1ull);
    if (at >= cap) continue;
    keys[at] = sl.key;
    c_old[at] = sl.c_old;
    const ShState st = tv.sh[s];
    const float v[6] = {st.c[0], st.c[1], st.c[2], st.c[3], st.co, st.cg};
    for (int k = 0; k < 6; ++k) coeff[(uint64_t)k * cap + at] = v[k];
  }
}

__global__ void k_compact_var(TableView tv, uint64_t nslots, unsigned long long* cursor, uint64_t cap,
                              unsigned long long* keys, float* var) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = tv.slots[s].key;
    if (k == kEmpty) continue;
    const unsigned long long at = atomicAdd(cursor, 1ull);
    if (at >= cap) continue;
    keys[at] = k;
    var[at] = tv.var[s];
  }
}

__global__ void k_clear_sh(TableView tv, uint64_t nslots) {
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    tv.sh[s] = ShState{};
    tv.sh_acc[s] = ShAcc{};
  }
}

// ------------------------------------------------------------------ launchers
static inline unsigned grid_for(uint64_t n, unsigned block) {
  uint64_t g = (n + block - 1) / block;
  return (unsigned)(g == 0 ? 1 : g);
}

static inline unsigned stride_grid(uint64_t n, unsigned block, unsigned cap) {
  uint64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  return (unsigned)(g == 0 ? 1 : g);
}

hipError_t launch_keys(const RecPtrs& rec, uint64_t n, const KeyParams& kp, unsigned long long* out,
                       hipStream_t s) {
  k_keys<<<grid_for(n, 256), 256, 0, s>>>(rec, n, kp, out);
  return hipGetLastError();
}

hipError_t launch_insert_direct(const RecPtrs& rec, uint64_t n, const KeyParams& kp,
                                const TableView& tv, hipStream_t s) {
  k_insert_direct<<<grid_for(n, kInsBlock), kInsBlock, 0, s>>>(rec, n, kp, tv);
  return hipGetLastError();
}

uint32_t update_grid(uint64_t nslots) { return stride_grid(nslots, 256, 2048); }

hipError_t launch_update(const TableView& tv, const BlendParams& bp, uint64_t nslots, hipStream_t s) {
  k_update<<<update_grid(nslots), 256, 0, s>>>(tv, bp, nslots);
  return hipGetLastError();
}

hipError_t launch_query(const QryPtrs& q, uint64_t n, const KeyParams& kp, const TableView& tv,
                        int32_t dtype, float* out, uint8_t* found, hipStream_t s) {
  k_query<<<grid_for(n, 256), 256, 0, s>>>(q, n, kp, tv, dtype, out, found);
  return hipGetLastError();
}

hipError_t launch_estimate(const EstPtrs& a, uint64_t n, const KeyParams& kp_o, const TableView& tv_o,
                           int32_t dt_o, const KeyParams& kp_i, const TableView& tv_i, int32_t dt_i,
                           int32_t mode, float param, float* out, uint8_t* applied, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_estimate<<<grid_for(n, kEstThreads * kEstPerThread), kEstThreads, 0, s>>>(a, n, kp_o, tv_o, dt_o, kp_i, tv_i,
                                                                             dt_i, mode, param, out, applied);
  return hipGetLastError();
}

hipError_t launch_step_samples(const StepPtrs& a, uint64_t n, const KeyParams& kp, const TableView& tv,
                               int32_t dtype, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_step_samples<<<grid_for(n, 256), 256, 0, s>>>(a, n, kp, tv, dtype, out);
  return hipGetLastError();
}

hipError_t launch_query_hier(const QryPtrs& q, uint64_t n, uint32_t up, const KeyParams& kp,
                             const TableView& tv, int32_t dtype, float* out, uint8_t* level_out,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_query_hier<<<grid_for(n, 256), 256, 0, s>>>(q, n, up, kp, tv, dtype, out, level_out);
  return hipGetLastError();
}

hipError_t launch_clear(const TableView& tv, uint64_t nslots, hipStream_t s) {
  k_clear<<<stride_grid(nslots, 256, 8192), 256, 0, s>>>(tv, nslots);
  return hipGetLastError();
}

hipError_t launch_reset_counters(const TableView& tv, uint64_t nslots, hipStream_t s) {
  k_reset_counters<<<stride_grid(nslots, 256, 8192), 256, 0, s>>>(tv, nslots);
  return hipGetLastError();
}

hipError_t launch_reset_region(const TableView& tv, uint64_t nslots, int32_t e_min, const float lo[3],
                               const float hi[3], hipStream_t s) {
  Box3 b;
  for (int c = 0; c < 3; ++c) {
    b.lo[c] = lo[c];
    b.hi[c] = hi[c];
  }
  k_reset_region<<<stride_grid(nslots, 256, 8192), 256, 0, s>>>(tv, nslots, e_min, b);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  k_zero_words<<<stride_grid(words, 256, 4096), 256, 0, s>>>(static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

hipError_t launch_count_occupied(const TableView& tv, uint64_t nslots, unsigned long long* out,
                                 hipStream_t s) {
  k_count_occupied<<<stride_grid(nslots, 256, 512), 256, 0, s>>>(tv, nslots, out);
  return hipGetLastError();
}

hipError_t launch_compact(const TableView& tv, uint64_t nslots, int32_t dtype,
                          unsigned long long* cursor, uint64_t cap, unsigned long long* keys,
                          uint32_t* n_new, uint32_t* c_old, float* rgb, hipStream_t s) {
  k_compact<<<stride_grid(nslots, 256, 4096), 256, 0, s>>>(tv, nslots, dtype, cursor, cap, keys,
                                                          n_new, c_old, rgb);
  return hipGetLastError();
}

hipError_t launch_insert_sh(const RecPtrs& rec, uint64_t n, const KeyParams& kp, const TableView& tv,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_insert_sh<<<grid_for(n, 256), 256, 0, s>>>(rec, n, kp, tv);
  return hipGetLastError();
}

hipError_t launch_update_sh(const TableView& tv, const BlendParams& bp, uint64_t nslots, hipStream_t s) {
  k_update_sh<<<update_grid(nslots), 256, 0, s>>>(tv, bp, nslots);
  return hipGetLastError();
}

hipError_t launch_query_sh(const QryPtrs& q, uint64_t n, const KeyParams& kp, const TableView& tv, float* out,
                           uint8_t* found, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_query_sh<<<grid_for(n, 256), 256, 0, s>>>(q, n, kp, tv, out, found);
  return hipGetLastError();
}

hipError_t launch_compact_sh(const TableView& tv, uint64_t nslots, unsigned long long* cursor, uint64_t cap,
                             unsigned long long* keys, uint32_t* c_old, float* coeff, hipStream_t s) {
  k_compact_sh<<<stride_grid(nslots, 256, 4096), 256, 0, s>>>(tv, nslots, cursor, cap, keys, c_old, coeff);
  return hipGetLastError();
}

hipError_t launch_compact_var(const TableView& tv, uint64_t nslots, unsigned long long* cursor, uint64_t cap,
                              unsigned long long* keys, float* var, hipStream_t s) {
  k_compact_var<<<stride_grid(nslots, 256, 4096), 256, 0, s>>>(tv, nslots, cursor, cap, keys, var);
  return hipGetLastError();
}

hipError_t launch_clear_sh(const TableView& tv, uint64_t nslots, hipStream_t s) {
  k_clear_sh<<<stride_grid(nslots, 256, 8192), 256, 0, s>>>(tv, nslots);
  return hipGetLastError();
}

}  // namespace psf

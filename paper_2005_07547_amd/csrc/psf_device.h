// Device-side definitions shared by the PSTF kernels: the cell key, the slot
// hash, the table layout and the 16-bit state encodings.
//
// Everything here runs on gfx950 only.  The translation units that include
// this header are compiled with -ffp-contract=off and correctly rounded FP32
// division, so the floating point that decides a key is plain IEEE binary32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psf {

constexpr uint64_t kEmpty = ~0ull;  // valid keys never set bit 63

// Parameters of the key function (spatio-directional hashing, Sec. 2.6 of the
// paper; the quantisation itself is this library's specification).
struct KeyParams {
  float cx, cy, cz;
  float kappa;
  int32_t e_min;
  int32_t max_level;
  int32_t nb_log2;
  int32_t db_log2;
  float rough_thr;
};

// One table slot, 32 bytes: everything a lookup needs sits in one sector.
struct alignas(32) Slot {
  unsigned long long key;  // kEmpty when free
  uint32_t c_old;          // cumulative counter (Sec. 2.4, c_h^old): a sample
                           // count, or in a weighted table the binary32 bits
                           // of a weight sum (0 bits = 0 either way)
  uint32_t pad;
  uint32_t L[4];           // approximant: 3 x f32, or 3 x 16-bit packed in L[0..1]
};

// Per-slot accumulator of the current frame (Eq. 5-6 numerator / counter;
// n holds binary32 bits of the weight sum in a weighted table).
struct alignas(16) Acc {
  uint32_t n;
  float s[3];
};

// Device-resident event counters (one atomic per wave or block when
// non-zero).  Rejected samples are not always rare (a field that leaves a
// sampling technique out rejects every sample of it), so the skip and
// overflow counts are spread over kStatLanes counters a cache line apart,
// picked by block index, and summed when the statistics are read: atomics
// on one address serialise.
constexpr uint32_t kStatLanes = 32;
struct alignas(256) DevStats {
  unsigned long long dropped;
  unsigned long long saturated;
  unsigned long long probe_hist[16];
  unsigned long long pad[14];
  unsigned long long skipped[kStatLanes][8];         // [lane][0] used
  unsigned long long coord_overflow[kStatLanes][8];  // [lane][0] used
};

__device__ __forceinline__ unsigned long long* stat_lane(unsigned long long (*c)[8], uint32_t block) {
  return &c[block % kStatLanes][0];
}

// Per-block count of blended cells, written by the block that owns the entry
// (no shared counters on the hot path).
struct alignas(16) BlockTouch {
  uint32_t last;
  uint32_t pad;
  unsigned long long total;
};
constexpr uint32_t kTouchEntries = 1u << 14;

// Two-band SH payload (Sec. 2.6): a cell's state, the four luminance
// coefficients and the chroma pair (24 bytes, padded to 32), and its frame
// sums in binary64: weight, Gram matrix of the basis over the sample
// normals (upper triangle), basis-weighted luminance, chroma sums.
struct alignas(16) ShState {
  float c[4];
  float co, cg;
  float pad[2];
};
struct alignas(16) ShAcc {
  double n;
  double g[10];
  double r[4];
  double co, cg;
  double pad;
};

// View of one table handed to kernels by value.
struct TableView {
  Slot* slots;
  unsigned long long* keys;  // mirror of slots[].key, read by the partitioned merge
  Acc* acc;
  ShState* sh;               // SH payload only (else null)
  ShAcc* sh_acc;
  DevStats* stats;
  BlockTouch* touch;         // kTouchEntries
  float* var;                // luminance variance per slot (PSF_FLAG_TRACK_VARIANCE, else null)
  double* acc_q;             // the frame's sum of squared luminances per slot (idem)
  uint32_t log2_slots;
  uint32_t part_log2;        // slots per partition = 2^part_log2 (<= log2_slots)
  uint32_t max_probe;
  uint32_t flags;            // public PSF_FLAG_* bits | kTvWeighted
};

// TableView::flags bit of a table with MIS-weighted (binary32) counters.
constexpr uint32_t kTvWeighted = 1u << 16;

__host__ __device__ __forceinline__ bool weighted(const TableView& tv) { return (tv.flags & kTvWeighted) != 0; }

// A counter word as a number: a count, or a weight sum's binary32 bits.
__device__ __forceinline__ float counter_value(uint32_t c, bool wtd) {
  return wtd ? __uint_as_float(c) : (float)c;
}

// c_old + n as a counter word.  In a weighted table both are binary32 weight
// sums and this addition rounds once; the frame's sum n is itself rounded
// once from binary64 by the partitioned merge, but accumulated with binary32
// atomics (in no fixed order) by the direct insert.
__device__ __forceinline__ uint32_t counter_add(uint32_t c, uint32_t n, bool wtd) {
  return wtd ? __float_as_uint(__uint_as_float(c) + __uint_as_float(n)) : c + n;
}

// Per-cell luminance variance (tables created with PSF_FLAG_TRACK_VARIANCE).
// A sample's luminance is Y of YCoCg, (r + 2 g + b) / 4, in binary64.
__device__ __forceinline__ double luma64(double r, double g, double b) { return ((r + 2.0 * g) + b) * 0.25; }

// The frame's luminance mean m and population variance s2 from its sums
// (channel sums s0..s2, squared-luminance sum q, n samples) in binary64.
__device__ __forceinline__ void frame_moments(double s0, double s1, double s2, double q, double n, double& m,
                                              double& var) {
  m = luma64(s0, s1, s2) / n;
  var = q / n - m * m;
  if (var < 0.0) var = 0.0;
}

// One blend of the variance (binary32): the two-component mixture of the
// cells' samples so far (weight 1 - alpha, variance V around mu, the
// luminance of the state the blend continues from) and the frame's (weight
// alpha, mean m, variance s2).
__device__ __forceinline__ float blend_variance(float V, float alpha, float mu, double m, double s2) {
  const float sf = (float)s2;
  if (alpha == 1.0f) return sf;
  const float d = (float)m - mu;
  return (1.0f - alpha) * V + alpha * (sf + (1.0f - alpha) * (d * d));
}

__device__ __forceinline__ float luma32(float r, float g, float b) { return ((r + 2.0f * g) + b) * 0.25f; }

struct BlendParams {
  int32_t mode;     // 0 Eq. 11, 1 constant alpha, 2 linear
  float alpha;
  float inv_t_max;
  int32_t dtype;    // 0 f32, 1 f16, 2 bf16
};

// ------------------------------------------------------------------ hashing
// 64-bit finaliser of MurmurHash3 (A. Appleby, public domain).
__device__ __forceinline__ uint64_t fmix64(uint64_t h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

// Probe sequence of a key: partition = top hash bits, start = low hash bits,
// linear probing wraps inside the partition.
struct ProbeSeq {
  uint64_t base;
  uint32_t start;
  uint32_t mask;
  __device__ __forceinline__ uint64_t at(uint32_t i) const { return base + ((start + i) & mask); }
};

__device__ __forceinline__ uint32_t partition_of(uint64_t h, uint32_t log2_slots, uint32_t part_log2) {
  uint32_t pbits = log2_slots - part_log2;
  return pbits == 0 ? 0u : (uint32_t)(h >> (64 - pbits));
}

__device__ __forceinline__ ProbeSeq probe_seq(uint64_t key, uint32_t log2_slots, uint32_t part_log2) {
  uint64_t h = fmix64(key);
  ProbeSeq p;
  p.mask = (1u << part_log2) - 1u;
  p.base = (uint64_t)partition_of(h, log2_slots, part_log2) << part_log2;
  p.start = (uint32_t)h & p.mask;
  return p;
}

// ------------------------------------------------------------------ key
#pragma clang fp contract(off)

__device__ __forceinline__ bool finite3(float a, float b, float c) {
  return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

// Level: floor(log2(kappa * d^2) / 2) clamped, read off the binary32 exponent.
__device__ __forceinline__ int32_t cell_level(const KeyParams& kp, float px, float py, float pz) {
  if (kp.kappa == 0.0f) return 0;
  const float dx = px - kp.cx, dy = py - kp.cy, dz = pz - kp.cz;
  const float d2 = (dx * dx + dy * dy) + dz * dz;
  const float q = d2 * kp.kappa;
  const int32_t biased = (int32_t)((__float_as_uint(q) >> 23) & 0xffu);
  const int32_t e = biased ? biased - 127 : -127;
  const int32_t lvl = e >> 1;  // arithmetic shift: floor(e / 2)
  return lvl < 0 ? 0 : (lvl > kp.max_level ? kp.max_level : lvl);
}

// Level from a path footprint (the world-space width a path covers at the
// vertex, the quantity the paper selects levels by in Sec. 2.3): the largest
// l with 2^(e_min + l) <= footprint, clamped to [0, max_level], read off the
// binary32 exponent (subnormals count as 2^-127).
__device__ __forceinline__ int32_t footprint_level(const KeyParams& kp, float fp) {
  const int32_t biased = (int32_t)((__float_as_uint(fp) >> 23) & 0xffu);
  const int32_t e = biased ? biased - 127 : -127;
  const int32_t lvl = e - kp.e_min;
  return lvl < 0 ? 0 : (lvl > kp.max_level ? kp.max_level : lvl);
}

// floor(p * 2^-shift) modulo 2^16, flagging values outside [-2^15, 2^15).
__device__ __forceinline__ uint32_t grid16(float p, int32_t shift, bool& ovf) {
  float f = floorf(ldexpf(p, -shift));
  ovf |= !(f >= -32768.0f && f < 32768.0f);
  f = fminf(fmaxf(f, -2147483648.0f), 2147483520.0f);
  return (uint32_t)(int32_t)f & 0xffffu;
}

// Octahedral map of a direction onto a B x B grid (B = 2^b): index iu*B + iw.
__device__ __forceinline__ uint32_t octa_bin(float x, float y, float z, int32_t b) {
  const float B = (float)(1 << b);
  const int32_t top = (1 << b) - 1;
  const float l1 = (fabsf(x) + fabsf(y)) + fabsf(z);
  float u = 0.0f, w = 0.0f;
  if (l1 > 0.0f) {
    u = x / l1;
    w = y / l1;
  }
  if (z < 0.0f) {
    const float fu = (1.0f - fabsf(w)) * (u >= 0.0f ? 1.0f : -1.0f);
    const float fw = (1.0f - fabsf(u)) * (w >= 0.0f ? 1.0f : -1.0f);
    u = fu;
    w = fw;
  }
  int32_t iu = (int32_t)floorf((u * 0.5f + 0.5f) * B);
  int32_t iw = (int32_t)floorf((w * 0.5f + 0.5f) * B);
  iu = iu < 0 ? 0 : (iu > top ? top : iu);
  iw = iw < 0 ? 0 : (iw > top ? top : iw);
  return (uint32_t)(iu * (1 << b) + iw);
}

// Cell key of one vertex.  Returns false for rejected (non-finite) input.
// has_rough is false when the caller supplied no roughness array (every
// vertex diffuse); the direction is read only for glossy vertices.  With a
// footprint (has_fp) the level comes from it (it must be finite and > 0),
// else from the camera distance.  up > 0 asks for the cell that many levels
// coarser (false if that passes max_level).
__device__ __forceinline__ bool cell_key(const KeyParams& kp, float px, float py, float pz, float nx,
                                         float ny, float nz, float ox, float oy, float oz,
                                         bool has_rough, float rough, bool has_fp, float fp,
                                         uint64_t& key, bool& ovf, int32_t up = 0) {
  if (!finite3(px, py, pz) || !finite3(nx, ny, nz)) return false;
  if (has_fp && !(__builtin_isfinite(fp) && fp > 0.0f)) return false;
  bool glossy = false;
  if (has_rough) {
    if (!__builtin_isfinite(rough)) return false;
    glossy = rough < kp.rough_thr;
    if (glossy && !finite3(ox, oy, oz)) return false;
  }
  const int32_t lvl = (has_fp ? footprint_level(kp, fp) : cell_level(kp, px, py, pz)) + up;
  if (lvl > kp.max_level) return false;
  const int32_t shift = kp.e_min + lvl;
  ovf = false;
  const uint64_t ix = grid16(px, shift, ovf);
  const uint64_t iy = grid16(py, shift, ovf);
  const uint64_t iz = grid16(pz, shift, ovf);
  const uint64_t nbin = octa_bin(nx, ny, nz, kp.nb_log2);
  const uint64_t dbin = glossy ? octa_bin(ox, oy, oz, kp.db_log2) : 0ull;
  key = ((uint64_t)lvl << 59) | ((uint64_t)glossy << 58) | (dbin << 52) | (nbin << 48) |
        (iz << 32) | (iy << 16) | ix;
  return true;
}

// ------------------------------------------------------------------ state encodings
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f, bool& sat) {
  (void)sat;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t f32_to_f16_rne(float f, bool& sat) {
  if (fabsf(f) > 65504.0f) {
    sat = true;
    f = f > 0.0f ? 65504.0f : -65504.0f;
  }
  _Float16 h = (_Float16)f;  // v_cvt_f16_f32, round to nearest even
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float f16_to_f32(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

// State formats: 0 binary32; 1 binary16 and 2 bfloat16, each re-rounded by
// every blend; 3 and 4 the same 16-bit values plus each channel's binary32
// rounding residual (value - stored 16-bit value, exact) kept in the slot's
// otherwise unused words, so that the blend continues from the unrounded
// binary32 state and a lookup sees a single rounding.
__device__ __forceinline__ bool state_is_f16(int32_t dtype) { return dtype == 1 || dtype == 3; }
__device__ __forceinline__ bool state_has_residual(int32_t dtype) { return dtype >= 3; }

// The approximant a lookup returns.
__device__ __forceinline__ void load_state(const Slot& s, int32_t dtype, float& r, float& g, float& b) {
  if (dtype == 0) {
    r = __uint_as_float(s.L[0]);
    g = __uint_as_float(s.L[1]);
    b = __uint_as_float(s.L[2]);
  } else if (state_is_f16(dtype)) {
    r = f16_to_f32(s.L[0] & 0xffffu);
    g = f16_to_f32(s.L[0] >> 16);
    b = f16_to_f32(s.L[1] & 0xffffu);
  } else {
    r = bf16_to_f32(s.L[0] & 0xffffu);
    g = bf16_to_f32(s.L[0] >> 16);
    b = bf16_to_f32(s.L[1] & 0xffffu);
  }
}

// The state the blend continues from: the lookup value, plus the carried
// residual in formats 3 and 4.
__device__ __forceinline__ void load_blend_state(const Slot& s, int32_t dtype, float& r, float& g, float& b) {
  load_state(s, dtype, r, g, b);
  if (state_has_residual(dtype)) {
    r = r + __uint_as_float(s.L[2]);
    g = g + __uint_as_float(s.L[3]);
    b = b + __uint_as_float(s.pad);
  }
}

// Encode a blended value: out[0..3] become Slot::L, *pad Slot::pad.
__device__ __forceinline__ void encode_state(int32_t dtype, float r, float g, float b, uint32_t out[4],
                                             uint32_t& pad, bool& sat) {
  pad = 0u;
  if (dtype == 0) {
    out[0] = __float_as_uint(r);
    out[1] = __float_as_uint(g);
    out[2] = __float_as_uint(b);
    out[3] = 0u;
    return;
  }
  const bool f16 = state_is_f16(dtype);
  const uint32_t hr = f16 ? f32_to_f16_rne(r, sat) : f32_to_bf16_rne(r, sat);
  const uint32_t hg = f16 ? f32_to_f16_rne(g, sat) : f32_to_bf16_rne(g, sat);
  const uint32_t hb = f16 ? f32_to_f16_rne(b, sat) : f32_to_bf16_rne(b, sat);
  out[0] = hr | (hg << 16);
  out[1] = hb;
  out[2] = 0u;
  out[3] = 0u;
  if (state_has_residual(dtype)) {
    // value - stored value: exact in binary32 (the two are within one
    // 16-bit ulp of each other), except past F16 saturation, where the
    // difference itself rounds
    const float sr = f16 ? f16_to_f32(hr) : bf16_to_f32(hr);
    const float sg = f16 ? f16_to_f32(hg) : bf16_to_f32(hg);
    const float sb = f16 ? f16_to_f32(hb) : bf16_to_f32(hb);
    out[2] = __float_as_uint(r - sr);
    out[3] = __float_as_uint(g - sg);
    pad = __float_as_uint(b - sb);
  }
}

// Lookup of one key (kEmpty = rejected record): the approximant if the cell
// exists and has been blended (c_old > 0), else zeros.  Returns the hit flag.
__device__ __forceinline__ uint8_t lookup_key(const TableView& tv, int32_t dtype, uint64_t key,
                                              float rgb[3]) {
  rgb[0] = rgb[1] = rgb[2] = 0.0f;
  if (key == kEmpty) return 0;
  const ProbeSeq ps = probe_seq(key, tv.log2_slots, tv.part_log2);
  for (uint32_t j = 0; j < tv.max_probe; ++j) {
    const Slot sl = tv.slots[ps.at(j)];
    if (sl.key == key) {
      if (sl.c_old == 0) return 0;
      load_state(sl, dtype, rgb[0], rgb[1], rgb[2]);
      return 1;
    }
    if (sl.key == kEmpty) return 0;
  }
  return 0;
}

// The same lookup split in two, so that the first probes of several
// lookups can be in flight together: lookup_first issues the load of the
// key's first slot (any key, also kEmpty: the slot is then ignored),
// lookup_finish resolves it and probes further only if needed.
struct PendingLookup {
  uint64_t key;
  ProbeSeq ps;
  Slot first;
};

__device__ __forceinline__ PendingLookup lookup_first(const TableView& tv, uint64_t key) {
  PendingLookup l;
  l.key = key;
  l.ps = probe_seq(key, tv.log2_slots, tv.part_log2);
  l.first = tv.slots[l.ps.at(0)];
  return l;
}

__device__ __forceinline__ uint8_t lookup_finish(const TableView& tv, int32_t dtype, const PendingLookup& l,
                                                 float rgb[3]) {
  rgb[0] = rgb[1] = rgb[2] = 0.0f;
  if (l.key == kEmpty) return 0;
  Slot sl = l.first;
  for (uint32_t j = 0;;) {
    if (sl.key == l.key) {
      if (sl.c_old == 0) return 0;
      load_state(sl, dtype, rgb[0], rgb[1], rgb[2]);
      return 1;
    }
    if (sl.key == kEmpty || ++j >= tv.max_probe) return 0;
    sl = tv.slots[l.ps.at(j)];
  }
}

// A value a pass reads once, and one it writes that no kernel of the pass
// reads: non-temporal, so streaming them does not evict from the caches the
// table the pass gathers from.
__device__ __forceinline__ float ld_once(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_once(float* p, float v) { __builtin_nontemporal_store(v, p); }

// Key of query i of a structure-of-arrays query set (kEmpty if rejected).
template <class Q>
__device__ __forceinline__ uint64_t query_key(const KeyParams& kp, const Q& q, uint64_t i, int32_t up = 0) {
  const bool hr = q.rough != nullptr;
  const float ro = hr ? ld_once(q.rough + i) : 0.0f;
  const bool gl = hr && ro < kp.rough_thr;
  const bool hf = q.footprint != nullptr;
  uint64_t key;
  bool ovf;
  if (!cell_key(kp, ld_once(q.px + i), ld_once(q.py + i), ld_once(q.pz + i), ld_once(q.nx + i),
                ld_once(q.ny + i), ld_once(q.nz + i), gl ? ld_once(q.ox + i) : 0.0f,
                gl ? ld_once(q.oy + i) : 0.0f, gl ? ld_once(q.oz + i) : 0.0f, hr, ro, hf,
                hf ? ld_once(q.footprint + i) : 0.0f, key, ovf, up))
    return kEmpty;
  return key;
}

// Eq. 10-11 for one cell, FP32, on counter words (counts, or weight sums
// in a weighted table).  n > 0.
__device__ __forceinline__ float blend_alpha(const BlendParams& bp, uint32_t n, uint32_t c_old, bool wtd) {
  if (bp.mode == 1) return c_old == 0 ? 1.0f : bp.alpha;
  const float nf = counter_value(n, wtd);
  const float ratio = nf / (counter_value(c_old, wtd) + nf);
  if (bp.mode == 2) return ratio;
  return fmaxf(sqrtf(ratio), bp.inv_t_max);
}

}  // namespace psf

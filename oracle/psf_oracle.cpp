// Reference oracle for progressive spatio-temporal filtering (PSTF).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded CPU
// statement of what the hash-filter hot path computes.  It exists so that the
// HIP library can be checked against it; nothing in the product links it.
// Only tests, the smoke entry point and the CPU-baseline leg of the benchmark
// may load it.  It shares no code with the HIP library.
//
// What it follows (Pantaleoni, "Online path sampling control with progressive
// spatio-temporal filtering", arXiv 2005.07547):
//   * Sec. 2.1, Eq. 5-6: per basis function h, a counter c_h (sum of box-basis
//     memberships times MIS weights) and the weighted sample mean of the path
//     tail estimates.  Box basis; weight w = 1 unless the records carry MIS
//     weights (Algorithm 1 sets the weight to 1 when no other technique is
//     used; Sec. 2.5 allows fields fed by only some techniques, whose weights
//     then do not sum to one).  A weight must be finite and > 0, else the
//     sample is skipped.
//   * Sec. 2.4, Eq. 10-11: temporal blend of the new mean into the previous
//     approximant with alpha = max(sqrt(c_new / (c_old + c_new)), 1/T_max);
//     c_old is the cumulative count up to the previous frame.  The same
//     section names the two limiting cases used as alternative modes: linear
//     accumulation (no square root) and exponential weighting (constant alpha).
//     Counters may be zeroed globally (reset).
//   * Sec. 2.6: the basis is a grid over position times a grid over direction,
//     i.e. a spatio-directional hash.  The paper leaves the exact quantisation
//     to Binder et al. and the level choice to a footprint heuristic; the key
//     function below is this project's fixed specification of both (positions
//     on power-of-two grids whose level grows with camera distance, octahedral
//     bins for the normal and, for glossy vertices, for the outgoing
//     direction).  Floating point that decides an integer is done in IEEE
//     binary32 exactly as specified (no contraction), so that any correct
//     implementation obtains the same bits.
//   * Algorithm 1: a lookup of the approximant at a vertex reads the state
//     left by the last completed temporal blend.
//   * Per-cell luminance variance (the paper defines none; this project's
//     reading): the spread of the cell's samples around the approximant,
//     under the same temporal weights.  With Y = (r + 2 g + b) / 4 (the
//     luminance of the YCoCg decomposition of Sec. 2.6), the blend of Eq.
//     10-11 makes the approximant's luminance the mixture mean of the
//     frames' sample distributions with weights beta_j (frame j's alpha
//     times (1 - alpha) of every later frame); the variance kept is that
//     mixture's variance, i.e. the population variance of every sample so
//     far, sample i of frame j weighted beta_j w_i / c_j.  One frame updates
//     it as a two-component mixture: V <- (1 - a) V + a s2 + a (1 - a)
//     (m - mu)^2 with m, s2 the frame's weighted mean and variance of Y and
//     mu the luminance of the approximant before the blend.
//
// Accumulation and blending are in binary64.  The table is a std::map with no
// capacity limit.  A key-sharded variant (orc_sharded_*, at the end) runs
// the same per-cell arithmetic on several host threads, one map per thread.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared (see build.py).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <thread>
#include <set>
#include <vector>

namespace {

struct Config {
  float cam[3];
  float kappa;        // level scale; 0 selects a fixed level 0
  int e_min;          // finest cell edge is 2^e_min
  int max_level;      // 0..15
  int normal_bins_log2;  // 0..2  (B = 1..4 bins per octahedral axis)
  int dir_bins_log2;     // 0..3  (B = 1..8)
  float rough_thr;    // glossy iff roughness < rough_thr (strict)
  int alpha_mode;     // 0 = Eq. 11, 1 = constant alpha, 2 = linear (no sqrt)
  float alpha;        // constant-mode alpha
  float t_max;        // Eq. 11 temporal window bound (> 0)
};

struct Cell {
  double n_new = 0.0;            // c_h^new of the current frame (sum of weights)
  double s[3] = {0.0, 0.0, 0.0}; // sum of the frame's weighted sample values
  double q = 0.0;                // sum of the frame's weighted squared luminances
  double c_old = 0.0;            // cumulative counter up to the previous frame
  double L[3] = {0.0, 0.0, 0.0}; // approximant
  double V = 0.0;                // luminance variance around the approximant
};

// Luminance of an RGB triple (Y of YCoCg).
double luma(double r, double g, double b) { return ((r + 2.0 * g) + b) * 0.25; }

struct Oracle {
  Config cfg;
  std::map<uint64_t, Cell> cells;
  bool filtered = false;
  std::set<uint64_t> filter;
  uint64_t skipped = 0;
  uint64_t coord_overflow = 0;
  uint64_t inserted = 0;
};

// --------------------------------------------------------------------------
// Key function K (project specification; Sec. 2.6 leaves it open).

bool finite3(float a, float b, float c) {
  return std::isfinite(a) && std::isfinite(b) && std::isfinite(c);
}

// Level from camera distance: floor(0.5 * log2(kappa * d^2)) clamped to
// [0, max_level], read from the binary32 exponent of kappa * d^2.
int level_of(const Config& c, float px, float py, float pz) {
  if (c.kappa == 0.0f) return 0;
  float dx = px - c.cam[0];
  float dy = py - c.cam[1];
  float dz = pz - c.cam[2];
  float xx = dx * dx;
  float yy = dy * dy;
  float zz = dz * dz;
  float d2 = xx + yy;
  d2 = d2 + zz;
  float q = d2 * c.kappa;
  uint32_t bits;
  std::memcpy(&bits, &q, sizeof bits);
  int field = (int)((bits >> 23) & 0xffu);
  int e = (field == 0) ? -127 : field - 127;
  // floor(e / 2) for negative e as well
  int lvl = (e >= 0) ? e / 2 : -((-e + 1) / 2);
  if (lvl < 0) lvl = 0;
  if (lvl > c.max_level) lvl = c.max_level;
  return lvl;
}

// Level from a path footprint (the width a path covers at the vertex; Sec.
// 2.3 selects hierarchy levels by footprint): the largest l with
// 2^(e_min + l) <= footprint, i.e. floor(log2(footprint)) - e_min, clamped
// to [0, max_level].  floor(log2) of a binary32 value is its exponent field
// (subnormals: taken as -127, far below any level).
int level_of_footprint(const Config& c, float fp) {
  uint32_t bits;
  std::memcpy(&bits, &fp, sizeof bits);
  int field = (int)((bits >> 23) & 0xffu);
  int e = (field == 0) ? -127 : field - 127;
  int lvl = e - c.e_min;
  if (lvl < 0) lvl = 0;
  if (lvl > c.max_level) lvl = c.max_level;
  return lvl;
}

// Grid coordinate floor(p * 2^-(e_min + lvl)); reports whether it lies
// outside the signed 16-bit range that the key stores.  The returned value is
// taken modulo 2^16 by the caller.
int64_t grid_coord(float p, int shift, bool* overflow) {
  float scaled = std::ldexp(p, -shift);
  float f = std::floor(scaled);
  if (!(f >= -32768.0f && f < 32768.0f)) *overflow = true;
  // clamp into a range that converts exactly, then convert
  if (f < -2147483648.0f) f = -2147483648.0f;
  if (f > 2147483520.0f) f = 2147483520.0f;
  return (int64_t)f;
}

// Octahedral bin index iu * B + iw of direction v with B = 2^b bins per axis.
uint32_t octa_bin(float vx, float vy, float vz, int b) {
  const int B = 1 << b;
  float ax = std::fabs(vx), ay = std::fabs(vy), az = std::fabs(vz);
  float a = ax + ay;
  a = a + az;
  float u = 0.0f, w = 0.0f;
  if (a > 0.0f) {
    u = vx / a;
    w = vy / a;
  }
  if (vz < 0.0f) {
    float su = (u >= 0.0f) ? 1.0f : -1.0f;
    float sw = (w >= 0.0f) ? 1.0f : -1.0f;
    float nu = (1.0f - std::fabs(w)) * su;
    float nw = (1.0f - std::fabs(u)) * sw;
    u = nu;
    w = nw;
  }
  float fu = u * 0.5f;
  fu = fu + 0.5f;
  fu = fu * (float)B;
  float fw = w * 0.5f;
  fw = fw + 0.5f;
  fw = fw * (float)B;
  int iu = (int)std::floor(fu);
  int iw = (int)std::floor(fw);
  if (iu > B - 1) iu = B - 1;
  if (iw > B - 1) iw = B - 1;
  if (iu < 0) iu = 0;
  if (iw < 0) iw = 0;
  return (uint32_t)(iu * B + iw);
}

struct KeyResult {
  bool valid;
  bool overflow;
  uint64_t key;
};

// rough may be null (all vertices diffuse); fp may be null (level from the
// camera distance), else it must be finite and positive.  up > 0 gives the
// key of the cell that many levels coarser (invalid past max_level).
KeyResult key_of(const Config& c, float px, float py, float pz, float nx, float ny, float nz,
                 float ox, float oy, float oz, const float* rough, const float* fp, int up = 0) {
  KeyResult r{false, false, 0};
  if (!finite3(px, py, pz) || !finite3(nx, ny, nz)) return r;
  if (fp && !(std::isfinite(*fp) && *fp > 0.0f)) return r;
  bool glossy = false;
  if (rough) {
    if (!std::isfinite(*rough)) return r;
    glossy = (*rough < c.rough_thr);
    if (glossy && !finite3(ox, oy, oz)) return r;
  }
  int lvl = (fp ? level_of_footprint(c, *fp) : level_of(c, px, py, pz)) + up;
  if (lvl > c.max_level) return r;
  int shift = c.e_min + lvl;
  bool ovf = false;
  int64_t ix = grid_coord(px, shift, &ovf);
  int64_t iy = grid_coord(py, shift, &ovf);
  int64_t iz = grid_coord(pz, shift, &ovf);
  uint64_t nb = octa_bin(nx, ny, nz, c.normal_bins_log2);
  uint64_t db = glossy ? octa_bin(ox, oy, oz, c.dir_bins_log2) : 0;
  uint64_t k = 0;
  k |= (uint64_t)lvl << 59;
  k |= (uint64_t)(glossy ? 1 : 0) << 58;
  k |= db << 52;
  k |= nb << 48;
  k |= ((uint64_t)ix & 0xffffu);
  k |= ((uint64_t)iy & 0xffffu) << 16;
  k |= ((uint64_t)iz & 0xffffu) << 32;
  r.valid = true;
  r.overflow = ovf;
  r.key = k;
  return r;
}

double alpha_of(const Config& c, double n, double o) {
  switch (c.alpha_mode) {
    case 1:  // constant alpha (exponential weighting); first touch takes the mean
      return o == 0.0 ? 1.0 : (double)c.alpha;
    case 2:  // linear accumulation
      return n / (o + n);
    default: {  // Eq. 11
      double a = std::sqrt(n / (o + n));
      double floor_a = 1.0 / (double)c.t_max;
      return a > floor_a ? a : floor_a;
    }
  }
}

}  // namespace

extern "C" {

// Record arrays: 15 pointers px,py,pz,nx,ny,nz,ox,oy,oz,r,g,b,rough,footprint,
// weight.  Any of ox..oz, r..b, rough, footprint and weight may be null where
// not used (rough null = diffuse, footprint null = level from the camera
// distance, weight null = every MIS weight 1).
struct orc_records {
  const float* f[15];
};

void* orc_create(const float* cam, float kappa, int e_min, int max_level, int normal_bins_log2,
                 int dir_bins_log2, float rough_thr, int alpha_mode, float alpha, float t_max) {
  Oracle* o = new Oracle();
  o->cfg.cam[0] = cam[0];
  o->cfg.cam[1] = cam[1];
  o->cfg.cam[2] = cam[2];
  o->cfg.kappa = kappa;
  o->cfg.e_min = e_min;
  o->cfg.max_level = max_level;
  o->cfg.normal_bins_log2 = normal_bins_log2;
  o->cfg.dir_bins_log2 = dir_bins_log2;
  o->cfg.rough_thr = rough_thr;
  o->cfg.alpha_mode = alpha_mode;
  o->cfg.alpha = alpha;
  o->cfg.t_max = t_max;
  return o;
}

void orc_destroy(void* h) { delete static_cast<Oracle*>(h); }

static KeyResult key_at(const Config& c, const orc_records* r, uint64_t i, int up = 0) {
  const float* const* f = r->f;
  float ox = f[6] ? f[6][i] : 0.0f, oy = f[7] ? f[7][i] : 0.0f, oz = f[8] ? f[8][i] : 0.0f;
  return key_of(c, f[0][i], f[1][i], f[2][i], f[3][i], f[4][i], f[5][i], ox, oy, oz,
                f[12] ? &f[12][i] : nullptr, f[13] ? &f[13][i] : nullptr, up);
}

// Keys of n records; invalid (skipped) records get all-ones.  overflow[i]
// (optional) receives 1 where a grid coordinate left the 16-bit range.
void orc_keys(void* h, const orc_records* r, uint64_t n, uint64_t* out, uint8_t* overflow) {
  Oracle* o = static_cast<Oracle*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    KeyResult k = key_at(o->cfg, r, i);
    out[i] = k.valid ? k.key : ~0ull;
    if (overflow) overflow[i] = k.overflow ? 1 : 0;
  }
}

// Restrict accumulation to a set of keys (sampled parity at large sizes).
// n = 0 removes the restriction.
void orc_set_filter(void* h, const uint64_t* keys, uint64_t n) {
  Oracle* o = static_cast<Oracle*>(h);
  o->filter.clear();
  o->filtered = n > 0;
  for (uint64_t i = 0; i < n; ++i) o->filter.insert(keys[i]);
}

// Eq. 5-6 with box basis: per cell, the counter (sum of the MIS weights w of
// its samples, 1 each without weights) and the sum of w times the sample
// value, in array order.
static void accumulate(Oracle* o, uint64_t key, float R, float G, float B, float w) {
  if (o->filtered && o->filter.count(key) == 0) return;
  Cell& c = o->cells[key];
  const double wd = (double)w;
  c.n_new += wd;
  c.s[0] += wd * (double)R;
  c.s[1] += wd * (double)G;
  c.s[2] += wd * (double)B;
  const double y = luma((double)R, (double)G, (double)B);
  c.q += wd * (y * y);
  o->inserted++;
}

void orc_insert(void* h, const orc_records* r, uint64_t n) {
  Oracle* o = static_cast<Oracle*>(h);
  const float* const* f = r->f;
  for (uint64_t i = 0; i < n; ++i) {
    float R = f[9][i], G = f[10][i], B = f[11][i];
    float w = f[14] ? f[14][i] : 1.0f;
    KeyResult k = key_at(o->cfg, r, i);
    if (!k.valid || !finite3(R, G, B) || !(std::isfinite(w) && w > 0.0f)) {
      o->skipped++;
      continue;
    }
    if (k.overflow) o->coord_overflow++;
    accumulate(o, k.key, R, G, B, w);
  }
}

// Eq. 10-11 for every cell touched since the last update.  Untouched cells
// keep their state.  Returns the number of cells blended.
uint64_t orc_update(void* h) {
  Oracle* o = static_cast<Oracle*>(h);
  uint64_t touched = 0;
  for (auto& kv : o->cells) {
    Cell& c = kv.second;
    if (c.n_new == 0.0) continue;
    double a = alpha_of(o->cfg, c.n_new, c.c_old);
    // the frame's weighted mean and variance of Y, the mixture update
    const double m = luma(c.s[0], c.s[1], c.s[2]) / c.n_new;
    double s2 = c.q / c.n_new - m * m;
    if (s2 < 0.0) s2 = 0.0;
    const double mu = luma(c.L[0], c.L[1], c.L[2]);
    c.V = (1.0 - a) * c.V + a * s2 + a * (1.0 - a) * (m - mu) * (m - mu);
    c.q = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      double mean = c.s[ch] / c.n_new;
      c.L[ch] = (1.0 - a) * c.L[ch] + a * mean;
      c.s[ch] = 0.0;
    }
    c.c_old += c.n_new;
    c.n_new = 0.0;
    touched++;
  }
  return touched;
}

// Lookup: the approximant of the query's cell if that cell has been blended
// at least once since its counters were last cleared; otherwise zero.
void orc_query(void* h, const orc_records* r, uint64_t n, double* out_rgb, uint8_t* found) {
  Oracle* o = static_cast<Oracle*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    KeyResult k = key_at(o->cfg, r, i);
    double v[3] = {0.0, 0.0, 0.0};
    uint8_t hit = 0;
    if (k.valid) {
      auto it = o->cells.find(k.key);
      if (it != o->cells.end() && it->second.c_old > 0.0) {
        hit = 1;
        for (int ch = 0; ch < 3; ++ch) v[ch] = it->second.L[ch];
      }
    }
    out_rgb[i] = v[0];
    out_rgb[n + i] = v[1];
    out_rgb[2 * n + i] = v[2];
    if (found) found[i] = hit;
  }
}

// what bit 0: zero c_old of every cell (global counter reset, Sec. 2.4);
// bit 1: remove every cell.
// Multi-level lookup (Sec. 2.3, a hierarchy of levels): the vertex's own
// cell if blended, else the finest blended cell up to `up` levels coarser.
// level[i] = 0 if none answered, else 1 + levels above the vertex's own.
void orc_query_levels(void* h, const orc_records* r, uint64_t n, int up, double* out_rgb, uint8_t* level) {
  Oracle* o = static_cast<Oracle*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    double v[3] = {0.0, 0.0, 0.0};
    uint8_t lv = 0;
    for (int k = 0; k <= up; ++k) {
      KeyResult kr = key_at(o->cfg, r, i, k);
      if (!kr.valid) break;
      auto it = o->cells.find(kr.key);
      if (it != o->cells.end() && it->second.c_old > 0.0) {
        for (int ch = 0; ch < 3; ++ch) v[ch] = it->second.L[ch];
        lv = (uint8_t)(k + 1);
        break;
      }
    }
    out_rgb[i] = v[0];
    out_rgb[n + i] = v[1];
    out_rgb[2 * n + i] = v[2];
    if (level) level[i] = lv;
  }
}

void orc_reset(void* h, uint32_t what) {
  Oracle* o = static_cast<Oracle*>(h);
  if (what & 2u) {
    o->cells.clear();
    return;
  }
  if (what & 1u)
    for (auto& kv : o->cells) kv.second.c_old = 0.0;
}

// Local counter reset (Sec. 2.4: counters zeroed locally, on demand): every
// cell whose box meets the closed box [lo, hi] gets c_old = 0.  A cell of
// level l covers [i s, (i + 1) s) per axis, s = 2^(e_min + l), with i its
// grid coordinate as stored in the key (signed 16-bit); binary32 as the key.
static bool cell_meets_axis(uint64_t key, int shift, float s, float lo, float hi) {
  int32_t i = (int32_t)(int16_t)(uint16_t)((key >> shift) & 0xffffu);
  float a = (float)i * s;
  float b = (float)(i + 1) * s;
  return b > lo && a <= hi;
}

void orc_reset_region(void* h, const float* lo, const float* hi) {
  Oracle* o = static_cast<Oracle*>(h);
  for (auto& kv : o->cells) {
    uint64_t key = kv.first;
    int lvl = (int)((key >> 59) & 15u);
    float s = std::ldexp(1.0f, o->cfg.e_min + lvl);
    if (cell_meets_axis(key, 0, s, lo[0], hi[0]) && cell_meets_axis(key, 16, s, lo[1], hi[1]) &&
        cell_meets_axis(key, 32, s, lo[2], hi[2]))
      kv.second.c_old = 0.0;
  }
}

uint64_t orc_count(void* h) { return static_cast<Oracle*>(h)->cells.size(); }

// Cells in ascending key order.  L and s are 3 x cap (SoA); the counters
// are sums of weights (integers without weights).  Returns the number
// written.
uint64_t orc_export(void* h, uint64_t* keys, double* n_new, double* c_old, double* L,
                    double* s, uint64_t cap) {
  Oracle* o = static_cast<Oracle*>(h);
  uint64_t i = 0;
  for (auto& kv : o->cells) {
    if (i >= cap) break;
    keys[i] = kv.first;
    if (n_new) n_new[i] = kv.second.n_new;
    if (c_old) c_old[i] = kv.second.c_old;
    for (int ch = 0; ch < 3; ++ch) {
      if (L) L[ch * cap + i] = kv.second.L[ch];
      if (s) s[ch * cap + i] = kv.second.s[ch];
    }
    ++i;
  }
  return i;
}

// Cells in ascending key order with their luminance variance.
uint64_t orc_export_variance(void* h, uint64_t* keys, double* var, uint64_t cap) {
  Oracle* o = static_cast<Oracle*>(h);
  uint64_t i = 0;
  for (auto& kv : o->cells) {
    if (i >= cap) break;
    keys[i] = kv.first;
    var[i] = kv.second.V;
    ++i;
  }
  return i;
}

void orc_counters(void* h, uint64_t* skipped, uint64_t* coord_overflow, uint64_t* inserted) {
  Oracle* o = static_cast<Oracle*>(h);
  *skipped = o->skipped;
  *coord_overflow = o->coord_overflow;
  *inserted = o->inserted;
}

}  // extern "C"

// --------------------------------------------------------------------------
// Key-sharded variant on several host threads (the CPU baseline's all-cores
// line; tests also use it to keep large sampled runs short).  T single-
// threaded oracles; cell key k belongs to shard owner(k) (a multiplicative
// hash of the key).  Cells are independent and each shard sees its cells'
// samples in array order, so every cell gets exactly the arithmetic, in the
// same order, as in the single oracle: the results are identical.
struct Sharded {
  std::vector<Oracle*> shard;
  std::vector<uint64_t> key;    // per record: key, or ~0 when rejected
  std::vector<uint8_t> ovf;
};

static uint32_t owner(uint64_t key, uint32_t t) {
  return (uint32_t)(((key * 0x9E3779B97F4A7C15ull) >> 32) % t);
}

template <class F>
static void parallel(uint32_t t, F&& f) {
  std::vector<std::thread> th;
  for (uint32_t i = 1; i < t; ++i) th.emplace_back(f, i);
  f(0u);
  for (auto& x : th) x.join();
}

extern "C" {

void* orc_sharded_create(uint32_t threads, const float* cam, float kappa, int e_min, int max_level,
                         int normal_bins_log2, int dir_bins_log2, float rough_thr, int alpha_mode, float alpha,
                         float t_max) {
  if (threads == 0) threads = 1;
  Sharded* s = new Sharded();
  for (uint32_t i = 0; i < threads; ++i)
    s->shard.push_back(static_cast<Oracle*>(orc_create(cam, kappa, e_min, max_level, normal_bins_log2,
                                                       dir_bins_log2, rough_thr, alpha_mode, alpha, t_max)));
  return s;
}

void orc_sharded_destroy(void* h) {
  Sharded* s = static_cast<Sharded*>(h);
  for (Oracle* o : s->shard) delete o;
  delete s;
}

void orc_sharded_set_filter(void* h, const uint64_t* keys, uint64_t n) {
  Sharded* s = static_cast<Sharded*>(h);
  const uint32_t t = (uint32_t)s->shard.size();
  for (uint32_t i = 0; i < t; ++i) {
    Oracle* o = s->shard[i];
    o->filter.clear();
    o->filtered = n > 0;
    for (uint64_t j = 0; j < n; ++j)
      if (owner(keys[j], t) == i) o->filter.insert(keys[j]);
  }
}

// As orc_insert: keys in parallel over record ranges, then every shard takes
// its own cells' samples in array order.  Skips and overflows are counted
// on shard 0.
void orc_sharded_insert(void* h, const orc_records* r, uint64_t n) {
  Sharded* s = static_cast<Sharded*>(h);
  const uint32_t t = (uint32_t)s->shard.size();
  s->key.assign(n, ~0ull);
  s->ovf.assign(n, 0);
  std::vector<uint64_t> skipped(t, 0), overflow(t, 0);
  const float* const* f = r->f;
  parallel(t, [&](uint32_t i) {
    const Config& c = s->shard[0]->cfg;
    const uint64_t lo = n * i / t, hi = n * (i + 1) / t;
    for (uint64_t j = lo; j < hi; ++j) {
      float R = f[9][j], G = f[10][j], B = f[11][j];
      float w = f[14] ? f[14][j] : 1.0f;
      KeyResult k = key_at(c, r, j);
      if (!k.valid || !finite3(R, G, B) || !(std::isfinite(w) && w > 0.0f)) {
        skipped[i]++;
        continue;
      }
      if (k.overflow) overflow[i]++;
      s->key[j] = k.key;
    }
  });
  parallel(t, [&](uint32_t i) {
    Oracle* o = s->shard[i];
    for (uint64_t j = 0; j < n; ++j) {
      const uint64_t k = s->key[j];
      if (k == ~0ull || owner(k, t) != i) continue;
      accumulate(o, k, f[9][j], f[10][j], f[11][j], f[14] ? f[14][j] : 1.0f);
    }
  });
  for (uint32_t i = 0; i < t; ++i) {
    s->shard[0]->skipped += skipped[i];
    s->shard[0]->coord_overflow += overflow[i];
  }
}

uint64_t orc_sharded_update(void* h) {
  Sharded* s = static_cast<Sharded*>(h);
  const uint32_t t = (uint32_t)s->shard.size();
  std::vector<uint64_t> touched(t, 0);
  parallel(t, [&](uint32_t i) { touched[i] = orc_update(s->shard[i]); });
  uint64_t sum = 0;
  for (uint64_t v : touched) sum += v;
  return sum;
}

// As orc_query, over record ranges in parallel (lookups only read).
void orc_sharded_query(void* h, const orc_records* r, uint64_t n, double* out_rgb, uint8_t* found) {
  Sharded* s = static_cast<Sharded*>(h);
  const uint32_t t = (uint32_t)s->shard.size();
  parallel(t, [&](uint32_t i) {
    const Config& c = s->shard[0]->cfg;
    const uint64_t lo = n * i / t, hi = n * (i + 1) / t;
    for (uint64_t j = lo; j < hi; ++j) {
      KeyResult k = key_at(c, r, j);
      double v[3] = {0.0, 0.0, 0.0};
      uint8_t hit = 0;
      if (k.valid) {
        const Oracle* o = s->shard[owner(k.key, t)];
        auto it = o->cells.find(k.key);
        if (it != o->cells.end() && it->second.c_old > 0.0) {
          hit = 1;
          for (int ch = 0; ch < 3; ++ch) v[ch] = it->second.L[ch];
        }
      }
      out_rgb[j] = v[0];
      out_rgb[n + j] = v[1];
      out_rgb[2 * n + j] = v[2];
      if (found) found[j] = hit;
    }
  });
}

uint64_t orc_sharded_count(void* h) {
  uint64_t c = 0;
  for (Oracle* o : static_cast<Sharded*>(h)->shard) c += o->cells.size();
  return c;
}

// As orc_export: every shard's cells, merged into ascending key order.
uint64_t orc_sharded_export(void* h, uint64_t* keys, double* n_new, double* c_old, double* L, double* s_out,
                            uint64_t cap) {
  Sharded* s = static_cast<Sharded*>(h);
  std::map<uint64_t, const Cell*> all;
  for (Oracle* o : s->shard)
    for (auto& kv : o->cells) all.emplace(kv.first, &kv.second);
  uint64_t i = 0;
  for (auto& kv : all) {
    if (i >= cap) break;
    const Cell& c = *kv.second;
    keys[i] = kv.first;
    if (n_new) n_new[i] = c.n_new;
    if (c_old) c_old[i] = c.c_old;
    for (int ch = 0; ch < 3; ++ch) {
      if (L) L[ch * cap + i] = c.L[ch];
      if (s_out) s_out[ch * cap + i] = c.s[ch];
    }
    ++i;
  }
  return i;
}

// As orc_export_variance over every shard.
uint64_t orc_sharded_export_variance(void* h, uint64_t* keys, double* var, uint64_t cap) {
  Sharded* s = static_cast<Sharded*>(h);
  std::map<uint64_t, double> all;
  for (Oracle* o : s->shard)
    for (auto& kv : o->cells) all.emplace(kv.first, kv.second.V);
  uint64_t i = 0;
  for (auto& kv : all) {
    if (i >= cap) break;
    keys[i] = kv.first;
    var[i] = kv.second;
    ++i;
  }
  return i;
}

void orc_sharded_counters(void* h, uint64_t* skipped, uint64_t* coord_overflow, uint64_t* inserted) {
  Sharded* s = static_cast<Sharded*>(h);
  *skipped = s->shard[0]->skipped;
  *coord_overflow = s->shard[0]->coord_overflow;
  uint64_t ins = 0;
  for (Oracle* o : s->shard) ins += o->inserted;
  *inserted = ins;
}

}  // extern "C"

// --------------------------------------------------------------------------
// Two-band spherical-harmonic luminance payload in YCoCg (Sec. 2.6: within a
// cell the luminance varies with the normal as two SH bands; chroma is one
// value per cell).  The paper gives no projection; this project's reading:
// each frame fits the four band-0/1 coefficients of the luminance to the
// cell's samples by weighted least squares over their normals, with a ridge
// of 1e-7 * (sum of weights) on the band-1 coefficients only (so the system
// is always positive definite, a constant field is reproduced exactly and a
// cell whose normals are all equal reproduces its mean there); the chroma
// pair is the frame's weighted mean.  The six numbers are blended like the
// approximant (Eq. 10-11 with the cell's counters).  A lookup evaluates the
// luminance at the query's normal and converts YCoCg back to RGB.

struct ShCell {
  double n_new = 0.0, g[10] = {}, r[4] = {}, co = 0.0, cg = 0.0;  // frame sums
  double c_old = 0.0, c[4] = {}, co_m = 0.0, cg_m = 0.0;          // state
};

struct ShOracle {
  Config cfg;
  std::map<uint64_t, ShCell> cells;
  uint64_t skipped = 0;
};

// Real SH basis of bands 0 and 1: 1 / (2 sqrt(pi)) and sqrt(3 / (4 pi)) (y, z, x).
static void sh_basis(double x, double y, double z, double b[4]) {
  const double k0 = 0.28209479177387814, k1 = 0.4886025119029199;
  b[0] = k0;
  b[1] = k1 * y;
  b[2] = k1 * z;
  b[3] = k1 * x;
}

// index of the upper-triangle entry (i <= j) of a symmetric 4 x 4 matrix
static int tri(int i, int j) {
  static const int idx[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
  return idx[i][j];
}

// (G + lambda D) c = r by Cholesky, D = diag(0, 1, 1, 1).
static void sh_solve(const double g[10], const double r[4], double lambda, double c[4]) {
  double a[4][4], l[4][4] = {};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) a[i][j] = g[tri(i, j)] + ((i == j && i > 0) ? lambda : 0.0);
  for (int j = 0; j < 4; ++j) {
    double d = a[j][j];
    for (int k = 0; k < j; ++k) d -= l[j][k] * l[j][k];
    l[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 4; ++i) {
      double v = a[i][j];
      for (int k = 0; k < j; ++k) v -= l[i][k] * l[j][k];
      l[i][j] = v / l[j][j];
    }
  }
  double y[4];
  for (int i = 0; i < 4; ++i) {
    double v = r[i];
    for (int k = 0; k < i; ++k) v -= l[i][k] * y[k];
    y[i] = v / l[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 4; ++k) v -= l[k][i] * c[k];
    c[i] = v / l[i][i];
  }
}

extern "C" {

void* orc_sh_create(const float* cam, float kappa, int e_min, int max_level, int normal_bins_log2,
                    int dir_bins_log2, float rough_thr, int alpha_mode, float alpha, float t_max) {
  ShOracle* o = new ShOracle();
  Oracle* tmp = static_cast<Oracle*>(orc_create(cam, kappa, e_min, max_level, normal_bins_log2, dir_bins_log2,
                                                rough_thr, alpha_mode, alpha, t_max));
  o->cfg = tmp->cfg;
  delete tmp;
  return o;
}

void orc_sh_destroy(void* h) { delete static_cast<ShOracle*>(h); }

// Per cell and frame: the weights, the Gram matrix of the basis over the
// samples' normals, the basis-weighted luminance and the chroma sums.
void orc_sh_insert(void* h, const orc_records* r, uint64_t n) {
  ShOracle* o = static_cast<ShOracle*>(h);
  const float* const* f = r->f;
  for (uint64_t i = 0; i < n; ++i) {
    const float R = f[9][i], G = f[10][i], B = f[11][i];
    const float w = f[14] ? f[14][i] : 1.0f;
    KeyResult k = key_at(o->cfg, r, i);
    if (!k.valid || !finite3(R, G, B) || !(std::isfinite(w) && w > 0.0f)) {
      o->skipped++;
      continue;
    }
    ShCell& c = o->cells[k.key];
    const double wd = w;
    const double y = 0.25 * R + 0.5 * G + 0.25 * B;
    const double co = 0.5 * R - 0.5 * B;
    const double cg = -0.25 * R + 0.5 * G - 0.25 * B;
    double b[4];
    sh_basis(f[3][i], f[4][i], f[5][i], b);
    c.n_new += wd;
    for (int a = 0; a < 4; ++a) {
      for (int e = a; e < 4; ++e) c.g[tri(a, e)] += wd * b[a] * b[e];
      c.r[a] += wd * y * b[a];
    }
    c.co += wd * co;
    c.cg += wd * cg;
  }
}

uint64_t orc_sh_update(void* h) {
  ShOracle* o = static_cast<ShOracle*>(h);
  uint64_t touched = 0;
  for (auto& kv : o->cells) {
    ShCell& c = kv.second;
    if (c.n_new == 0.0) continue;
    double fit[4];
    sh_solve(c.g, c.r, 1e-7 * c.n_new, fit);
    const double a = alpha_of(o->cfg, c.n_new, c.c_old);
    for (int k = 0; k < 4; ++k) c.c[k] = (1.0 - a) * c.c[k] + a * fit[k];
    c.co_m = (1.0 - a) * c.co_m + a * (c.co / c.n_new);
    c.cg_m = (1.0 - a) * c.cg_m + a * (c.cg / c.n_new);
    c.c_old += c.n_new;
    c.n_new = 0.0;
    for (double& v : c.g) v = 0.0;
    for (double& v : c.r) v = 0.0;
    c.co = c.cg = 0.0;
    touched++;
  }
  return touched;
}

void orc_sh_query(void* h, const orc_records* r, uint64_t n, double* out_rgb, uint8_t* found) {
  ShOracle* o = static_cast<ShOracle*>(h);
  const float* const* f = r->f;
  for (uint64_t i = 0; i < n; ++i) {
    KeyResult k = key_at(o->cfg, r, i);
    double v[3] = {0.0, 0.0, 0.0};
    uint8_t hit = 0;
    if (k.valid) {
      auto it = o->cells.find(k.key);
      if (it != o->cells.end() && it->second.c_old > 0.0) {
        const ShCell& c = it->second;
        double b[4];
        sh_basis(f[3][i], f[4][i], f[5][i], b);
        const double y = c.c[0] * b[0] + c.c[1] * b[1] + c.c[2] * b[2] + c.c[3] * b[3];
        v[0] = y + c.co_m - c.cg_m;
        v[1] = y + c.cg_m;
        v[2] = y - c.co_m - c.cg_m;
        hit = 1;
      }
    }
    out_rgb[i] = v[0];
    out_rgb[n + i] = v[1];
    out_rgb[2 * n + i] = v[2];
    if (found) found[i] = hit;
  }
}

uint64_t orc_sh_count(void* h) { return static_cast<ShOracle*>(h)->cells.size(); }

// Cells in ascending key order: keys, c_old, and the six state numbers as
// 6 x cap (SoA: c0..c3, Co, Cg).
uint64_t orc_sh_export(void* h, uint64_t* keys, double* c_old, double* coeff, uint64_t cap) {
  ShOracle* o = static_cast<ShOracle*>(h);
  uint64_t i = 0;
  for (auto& kv : o->cells) {
    if (i >= cap) break;
    keys[i] = kv.first;
    c_old[i] = kv.second.c_old;
    for (int k = 0; k < 4; ++k) coeff[k * cap + i] = kv.second.c[k];
    coeff[4 * cap + i] = kv.second.co_m;
    coeff[5 * cap + i] = kv.second.cg_m;
    ++i;
  }
  return i;
}

}  // extern "C"

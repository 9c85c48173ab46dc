// C-ABI layer of the PSTF hash library: argument validation, memory layout,
// strategy selection and kernel launches.  Nothing here throws across the
// ABI; every entry point returns a psf_status.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "psf.h"
#include "psf_internal.h"

#define PSF_API extern "C" __attribute__((visibility("default")))

// Ring of HIP-event pairs bracketing kernel launches (PSF_FLAG_TIMING).
struct KernelTimer {
  static constexpr uint32_t kCap = 4096;
  std::vector<hipEvent_t> ev;  // 2 per launch
  std::vector<uint8_t> kind;
  uint32_t next = 0, used = 0;
  uint64_t launches[PSF_K_COUNT] = {};
  double total_ms[PSF_K_COUNT] = {};

  hipError_t init() {
    ev.assign(2 * kCap, nullptr);
    kind.assign(kCap, 0);
    for (auto& e : ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
  void destroy() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    ev.clear();
  }
  hipError_t fold(uint32_t i) {
    hipError_t r = hipEventSynchronize(ev[2 * i + 1]);
    float ms = 0.0f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
    if (r != hipSuccess) return r;
    launches[kind[i]] += 1;
    total_ms[kind[i]] += ms;
    return hipSuccess;
  }
  hipError_t flush() {
    const uint32_t first = (next + kCap - used) % kCap;
    for (uint32_t j = 0; j < used; ++j) {
      hipError_t r = fold((first + j) % kCap);
      if (r != hipSuccess) return r;
    }
    used = 0;
    return hipSuccess;
  }
};

struct psf_table {
  psf_config cfg;
  KernelTimer* timer = nullptr;
  void* base = nullptr;
  size_t bytes = 0;
  bool owns = false;
  psf::TableView tv{};
  psf::KeyParams kp{};
  psf::BlendParams bp{};
  psf::PartView pv{};
  bool partitioned = false;  // strategy used by inserts
  uint64_t submitted = 0;
  uint64_t updates = 0;
  uint32_t touch_entries = 0;  // BlockTouch entries written by the last blend
  bool pending = false;      // accumulators hold samples not yet blended
  hipStream_t last = nullptr;
};

namespace {

thread_local std::string g_err;

psf_status fail(psf_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

psf_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return PSF_HIP_ERROR;
}

// Run one kernel launch, bracketed by events when the table records timing.
template <class F>
hipError_t timed(psf_table* t, int kind, hipStream_t s, F&& launch) {
  KernelTimer* tm = t->timer;
  if (!tm) return launch();
  const uint32_t i = tm->next;
  if (tm->used == KernelTimer::kCap) {
    hipError_t r = tm->fold(i);
    if (r != hipSuccess) return r;
    tm->used--;
  }
  hipError_t r = hipEventRecord(tm->ev[2 * i], s);
  if (r != hipSuccess) return r;
  r = launch();
  if (r != hipSuccess) return r;
  r = hipEventRecord(tm->ev[2 * i + 1], s);
  if (r != hipSuccess) return r;
  tm->kind[i] = (uint8_t)kind;
  tm->next = (i + 1) % KernelTimer::kCap;
  tm->used++;
  return hipSuccess;
}

constexpr uint32_t kDefaultPartLog2 = 11;
constexpr uint32_t kDefaultBinPer = 8;
constexpr uint64_t kDefaultBatch = 1ull << 22;
// Partitions of a partitioned table: at most 2^14 (beyond, the merge's
// fixed work per partition, its column of the run table over every tile,
// LDS set-up and barrier-separated phases, outweighs what it saves: 2^27
// slots took 1.45 ms partitioned against 1.20 ms direct on the plain
// workload, 2^26 slots 0.78 against 0.96 ms), and the default width is
// raised until there are at most 2^13 (the binning pass's LDS histogram
// then takes 32 KB).
constexpr uint32_t kMaxPartitions = 1u << 14;
constexpr uint32_t kDefaultPartitions = 1u << 13;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool validate(const psf_config* c, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return false;
  };
  if (!c) return bad("config is NULL");
  if (c->log2_slots < 4 || c->log2_slots > 30) return bad("log2_slots must be in [4, 30]");
  if (c->max_probe < 1 || (uint64_t)c->max_probe > (1ull << c->log2_slots))
    return bad("max_probe must be in [1, 2^log2_slots]");
  if (!std::isfinite(c->cam[0]) || !std::isfinite(c->cam[1]) || !std::isfinite(c->cam[2]))
    return bad("cam must be finite");
  if (!std::isfinite(c->kappa) || c->kappa < 0.0f) return bad("kappa must be finite and >= 0");
  if (c->e_min < -100 || c->e_min > 100) return bad("e_min must be in [-100, 100]");
  if (c->max_level < 0 || c->max_level > 15) return bad("max_level must be in [0, 15]");
  if (c->normal_bins_log2 < 0 || c->normal_bins_log2 > 2) return bad("normal_bins_log2 must be in [0, 2]");
  if (c->dir_bins_log2 < 0 || c->dir_bins_log2 > 3) return bad("dir_bins_log2 must be in [0, 3]");
  if (std::isnan(c->rough_thr)) return bad("rough_thr is NaN");
  if (c->alpha_mode < 0 || c->alpha_mode > 2) return bad("alpha_mode must be PAPER, CONST or LINEAR");
  if (c->alpha_mode == PSF_ALPHA_CONST && !(c->alpha > 0.0f && c->alpha <= 1.0f))
    return bad("alpha must be in (0, 1]");
  if (c->alpha_mode == PSF_ALPHA_PAPER && !(std::isfinite(c->t_max) && c->t_max >= 1.0f))
    return bad("t_max must be finite and >= 1");
  if (c->state_dtype < 0 || c->state_dtype > 4)
    return bad("state_dtype must be F32, F16, BF16, F16_EF or BF16_EF");
  if (c->insert_mode < 0 || c->insert_mode > 2) return bad("insert_mode must be AUTO, DIRECT or PARTITIONED");
  if (c->part_log2 != 0 && (c->part_log2 < 8 || c->part_log2 > 12)) return bad("part_log2 must be 0 or in [8, 12]");
  if (((c->flags & PSF_FLAG_TRACK_VARIANCE) || c->weighted) && c->part_log2 == 12)
    return bad("part_log2 must be at most 11 in a weighted table or one that keeps the variance");
  if (c->flags & ~(uint32_t)(PSF_FLAG_PROBE_STATS | PSF_FLAG_TIMING | PSF_FLAG_TRANSPOSE_RUNS |
                             PSF_FLAG_TRACK_VARIANCE | PSF_FLAG_NO_ACCUMULATORS))
    return bad("unknown flags");
  if ((c->flags & PSF_FLAG_NO_ACCUMULATORS) &&
      (c->payload != PSF_PAYLOAD_RGB || c->insert_mode == PSF_INSERT_DIRECT))
    return bad("a table without accumulators takes the RGB payload and the partitioned strategy");
  if (c->max_batch > (1ull << 31)) return bad("max_batch must be <= 2^31");
  if (c->bin_per != 0 && !psf::bin_per_ok(c->bin_per)) return bad("bin_per must be 0, 8, 12 or 16");
  if (c->payload > PSF_PAYLOAD_SH2_YCOCG) return bad("payload must be RGB or SH2_YCOCG");
  if (c->weighted > 1) return bad("weighted must be 0 or 1");
  return true;
}

struct Layout {
  size_t sh = 0, sh_acc = 0, var = 0, acc_q = 0;
  size_t stats = 0, touch = 0, slots = 0, keys = 0, acc = 0, stage_key = 0, stage_v = 0, stage_q = 0, runs = 0,
         runs_t = 0, perm = 0, total = 0;
  uint32_t part_log2 = 0;
  bool part = false;
  uint64_t cap = 0;
  uint32_t tiles = 0;
};

Layout layout_of(const psf_config& c) {
  Layout L;
  const uint64_t S = 1ull << c.log2_slots;
  // default partition width: 2^11 slots, wider for tables that would
  // otherwise exceed the binning pass's partition count
  // (with the further LDS sum of the variance or of the weights, 2^10 by
  // default, which keeps two blocks per CU, and at most 2^11: 2^12 slots of
  // 46 bytes exceed a workgroup's LDS)
  const bool extra = (c.flags & PSF_FLAG_TRACK_VARIANCE) || c.weighted;
  const uint32_t widest = extra ? 11u : 12u;
  uint32_t def = extra ? kDefaultPartLog2 - 1 : kDefaultPartLog2;
  while (def < widest && c.log2_slots > def && (1ull << (c.log2_slots - def)) > kDefaultPartitions) ++def;
  L.part_log2 = c.part_log2 ? c.part_log2 : def;
  if (L.part_log2 > c.log2_slots) L.part_log2 = c.log2_slots;
  const uint64_t P = 1ull << (c.log2_slots - L.part_log2);
  L.part = c.insert_mode != PSF_INSERT_DIRECT && P <= kMaxPartitions && c.payload == PSF_PAYLOAD_RGB;
  size_t off = 0;
  L.stats = off;
  off = align_up(off + sizeof(psf::DevStats), 256);
  L.touch = off;
  off = align_up(off + psf::kTouchEntries * sizeof(psf::BlockTouch), 256);
  L.slots = off;
  off = align_up(off + S * sizeof(psf::Slot), 256);
  L.keys = off;
  off = align_up(off + S * 8, 256);
  const bool no_acc = (c.flags & PSF_FLAG_NO_ACCUMULATORS) != 0;
  if (!no_acc) {
    L.acc = off;
    off = align_up(off + S * sizeof(psf::Acc), 256);
  }
  if (c.payload == PSF_PAYLOAD_SH2_YCOCG) {
    L.sh = off;
    off = align_up(off + S * sizeof(psf::ShState), 256);
    L.sh_acc = off;
    off = align_up(off + S * sizeof(psf::ShAcc), 256);
  }
  if (c.flags & PSF_FLAG_TRACK_VARIANCE) {
    L.var = off;
    off = align_up(off + S * 4, 256);
    if (!no_acc) {
      L.acc_q = off;
      off = align_up(off + S * 8, 256);
    }
  }
  if (L.part) {
    const uint64_t tile = psf::bin_tile(c.bin_per ? c.bin_per : kDefaultBinPer);
    L.cap = c.max_batch ? c.max_batch : kDefaultBatch;
    L.tiles = (uint32_t)((L.cap + tile - 1) / tile);
    L.cap = (uint64_t)L.tiles * tile;
    L.stage_key = off;
    off = align_up(off + L.cap * 8, 256);
    L.stage_v = off;
    off = align_up(off + L.cap * 16, 256);
    if (c.flags & PSF_FLAG_TRACK_VARIANCE) {
      L.stage_q = off;
      off = align_up(off + L.cap * 4, 256);
    }
    L.runs = off;
    off = align_up(off + (P + 1) * (uint64_t)L.tiles * 4, 256);
    L.runs_t = off;  // rows padded to a multiple of 4 tiles (16-byte loads)
    off = align_up(off + (P + 1) * (uint64_t)((L.tiles + 3) & ~3u) * 4, 256);
    L.perm = off;
    off = align_up(off + L.cap * 2, 256);
  }
  L.total = off;
  return L;
}

bool rec_ok(const psf_records* r, const psf_table* t, std::string* why) {
  if (!r) return (*why = "records is NULL", false);
  if (r->weight && !t->cfg.weighted) return (*why = "record weights need a table created with weighted = 1", false);
  if (!r->px || !r->py || !r->pz || !r->nx || !r->ny || !r->nz)
    return (*why = "position and normal arrays are required", false);
  if (!r->r || !r->g || !r->b) return (*why = "r, g, b arrays are required", false);
  if (r->rough && (!r->ox || !r->oy || !r->oz))
    return (*why = "direction arrays are required when roughness is given", false);
  return true;
}

bool qry_ok(const psf_queries* q, std::string* why) {
  if (!q) return (*why = "queries is NULL", false);
  if (!q->px || !q->py || !q->pz || !q->nx || !q->ny || !q->nz)
    return (*why = "position and normal arrays are required", false);
  if (q->rough && (!q->ox || !q->oy || !q->oz))
    return (*why = "direction arrays are required when roughness is given", false);
  return true;
}

psf::RecPtrs rec_ptrs(const psf_records* r) {
  return psf::RecPtrs{r->px, r->py, r->pz, r->nx, r->ny, r->nz, r->ox, r->oy, r->oz,
                      r->r,  r->g,  r->b,  r->rough, r->footprint, r->weight};
}

psf::QryPtrs qry_ptrs(const psf_queries* q) {
  return psf::QryPtrs{q->px, q->py, q->pz, q->nx, q->ny, q->nz, q->ox, q->oy, q->oz, q->rough, q->footprint};
}

psf::QryPtrs qry_from_rec(const psf_records* r) {
  return psf::QryPtrs{r->px, r->py, r->pz, r->nx, r->ny, r->nz, r->ox, r->oy, r->oz, r->rough, r->footprint};
}

uint64_t nslots(const psf_table* t) { return 1ull << t->cfg.log2_slots; }

psf::RecPtrs offset_rec(const psf::RecPtrs& rp, uint64_t off) {
  psf::RecPtrs sub = rp;
  const float** f[] = {&sub.px, &sub.py, &sub.pz, &sub.nx,    &sub.ny,       &sub.nz,    &sub.ox, &sub.oy,
                       &sub.oz, &sub.r,  &sub.g,  &sub.b,     &sub.rough,    &sub.footprint, &sub.weight};
  for (auto* p : f)
    if (*p) *p += off;
  return sub;
}

// Whether a partitioned launch of ntiles tiles transposes its run table.
bool transpose_runs(const psf_table* t, uint32_t ntiles) {
  return (t->cfg.flags & PSF_FLAG_TRANSPOSE_RUNS) ||
         psf::transpose_pays(ntiles, 1u << (t->cfg.log2_slots - t->tv.part_log2));
}

psf_status do_insert(psf_table* t, const psf::RecPtrs& rp, uint64_t n, hipStream_t s) {
  hipError_t e;
  if (t->tv.sh) {
    e = timed(t, PSF_K_INSERT_DIRECT, s, [&] { return psf::launch_insert_sh(rp, n, t->kp, t->tv, s); });
    if (e != hipSuccess) return hip_fail(e, "insert launch");
  } else if (t->partitioned) {
    for (uint64_t off = 0; off < n; off += t->pv.capacity) {
      const uint64_t m = (n - off < t->pv.capacity) ? n - off : t->pv.capacity;
      const psf::RecPtrs sub = offset_rec(rp, off);
      psf::PartView pv = t->pv;
      pv.perm = nullptr;
      pv.weights = sub.weight != nullptr;
      const uint32_t nt = (uint32_t)((m + pv.tile - 1) / pv.tile);
      if (!transpose_runs(t, nt)) pv.runs_t = nullptr;
      e = timed(t, PSF_K_BIN, s, [&] { return psf::launch_bin(sub, m, t->kp, t->tv, pv, s); });
      if (e == hipSuccess && pv.runs_t)
        e = timed(t, PSF_K_TRANSPOSE, s, [&] { return psf::launch_transpose_runs(t->tv, pv, nt, s); });
      if (e == hipSuccess)
        e = timed(t, PSF_K_MERGE, s, [&] { return psf::launch_merge(m, t->tv, pv, nullptr, false, s); });
      if (e != hipSuccess) return hip_fail(e, "partitioned insert launch");
    }
  } else {
    e = timed(t, PSF_K_INSERT_DIRECT, s,
              [&] { return psf::launch_insert_direct(rp, n, t->kp, t->tv, s); });
    if (e != hipSuccess) return hip_fail(e, "insert launch");
  }
  t->pending = true;
  t->submitted += n;
  return PSF_OK;
}

psf_status do_update(psf_table* t, hipStream_t s) {
  hipError_t e = timed(t, PSF_K_UPDATE, s, [&] {
    return t->tv.sh ? psf::launch_update_sh(t->tv, t->bp, nslots(t), s)
                    : psf::launch_update(t->tv, t->bp, nslots(t), s);
  });
  if (e != hipSuccess) return hip_fail(e, "update launch");
  t->pending = false;
  t->updates++;
  t->touch_entries = psf::update_grid(nslots(t));
  return PSF_OK;
}

bool same_vertices(const psf_records* r, const psf_queries* q) {
  return r->px == q->px && r->py == q->py && r->pz == q->pz && r->nx == q->nx && r->ny == q->ny &&
         r->nz == q->nz && r->rough == q->rough && r->footprint == q->footprint &&
         (!r->rough || (r->ox == q->ox && r->oy == q->oy && r->oz == q->oz));
}

psf_status do_query(psf_table* t, const psf::QryPtrs& q, uint64_t n, float* out, uint8_t* found,
                    hipStream_t s) {
  hipError_t e = timed(t, PSF_K_QUERY, s, [&] {
    return t->tv.sh ? psf::launch_query_sh(q, n, t->kp, t->tv, out, found, s)
                    : psf::launch_query(q, n, t->kp, t->tv, t->cfg.state_dtype, out, found, s);
  });
  return e == hipSuccess ? PSF_OK : hip_fail(e, "query launch");
}

}  // namespace

PSF_API size_t psf_table_bytes(const psf_config* cfg) {
  std::string why;
  if (!validate(cfg, &why)) {
    g_err = why;
    return 0;
  }
  const Layout L = layout_of(*cfg);
  if ((cfg->flags & PSF_FLAG_NO_ACCUMULATORS) && !L.part) {
    g_err = "a table without accumulators needs the partitioned strategy (too many partitions)";
    return 0;
  }
  return L.total;
}

PSF_API psf_status psf_create_table(const psf_config* cfg, void* device_buffer, size_t buffer_bytes,
                                    psf_stream stream, psf_table** out) {
  std::string why;
  if (!out) return fail(PSF_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!validate(cfg, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (cfg->payload == PSF_PAYLOAD_SH2_YCOCG &&
      (cfg->state_dtype != PSF_STATE_F32 || cfg->insert_mode == PSF_INSERT_PARTITIONED))
    return fail(PSF_NOT_SUPPORTED, "the SH payload takes F32 state and the direct insert strategy");
  if ((cfg->flags & PSF_FLAG_TRACK_VARIANCE) && (cfg->payload != PSF_PAYLOAD_RGB || cfg->weighted))
    return fail(PSF_NOT_SUPPORTED, "the luminance variance is kept for unweighted RGB tables only");
  const Layout L = layout_of(*cfg);
  if ((cfg->flags & PSF_FLAG_NO_ACCUMULATORS) && !L.part)
    return fail(PSF_NOT_SUPPORTED, "a table without accumulators needs the partitioned strategy (too many partitions)");
  if (device_buffer) {
    if (buffer_bytes < L.total)
      return fail(PSF_BUFFER_TOO_SMALL, "device buffer smaller than psf_table_bytes(cfg)");
    if (reinterpret_cast<uintptr_t>(device_buffer) % 256 != 0)
      return fail(PSF_INVALID_ARGUMENT, "device buffer must be 256-byte aligned");
  }
  psf_table* t = new (std::nothrow) psf_table();
  if (!t) return fail(PSF_OUT_OF_MEMORY, "host allocation failed");
  t->cfg = *cfg;
  t->bytes = L.total;
  if (device_buffer) {
    t->base = device_buffer;
  } else {
    hipError_t e = hipMalloc(&t->base, L.total);
    if (e != hipSuccess) {
      delete t;
      (void)hipGetLastError();
      return fail(PSF_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    t->owns = true;
  }
  char* b = static_cast<char*>(t->base);
  t->tv.stats = reinterpret_cast<psf::DevStats*>(b + L.stats);
  t->tv.touch = reinterpret_cast<psf::BlockTouch*>(b + L.touch);
  t->tv.slots = reinterpret_cast<psf::Slot*>(b + L.slots);
  t->tv.keys = reinterpret_cast<unsigned long long*>(b + L.keys);
  t->tv.acc = L.acc ? reinterpret_cast<psf::Acc*>(b + L.acc) : nullptr;
  t->tv.sh = L.sh ? reinterpret_cast<psf::ShState*>(b + L.sh) : nullptr;
  t->tv.sh_acc = L.sh_acc ? reinterpret_cast<psf::ShAcc*>(b + L.sh_acc) : nullptr;
  t->tv.var = L.var ? reinterpret_cast<float*>(b + L.var) : nullptr;
  t->tv.acc_q = L.acc_q ? reinterpret_cast<double*>(b + L.acc_q) : nullptr;
  t->tv.log2_slots = cfg->log2_slots;
  t->tv.part_log2 = L.part_log2;
  t->tv.max_probe = cfg->max_probe < (1u << L.part_log2) ? cfg->max_probe : (1u << L.part_log2);
  t->tv.flags = cfg->flags | (cfg->weighted ? psf::kTvWeighted : 0u);
  t->kp = psf::KeyParams{cfg->cam[0], cfg->cam[1], cfg->cam[2], cfg->kappa, cfg->e_min,
                         cfg->max_level, cfg->normal_bins_log2, cfg->dir_bins_log2, cfg->rough_thr};
  t->bp = psf::BlendParams{cfg->alpha_mode, cfg->alpha, 1.0f / cfg->t_max, cfg->state_dtype};
  if (cfg->alpha_mode != PSF_ALPHA_PAPER) t->bp.inv_t_max = 0.0f;
  if (L.part) {
    t->pv.stage_key = reinterpret_cast<unsigned long long*>(b + L.stage_key);
    t->pv.stage_v = reinterpret_cast<float4*>(b + L.stage_v);
    t->pv.stage_q = L.stage_q ? reinterpret_cast<float*>(b + L.stage_q) : nullptr;
    t->pv.weights = 0;
    t->pv.runs = reinterpret_cast<uint32_t*>(b + L.runs);
    t->pv.runs_t = reinterpret_cast<uint32_t*>(b + L.runs_t);
    t->pv.perm = reinterpret_cast<uint16_t*>(b + L.perm);
    t->pv.tile = psf::bin_tile(cfg->bin_per ? cfg->bin_per : kDefaultBinPer);
    t->pv.max_tiles = L.tiles;
    t->pv.capacity = L.cap;
    t->partitioned = true;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (cfg->flags & PSF_FLAG_TIMING) {
    t->timer = new (std::nothrow) KernelTimer();
    e = t->timer ? t->timer->init() : hipErrorOutOfMemory;
  }
  if (e == hipSuccess) e = psf::launch_zero(t->tv.stats, L.slots - L.stats, s);
  if (e == hipSuccess) e = psf::launch_clear(t->tv, nslots(t), s);
  if (e == hipSuccess && t->tv.sh) e = psf::launch_clear_sh(t->tv, nslots(t), s);
  if (e != hipSuccess) {
    if (t->timer) {
      t->timer->destroy();
      delete t->timer;
    }
    if (t->owns) (void)hipFree(t->base);
    delete t;
    return hip_fail(e, "table initialisation");
  }
  t->last = s;
  *out = t;
  return PSF_OK;
}

PSF_API psf_status psf_destroy(psf_table* t) {
  if (!t) return PSF_OK;
  // only memory the library frees needs the stream drained first (a pending
  // timing event is released by the runtime once it completes)
  hipError_t e = t->owns ? hipStreamSynchronize(t->last) : hipSuccess;
  hipError_t f = hipSuccess;
  if (t->owns) f = hipFree(t->base);
  if (t->timer) {
    t->timer->destroy();
    delete t->timer;
  }
  delete t;
  if (e != hipSuccess) return hip_fail(e, "synchronise before destroy");
  if (f != hipSuccess) return hip_fail(f, "hipFree");
  return PSF_OK;
}

PSF_API psf_status psf_insert_samples(psf_table* t, const psf_records* rec, uint64_t n,
                                      psf_stream stream) {
  std::string why;
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n == 0) return PSF_OK;
  if (!rec_ok(rec, t, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (!t->tv.acc) return fail(PSF_NOT_SUPPORTED, "separate inserts on a table without accumulators");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  return do_insert(t, rec_ptrs(rec), n, s);
}

PSF_API psf_status psf_temporal_update(psf_table* t, psf_stream stream) {
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (!t->tv.acc) return fail(PSF_NOT_SUPPORTED, "separate updates on a table without accumulators");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  return do_update(t, s);
}

PSF_API psf_status psf_query(psf_table* t, const psf_queries* q, uint64_t n, float* d_out_rgb,
                             uint8_t* d_out_found, psf_stream stream) {
  std::string why;
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n == 0) return PSF_OK;
  if (!qry_ok(q, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (!d_out_rgb) return fail(PSF_INVALID_ARGUMENT, "output array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  return do_query(t, qry_ptrs(q), n, d_out_rgb, d_out_found, s);
}

PSF_API psf_status psf_iterate(psf_table* t, const psf_records* rec, uint64_t n, const psf_queries* q,
                               uint64_t nq, float* d_out_rgb, uint8_t* d_out_found, psf_stream stream) {
  std::string why;
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n > 0 && !rec_ok(rec, t, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (nq > 0 && !qry_ok(q, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (nq > 0 && !d_out_rgb) return fail(PSF_INVALID_ARGUMENT, "output array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  psf_status st = PSF_OK;
  if (n > 0 && t->partitioned && !t->pending && n <= t->pv.capacity) {
    const psf::RecPtrs rp = rec_ptrs(rec);
    // when the queries are the records being inserted, the merge pass hands
    // every staged entry its cell's new value and the unstage pass returns
    // them in record order: no second lookup
    const bool fq = nq == n && same_vertices(rec, q);
    psf::PartView pv = t->pv;
    if (!fq) pv.perm = nullptr;
    pv.weights = rp.weight != nullptr;
    const uint32_t nt = (uint32_t)((n + pv.tile - 1) / pv.tile);
    if (!transpose_runs(t, nt)) pv.runs_t = nullptr;
    hipError_t e = timed(t, PSF_K_BIN, s, [&] { return psf::launch_bin(rp, n, t->kp, t->tv, pv, s); });
    if (e == hipSuccess && pv.runs_t)
      e = timed(t, PSF_K_TRANSPOSE, s, [&] { return psf::launch_transpose_runs(t->tv, pv, nt, s); });
    if (e == hipSuccess)
      e = timed(t, PSF_K_MERGE_BLEND, s, [&] { return psf::launch_merge(n, t->tv, pv, &t->bp, fq, s); });
    if (e != hipSuccess) return hip_fail(e, "fused insert launch");
    t->submitted += n;
    t->updates++;
    t->touch_entries = 1u << (t->cfg.log2_slots - t->tv.part_log2);
    if (fq) {
      e = timed(t, PSF_K_QUERY, s, [&] { return psf::launch_unstage(n, t->tv, pv, d_out_rgb, d_out_found, s); });
      return e == hipSuccess ? PSF_OK : hip_fail(e, "query launch");
    }
  } else if (!t->tv.acc) {
    // no accumulators: nothing to blend without records, and a launch past
    // the staging capacity would need the separate insert and update
    if (n > 0) return fail(PSF_NOT_SUPPORTED, "more records than max_batch on a table without accumulators");
    t->updates++;
    t->touch_entries = 0;
  } else {
    if (n > 0) st = do_insert(t, rec_ptrs(rec), n, s);
    if (st == PSF_OK) st = do_update(t, s);
  }
  if (st != PSF_OK || nq == 0) return st;
  return do_query(t, qry_ptrs(q), nq, d_out_rgb, d_out_found, s);
}

PSF_API psf_status psf_reset(psf_table* t, uint32_t what, psf_stream stream) {
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (what & ~(uint32_t)(PSF_RESET_COUNTERS | PSF_RESET_CLEAR | PSF_RESET_STATS))
    return fail(PSF_INVALID_ARGUMENT, "unknown reset bits");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  hipError_t e = hipSuccess;
  if (what & PSF_RESET_CLEAR) {
    e = psf::launch_clear(t->tv, nslots(t), s);
    if (e == hipSuccess && t->tv.sh) e = psf::launch_clear_sh(t->tv, nslots(t), s);
    t->pending = false;
  } else if (what & PSF_RESET_COUNTERS) {
    e = psf::launch_reset_counters(t->tv, nslots(t), s);
  }
  if (e == hipSuccess && (what & PSF_RESET_STATS)) {
    e = psf::launch_zero(t->tv.stats, reinterpret_cast<char*>(t->tv.slots) - reinterpret_cast<char*>(t->tv.stats), s);
    t->submitted = 0;
    t->updates = 0;
    t->touch_entries = 0;
  }
  return e == hipSuccess ? PSF_OK : hip_fail(e, "reset launch");
}

PSF_API psf_status psf_query_levels(psf_table* t, const psf_queries* q, uint64_t n, uint32_t levels_up,
                                    float* d_out_rgb, uint8_t* d_out_level, psf_stream stream) {
  std::string why;
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n == 0) return PSF_OK;
  if (!qry_ok(q, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (!d_out_rgb) return fail(PSF_INVALID_ARGUMENT, "output array is NULL");
  if (levels_up > 15) return fail(PSF_INVALID_ARGUMENT, "levels_up must be <= 15");
  if (t->tv.sh) return fail(PSF_NOT_SUPPORTED, "multi-level lookup of an SH payload table");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  hipError_t e = timed(t, PSF_K_QUERY, s, [&] {
    return psf::launch_query_hier(qry_ptrs(q), n, levels_up, t->kp, t->tv, t->cfg.state_dtype, d_out_rgb,
                                  d_out_level, s);
  });
  return e == hipSuccess ? PSF_OK : hip_fail(e, "query launch");
}

PSF_API psf_status psf_progressive_step(psf_table* t, const psf_records* x, const psf_queries* next,
                                        const psf_step_args* a, uint64_t n, float* d_samples,
                                        psf_stream stream) {
  std::string why;
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n == 0) return PSF_OK;
  if (!x || !x->px || !x->py || !x->pz || !x->nx || !x->ny || !x->nz)
    return fail(PSF_INVALID_ARGUMENT, "vertex position and normal arrays are required");
  if (x->rough && (!x->ox || !x->oy || !x->oz))
    return fail(PSF_INVALID_ARGUMENT, "direction arrays are required when roughness is given");
  if (x->weight && !t->cfg.weighted)
    return fail(PSF_INVALID_ARGUMENT, "record weights need a table created with weighted = 1");
  if (!qry_ok(next, &why)) return fail(PSF_INVALID_ARGUMENT, why);
  if (!a || !a->t_r || !a->t_g || !a->t_b) return fail(PSF_INVALID_ARGUMENT, "throughput arrays are required");
  if ((a->le_r != nullptr) != (a->le_g != nullptr) || (a->le_r != nullptr) != (a->le_b != nullptr))
    return fail(PSF_INVALID_ARGUMENT, "emission arrays: all three or none");
  if (!d_samples) return fail(PSF_INVALID_ARGUMENT, "sample array is NULL");
  if (t->tv.sh) return fail(PSF_NOT_SUPPORTED, "progressive step on an SH payload table");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  psf::StepPtrs sp{qry_ptrs(next), a->le_r, a->le_g, a->le_b, a->t_r, a->t_g, a->t_b};
  hipError_t e = timed(t, PSF_K_STEP, s, [&] {
    return psf::launch_step_samples(sp, n, t->kp, t->tv, t->cfg.state_dtype, d_samples, s);
  });
  if (e != hipSuccess) return hip_fail(e, "progressive step launch");
  psf_records r = *x;
  r.r = d_samples;
  r.g = d_samples + n;
  r.b = d_samples + 2 * n;
  return psf_iterate(t, &r, n, nullptr, 0, nullptr, nullptr, stream);
}

PSF_API psf_status psf_reset_region(psf_table* t, const float* lo, const float* hi, psf_stream stream) {
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (!lo || !hi) return fail(PSF_INVALID_ARGUMENT, "region corners are NULL");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(lo[c]) || !std::isfinite(hi[c]) || lo[c] > hi[c])
      return fail(PSF_INVALID_ARGUMENT, "region corners must be finite with lo <= hi");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  hipError_t e = psf::launch_reset_region(t->tv, nslots(t), t->cfg.e_min, lo, hi, s);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "reset launch");
}

PSF_API psf_status psf_compute_keys(psf_table* t, const psf_records* rec, uint64_t n,
                                    uint64_t* d_out_keys, psf_stream stream) {
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n == 0) return PSF_OK;
  if (!rec || !rec->px || !rec->py || !rec->pz || !rec->nx || !rec->ny || !rec->nz ||
      (rec->rough && (!rec->ox || !rec->oy || !rec->oz)))
    return fail(PSF_INVALID_ARGUMENT, "position, normal (and direction with roughness) arrays are required");
  if (!d_out_keys) return fail(PSF_INVALID_ARGUMENT, "output array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  hipError_t e = timed(t, PSF_K_KEYS, s, [&] {
    return psf::launch_keys(rec_ptrs(rec), n, t->kp, reinterpret_cast<unsigned long long*>(d_out_keys), s);
  });
  return e == hipSuccess ? PSF_OK : hip_fail(e, "keys launch");
}

namespace {
psf_status count_occupied(psf_table* t, hipStream_t s, uint64_t* out) {
  unsigned long long* d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(unsigned long long));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  e = hipMemsetAsync(d, 0, sizeof(unsigned long long), s);
  if (e == hipSuccess) e = psf::launch_count_occupied(t->tv, nslots(t), d, s);
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(e, "count occupied");
  *out = h;
  return PSF_OK;
}
}  // namespace

PSF_API psf_status psf_get_stats(psf_table* t, psf_stats* out, psf_stream stream) {
  if (!t || !out) return fail(PSF_INVALID_ARGUMENT, "table or output is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  psf::DevStats d;
  std::vector<psf::BlockTouch> bt(psf::kTouchEntries);
  hipError_t e = hipMemcpyAsync(&d, t->tv.stats, sizeof d, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(bt.data(), t->tv.touch, bt.size() * sizeof(psf::BlockTouch),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "read statistics");
  uint64_t occ = 0;
  psf_status st = count_occupied(t, s, &occ);
  if (st != PSF_OK) return st;
  std::memset(out, 0, sizeof *out);
  out->submitted = t->submitted;
  for (uint32_t l = 0; l < psf::kStatLanes; ++l) {
    out->skipped += d.skipped[l][0];
    out->coord_overflow += d.coord_overflow[l][0];
  }
  out->dropped = d.dropped;
  for (uint32_t i = 0; i < psf::kTouchEntries; ++i) {
    if (i < t->touch_entries) out->touched_last += bt[i].last;
    out->touched_total += bt[i].total;
  }
  out->updates = t->updates;
  out->saturated = d.saturated;
  out->occupied = occ;
  for (int i = 0; i < 16; ++i) out->probe_hist[i] = d.probe_hist[i];
  return PSF_OK;
}

PSF_API psf_status psf_export_cells(psf_table* t, uint64_t* keys, uint32_t* n_new, uint32_t* c_old,
                                    float* state_rgb, uint64_t cap, uint64_t* count,
                                    psf_stream stream) {
  if (!t || !keys || !count) return fail(PSF_INVALID_ARGUMENT, "table, keys or count is NULL");
  if (t->tv.sh) return fail(PSF_NOT_SUPPORTED, "an SH payload table exports with psf_export_sh_cells");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  uint64_t occ = 0;
  psf_status st = count_occupied(t, s, &occ);
  if (st != PSF_OK) return st;
  *count = occ;
  if (occ > cap) return fail(PSF_BUFFER_TOO_SMALL, "more occupied cells than cap");
  if (occ == 0) return PSF_OK;
  // device scratch: cursor, keys, n_new, c_old, rgb
  const size_t bytes = 256 + occ * 8 + occ * 4 * 2 + occ * 12;
  char* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc export scratch");
  auto* cur = reinterpret_cast<unsigned long long*>(d);
  auto* dk = reinterpret_cast<unsigned long long*>(d + 256);
  auto* dn = reinterpret_cast<uint32_t*>(d + 256 + occ * 8);
  auto* dc = dn + occ;
  auto* drgb = reinterpret_cast<float*>(dc + occ);
  e = hipMemsetAsync(cur, 0, 8, s);
  if (e == hipSuccess)
    e = psf::launch_compact(t->tv, nslots(t), t->cfg.state_dtype, cur, occ, dk, dn, dc, drgb, s);
  if (e == hipSuccess) e = hipMemcpyAsync(keys, dk, occ * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && n_new) e = hipMemcpyAsync(n_new, dn, occ * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && c_old) e = hipMemcpyAsync(c_old, dc, occ * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && state_rgb) {
    for (int ch = 0; ch < 3 && e == hipSuccess; ++ch)
      e = hipMemcpyAsync(state_rgb + ch * cap, drgb + ch * occ, occ * 4, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "export");
}

PSF_API psf_status psf_export_variance(psf_table* t, uint64_t* keys, float* var, uint64_t cap, uint64_t* count,
                                       psf_stream stream) {
  if (!t || !keys || !count) return fail(PSF_INVALID_ARGUMENT, "table, keys or count is NULL");
  if (!t->tv.var) return fail(PSF_NOT_SUPPORTED, "the table keeps no variance (PSF_FLAG_TRACK_VARIANCE)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  uint64_t occ = 0;
  psf_status st = count_occupied(t, s, &occ);
  if (st != PSF_OK) return st;
  *count = occ;
  if (occ > cap) return fail(PSF_BUFFER_TOO_SMALL, "more occupied cells than cap");
  if (occ == 0) return PSF_OK;
  const size_t bytes = 256 + occ * 8 + occ * 4;
  char* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc export scratch");
  auto* cur = reinterpret_cast<unsigned long long*>(d);
  auto* dk = reinterpret_cast<unsigned long long*>(d + 256);
  auto* dv = reinterpret_cast<float*>(d + 256 + occ * 8);
  e = psf::launch_zero(cur, 16, s);
  if (e == hipSuccess) e = psf::launch_compact_var(t->tv, nslots(t), cur, occ, dk, dv, s);
  if (e == hipSuccess) e = hipMemcpyAsync(keys, dk, occ * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && var) e = hipMemcpyAsync(var, dv, occ * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "export");
}

PSF_API psf_status psf_export_sh_cells(psf_table* t, uint64_t* keys, uint32_t* c_old, float* coeff, uint64_t cap,
                                       uint64_t* count, psf_stream stream) {
  if (!t || !keys || !count) return fail(PSF_INVALID_ARGUMENT, "table, keys or count is NULL");
  if (!t->tv.sh) return fail(PSF_NOT_SUPPORTED, "not an SH payload table");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  uint64_t occ = 0;
  psf_status st = count_occupied(t, s, &occ);
  if (st != PSF_OK) return st;
  *count = occ;
  if (occ > cap) return fail(PSF_BUFFER_TOO_SMALL, "more occupied cells than cap");
  if (occ == 0) return PSF_OK;
  const size_t bytes = 256 + occ * 8 + occ * 4 + occ * 24;
  char* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc export scratch");
  auto* cur = reinterpret_cast<unsigned long long*>(d);
  auto* dk = reinterpret_cast<unsigned long long*>(d + 256);
  auto* dc = reinterpret_cast<uint32_t*>(d + 256 + occ * 8);
  auto* dv = reinterpret_cast<float*>(dc + occ);
  e = psf::launch_zero(cur, 16, s);
  if (e == hipSuccess) e = psf::launch_compact_sh(t->tv, nslots(t), cur, occ, dk, dc, dv, s);
  if (e == hipSuccess) e = hipMemcpyAsync(keys, dk, occ * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && c_old) e = hipMemcpyAsync(c_old, dc, occ * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && coeff) {
    for (int k = 0; k < 6 && e == hipSuccess; ++k)
      e = hipMemcpyAsync(coeff + k * cap, dv + k * occ, occ * 4, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "export");
}

// ------------------------------------------------------------------ allocation-free export
// Device scratch of psf_export_cells_noalloc: two counters (occupied cells,
// compaction cursor) in the first 256 bytes, then the compacted cells of at
// most kNoAllocCells entries (keys, n_new, c_old, rgb).  One copy per GPU,
// held until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): it uses the
// device address hipGetSymbolAddress returned for the current device.
constexpr uint64_t kNoAllocCells = 1ull << 20;
constexpr size_t kNoAllocBytes = 256 + kNoAllocCells * (8 + 4 + 4 + 12);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// The current device's copy of the scratch array (looked up once per device).
psf_status scratch_ptr(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices)
    return fail(PSF_NOT_SUPPORTED, "allocation-free export: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return PSF_OK;
}
}  // namespace

PSF_API psf_status psf_export_cells_noalloc(psf_table* t, uint64_t* keys, uint32_t* n_new, uint32_t* c_old,
                                            float* state_rgb, uint64_t cap, uint64_t* count,
                                            psf_stream stream) {
  if (!t || !keys || !count) return fail(PSF_INVALID_ARGUMENT, "table, keys or count is NULL");
  if (t->tv.sh) return fail(PSF_NOT_SUPPORTED, "an SH payload table exports with psf_export_sh_cells");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t->last = s;
  char* d = nullptr;
  psf_status st = scratch_ptr(&d);
  if (st != PSF_OK) return st;
  auto* occ_d = reinterpret_cast<unsigned long long*>(d);
  auto* cur = occ_d + 1;
  // counters cleared by a fill kernel (no memset node)
  hipError_t e = psf::launch_zero(d, 16, s);
  if (e == hipSuccess) e = psf::launch_count_occupied(t->tv, nslots(t), occ_d, s);
  unsigned long long occ = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&occ, occ_d, sizeof occ, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "count occupied");
  *count = occ;
  if (occ > kNoAllocCells)
    return fail(PSF_NOT_SUPPORTED, "allocation-free export handles at most 1048576 occupied cells; the table has " +
                                       std::to_string(occ) + " (use psf_export_cells)");
  if (occ > cap) return fail(PSF_BUFFER_TOO_SMALL, "more occupied cells than cap");
  if (occ == 0) return PSF_OK;
  // the arrays are packed for this call's count, as psf_export_cells packs them
  auto* dk = reinterpret_cast<unsigned long long*>(d + 256);
  auto* dn = reinterpret_cast<uint32_t*>(d + 256 + occ * 8);
  auto* dc = dn + occ;
  auto* drgb = reinterpret_cast<float*>(dc + occ);
  e = psf::launch_compact(t->tv, nslots(t), t->cfg.state_dtype, cur, occ, dk, dn, dc, drgb, s);
  if (e == hipSuccess) e = hipMemcpyAsync(keys, dk, occ * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && n_new) e = hipMemcpyAsync(n_new, dn, occ * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && c_old) e = hipMemcpyAsync(c_old, dc, occ * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && state_rgb) {
    for (int ch = 0; ch < 3 && e == hipSuccess; ++ch)
      e = hipMemcpyAsync(state_rgb + ch * cap, drgb + ch * occ, occ * 4, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "export");
}

// One allocation each side: the per-pass first blocks of the sessions
// (4 x cap words, padded to 256 bytes), then the session descriptors, so a
// launch uploads both with one copy.
struct psf_batch {
  uint32_t cap = 0;
  size_t begins_bytes = 0;
  void* host_raw = nullptr;  // pinned
  void* dev_raw = nullptr;
  uint32_t* hbeg = nullptr;
  psf::BatchSession* host = nullptr;
  uint32_t* dbeg = nullptr;
  psf::BatchSession* dev = nullptr;
  hipEvent_t copied = nullptr;
  bool in_flight = false;
};

PSF_API psf_status psf_batch_create(uint32_t max_sessions, psf_batch** out) {
  if (!out) return fail(PSF_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (max_sessions == 0 || max_sessions > 4096) return fail(PSF_INVALID_ARGUMENT, "max_sessions must be in [1, 4096]");
  psf_batch* b = new (std::nothrow) psf_batch();
  if (!b) return fail(PSF_OUT_OF_MEMORY, "host allocation failed");
  b->cap = max_sessions;
  b->begins_bytes = align_up((size_t)4 * max_sessions * sizeof(uint32_t), 256);
  const size_t bytes = b->begins_bytes + sizeof(psf::BatchSession) * max_sessions;
  hipError_t e = hipHostMalloc(&b->host_raw, bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&b->dev_raw, bytes);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
  if (e == hipSuccess) {
    b->hbeg = static_cast<uint32_t*>(b->host_raw);
    b->host = reinterpret_cast<psf::BatchSession*>(static_cast<char*>(b->host_raw) + b->begins_bytes);
    b->dbeg = static_cast<uint32_t*>(b->dev_raw);
    b->dev = reinterpret_cast<psf::BatchSession*>(static_cast<char*>(b->dev_raw) + b->begins_bytes);
  }
  if (e != hipSuccess) {
    if (b->host_raw) (void)hipHostFree(b->host_raw);
    if (b->dev_raw) (void)hipFree(b->dev_raw);
    delete b;
    (void)hipGetLastError();
    return fail(PSF_OUT_OF_MEMORY, std::string("batch context: ") + hipGetErrorString(e));
  }
  *out = b;
  return PSF_OK;
}

PSF_API psf_status psf_batch_destroy(psf_batch* b) {
  if (!b) return PSF_OK;
  hipError_t e = b->in_flight ? hipEventSynchronize(b->copied) : hipSuccess;
  (void)hipEventDestroy(b->copied);
  (void)hipHostFree(b->host_raw);
  (void)hipFree(b->dev_raw);
  delete b;
  return e == hipSuccess ? PSF_OK : hip_fail(e, "batch destroy");
}

PSF_API psf_status psf_iterate_batch(psf_batch* b, const psf_session* sessions, uint32_t k,
                                     psf_stream stream) {
  if (k == 0) return PSF_OK;
  if (!b || !sessions) return fail(PSF_INVALID_ARGUMENT, "batch context or sessions is NULL");
  if (k > b->cap) return fail(PSF_INVALID_ARGUMENT, "more sessions than the batch context holds");
  std::string why;
  for (uint32_t i = 0; i < k; ++i) {
    const psf_session& ss = sessions[i];
    if (!ss.table) return fail(PSF_INVALID_ARGUMENT, "session table is NULL");
    if (ss.n > 0 && !rec_ok(&ss.rec, ss.table, &why)) return fail(PSF_INVALID_ARGUMENT, why);
    if (ss.nq > 0 && !qry_ok(&ss.q, &why)) return fail(PSF_INVALID_ARGUMENT, why);
    if (ss.nq > 0 && !ss.d_out_rgb) return fail(PSF_INVALID_ARGUMENT, "session output is NULL");
    for (uint32_t j = 0; j < i; ++j)
      if (sessions[j].table == ss.table) return fail(PSF_INVALID_ARGUMENT, "a table appears twice in one batch");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // sessions that cannot join run alone first.  The merge launch sizes its
  // LDS for the widest partitions in it, so a session whose partitions are
  // wider than both the default and the narrowest candidate's runs alone
  // rather than slowing every other session's merge blocks.
  auto candidate = [&](const psf_session& ss) {
    const psf_table* t = ss.table;
    return ss.n > 0 && t->partitioned && !t->pending && ss.n <= t->pv.capacity;
  };
  uint32_t part_cap = 0;
  for (uint32_t i = 0; i < k; ++i)
    if (candidate(sessions[i]) && (part_cap == 0 || sessions[i].table->tv.part_log2 < part_cap))
      part_cap = sessions[i].table->tv.part_log2;
  if (part_cap < kDefaultPartLog2) part_cap = kDefaultPartLog2;
  uint32_t tile = 0;
  std::vector<uint32_t> batch;
  for (uint32_t i = 0; i < k; ++i) {
    const psf_session& ss = sessions[i];
    psf_table* t = ss.table;
    const bool ok = candidate(ss) && t->tv.part_log2 <= part_cap && (tile == 0 || t->pv.tile == tile);
    if (ok) {
      tile = t->pv.tile;
      batch.push_back(i);
      continue;
    }
    psf_status st = psf_iterate(t, &ss.rec, ss.n, &ss.q, ss.nq, ss.d_out_rgb, ss.d_out_found, stream);
    if (st != PSF_OK) return st;
  }
  if (batch.empty()) return PSF_OK;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return hip_fail(e, "capture query");
  if (cap == hipStreamCaptureStatusNone && b->in_flight) {
    e = hipEventSynchronize(b->copied);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor reuse");
    b->in_flight = false;
  }
  uint32_t tiles = 0, parts = 0, qblks = 0, trans = 0;
  for (uint32_t j = 0; j < batch.size(); ++j) {
    const psf_session& ss = sessions[batch[j]];
    psf_table* t = ss.table;
    psf::BatchSession& d = b->host[j];
    std::memset(&d, 0, sizeof d);
    d.tv = t->tv;
    d.pv = t->pv;
    d.kp = t->kp;
    d.bp = t->bp;
    d.rec = rec_ptrs(&ss.rec);
    d.n = ss.n;
    d.nq = ss.nq;
    if (ss.nq > 0) d.q = qry_ptrs(&ss.q);
    d.out = ss.d_out_rgb;
    d.found = ss.d_out_found;
    d.fused_query = (ss.nq == ss.n && same_vertices(&ss.rec, &ss.q)) ? 1 : 0;
    if (!d.fused_query) d.pv.perm = nullptr;
    d.pv.weights = d.rec.weight != nullptr;
    d.tile_begin = tiles;
    d.ntiles = (uint32_t)((ss.n + t->pv.tile - 1) / t->pv.tile);
    d.part_begin = parts;
    d.nparts = 1u << (t->cfg.log2_slots - t->tv.part_log2);
    d.trans_begin = trans;
    if (!transpose_runs(t, d.ntiles)) d.pv.runs_t = nullptr;
    d.ntrans = d.pv.runs_t ? psf::transpose_blocks(d.ntiles, d.nparts) : 0u;
    d.qblk_begin = qblks;
    d.nqblk = d.fused_query ? d.ntiles : (uint32_t)((ss.nq + psf::kQueryBlock - 1) / psf::kQueryBlock);
    b->hbeg[j] = d.tile_begin;
    b->hbeg[b->cap + j] = d.part_begin;
    b->hbeg[2 * b->cap + j] = d.qblk_begin;
    b->hbeg[3 * b->cap + j] = d.trans_begin;
    tiles += d.ntiles;
    parts += (d.nparts + 7u) & ~7u;
    trans += d.ntrans;
    qblks += d.nqblk;
  }
  const uint32_t m = (uint32_t)batch.size();
  e = hipMemcpyAsync(b->dev_raw, b->host_raw, b->begins_bytes + sizeof(psf::BatchSession) * m,
                     hipMemcpyHostToDevice, s);
  if (e == hipSuccess && cap == hipStreamCaptureStatusNone) e = hipEventRecord(b->copied, s);
  if (e != hipSuccess) return hip_fail(e, "batch descriptor copy");
  b->in_flight = cap == hipStreamCaptureStatusNone;
  e = psf::launch_batch(b->dev, b->dbeg, b->hbeg, b->cap, b->host, m, s);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  for (uint32_t j = 0; j < m; ++j) {
    const psf_session& ss = sessions[batch[j]];
    psf_table* t = ss.table;
    t->last = s;
    t->submitted += ss.n;
    t->updates++;
    t->touch_entries = b->host[j].nparts;
  }
  return PSF_OK;
}

PSF_API psf_status psf_estimate(psf_table* t_oe, psf_table* t_fli, const psf_estimate_args* a, uint64_t n,
                                int32_t mode, float param, float* d_out_rgb, uint8_t* d_out_applied,
                                psf_stream stream) {
  if (!t_oe || !t_fli) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (n == 0) return PSF_OK;
  if (!a) return fail(PSF_INVALID_ARGUMENT, "estimate arguments are NULL");
  if (!a->px || !a->py || !a->pz || !a->nx || !a->ny || !a->nz)
    return fail(PSF_INVALID_ARGUMENT, "position and normal arrays are required");
  if (a->rough && (!a->oox || !a->ooy || !a->ooz || !a->oix || !a->oiy || !a->oiz))
    return fail(PSF_INVALID_ARGUMENT, "direction arrays are required when roughness is given");
  if (!a->gr || !a->gg || !a->gb || !a->wp) return fail(PSF_INVALID_ARGUMENT, "sample and weight arrays are required");
  if (mode != PSF_EST_CV && mode != PSF_EST_BIASED) return fail(PSF_INVALID_ARGUMENT, "mode must be CV or BIASED");
  if (!std::isfinite(param)) return fail(PSF_INVALID_ARGUMENT, "param must be finite");
  if (t_oe->tv.sh || t_fli->tv.sh) return fail(PSF_NOT_SUPPORTED, "estimators on SH payload tables");
  if (!d_out_rgb) return fail(PSF_INVALID_ARGUMENT, "output array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  t_oe->last = s;
  t_fli->last = s;
  psf::EstPtrs ep;
  ep.qo = psf::QryPtrs{a->px, a->py, a->pz, a->nx, a->ny, a->nz, a->oox, a->ooy, a->ooz, a->rough, a->footprint};
  ep.qi = psf::QryPtrs{a->px, a->py, a->pz, a->nx, a->ny, a->nz, a->oix, a->oiy, a->oiz, a->rough, a->footprint};
  ep.gr = a->gr;
  ep.gg = a->gg;
  ep.gb = a->gb;
  ep.wp = a->wp;
  hipError_t e = timed(t_oe, PSF_K_ESTIMATE, s, [&] {
    return psf::launch_estimate(ep, n, t_oe->kp, t_oe->tv, t_oe->cfg.state_dtype, t_fli->kp, t_fli->tv,
                                t_fli->cfg.state_dtype, mode, param, d_out_rgb, d_out_applied, s);
  });
  return e == hipSuccess ? PSF_OK : hip_fail(e, "estimate launch");
}

PSF_API psf_status psf_sample_paths(const psf_prim* d_prims, uint32_t n_prims, const psf_camera* cam,
                                    const psf_path_params* p, const psf_path_out* out, psf_stream stream) {
  if (!cam || !p || !out) return fail(PSF_INVALID_ARGUMENT, "camera, parameters or outputs are NULL");
  if (n_prims > 4096) return fail(PSF_INVALID_ARGUMENT, "at most 4096 primitives");
  if (n_prims > 0 && !d_prims) return fail(PSF_INVALID_ARGUMENT, "primitives are NULL");
  if (p->verts == 0) return fail(PSF_INVALID_ARGUMENT, "verts must be >= 1");
  if (p->mode != PSF_PATHS_LO && p->mode != PSF_PATHS_LOE) return fail(PSF_INVALID_ARGUMENT, "unknown mode");
  if (p->origin != PSF_ORIGIN_CAMERA && p->origin != PSF_ORIGIN_POINT)
    return fail(PSF_INVALID_ARGUMENT, "unknown origin");
  if (cam->width == 0 || cam->height == 0 || cam->spp == 0) return fail(PSF_INVALID_ARGUMENT, "empty image");
  if (!(cam->fov_y > 0.0f && cam->fov_y < 3.14159f)) return fail(PSF_INVALID_ARGUMENT, "fov_y must be in (0, pi)");
  const uint64_t paths = (uint64_t)cam->width * cam->height * cam->spp;
  if (paths > (1ull << 32)) return fail(PSF_INVALID_ARGUMENT, "more than 2^32 paths");
  float* const arrays[] = {out->px,  out->py,  out->pz,  out->nx,  out->ny,  out->nz,   out->ox,
                           out->oy,  out->oz,  out->rough, out->qx, out->qy, out->qz,  out->qnx,
                           out->qny, out->qnz, out->qox, out->qoy, out->qoz, out->qrough, out->t_r,
                           out->t_g, out->t_b, out->le_r, out->le_g, out->le_b};
  for (float* a : arrays)
    if (!a) return fail(PSF_INVALID_ARGUMENT, "an output array is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = psf::launch_sample_paths(d_prims, n_prims, *cam, *p, paths, *out, s);
  return e == hipSuccess ? PSF_OK : hip_fail(e, "path sampler launch");
}

PSF_API psf_status psf_philox(const uint32_t* d_ctr, const uint32_t* d_key, uint64_t n, uint32_t* d_out,
                              psf_stream stream) {
  if (n == 0) return PSF_OK;
  if (!d_ctr || !d_key || !d_out) return fail(PSF_INVALID_ARGUMENT, "arrays are NULL");
  hipError_t e = psf::launch_philox(d_ctr, d_key, n, d_out, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? PSF_OK : hip_fail(e, "philox launch");
}

PSF_API psf_status psf_kernel_times(psf_table* t, uint64_t* launches, double* total_ms, int reset) {
  if (!t) return fail(PSF_INVALID_ARGUMENT, "table is NULL");
  if (!t->timer) return fail(PSF_NOT_SUPPORTED, "table was created without PSF_FLAG_TIMING");
  hipError_t e = t->timer->flush();
  if (e != hipSuccess) return hip_fail(e, "kernel timing");
  for (int k = 0; k < PSF_K_COUNT; ++k) {
    if (launches) launches[k] = t->timer->launches[k];
    if (total_ms) total_ms[k] = t->timer->total_ms[k];
    if (reset) {
      t->timer->launches[k] = 0;
      t->timer->total_ms[k] = 0.0;
    }
  }
  return PSF_OK;
}

PSF_API const char* psf_kernel_name(uint32_t k) {
  static const char* names[PSF_K_COUNT] = {"keys", "insert_direct", "bin", "merge", "merge_blend",
                                           "update", "query", "batch", "transpose", "estimate", "step"};
  return k < PSF_K_COUNT ? names[k] : "";
}

PSF_API const char* psf_last_error(void) { return g_err.c_str(); }

PSF_API const char* psf_version(void) { return "psf 0.1 gfx950"; }

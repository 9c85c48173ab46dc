// Seeded synthetic path-vertex generator.
//
// Produces the vertex records a path tracer would hand to the filtering
// library: one path per pixel sample, V vertices per path, written depth-major
// with scanline pixel order inside a depth (paths are cast in waves, one path
// per pixel per frame, as in the paper's progressive solver).  The scenes are
// procedural (axis-aligned open box with a sphere, or random quads and
// spheres), the radiance attached to each vertex is a smooth analytic field
// times seeded noise.  Nothing here implements the filtering method; the
// same records feed both the oracle and the GPU library.
//
// Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), keyed by (seed, iteration),
// counter (pixel, sample, attempt/vertex, purpose), so every record is a pure
// function of its coordinates and the output does not depend on threading.
// Orthonormal basis construction: Duff et al., "Building an Orthonormal
// Basis, Revisited", JCGT 2017.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------- Philox
struct U4 {
  uint32_t v[4];
};

inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

U4 philox4x32_10(U4 ctr, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int round = 0; round < 10; ++round) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, ctr.v[0], &hi0, &lo0);
    mulhilo32(M1, ctr.v[2], &hi1, &lo1);
    U4 nx;
    nx.v[0] = hi1 ^ ctr.v[1] ^ k0;
    nx.v[1] = lo1;
    nx.v[2] = hi0 ^ ctr.v[3] ^ k1;
    nx.v[3] = lo0;
    ctr = nx;
    k0 += W0;
    k1 += W1;
  }
  return ctr;
}

// uniform in (0, 1): 24 random bits, centred in their interval
inline float u01(uint32_t x) { return ((float)(x >> 8) + 0.5f) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------- vectors
struct V3 {
  float x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
inline float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline V3 normalize(V3 a) {
  float l = std::sqrt(dot(a, a));
  return l > 0.0f ? a * (1.0f / l) : V3{0.0f, 0.0f, 1.0f};
}

void onb(V3 n, V3* b1, V3* b2) {
  float sign = std::copysign(1.0f, n.z);
  float a = -1.0f / (sign + n.z);
  float b = n.x * n.y * a;
  *b1 = {1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x};
  *b2 = {b, sign + n.y * n.y * a, -n.y};
}

// ---------------------------------------------------------------- scene
struct Quad {
  V3 c, u, v, n;
  float hu, hv, rough;
  int32_t tex;  // >= 0: roughness drawn per 1x1 tile from this id
};
struct Sphere {
  V3 c;
  float r, rough;
};
struct Scene {
  std::vector<Quad> quads;
  std::vector<Sphere> spheres;
  uint32_t seed = 0;
  float glossy_frac = -1.0f;
};

// roughness distribution of the random scenes: U[0.05, 1] when glossy_frac is
// negative, else a glossy_frac share in [0.05, 0.3) and the rest in [0.3, 1]
float rough_from(float glossy_frac, float a, float b) {
  if (glossy_frac < 0.0f) return 0.05f + 0.95f * a;
  if (a < glossy_frac) return 0.05f + 0.25f * b * 0.999f;
  return 0.3f + 0.7f * b;
}

struct Hit {
  float t;
  V3 p, n;
  float rough;
};

bool intersect(const Scene& sc, V3 o, V3 d, Hit* h) {
  const Quad* hq = nullptr;
  V3 hl{0.0f, 0.0f, 0.0f};
  const float eps = 1e-4f;
  float best = 1e30f;
  bool any = false;
  for (const Quad& q : sc.quads) {
    float den = dot(d, q.n);
    if (std::fabs(den) < 1e-9f) continue;
    float t = dot(q.c - o, q.n) / den;
    if (!(t > eps && t < best)) continue;
    V3 p = o + d * t;
    V3 l = p - q.c;
    if (std::fabs(dot(l, q.u)) > q.hu || std::fabs(dot(l, q.v)) > q.hv) continue;
    best = t;
    any = true;
    h->t = t;
    h->p = p;
    h->n = q.n;
    h->rough = q.rough;
    hq = &q;
    hl = l;
  }
  for (const Sphere& s : sc.spheres) {
    V3 oc = o - s.c;
    float b = dot(oc, d);
    float cc = dot(oc, oc) - s.r * s.r;
    float disc = b * b - cc;
    if (disc < 0.0f) continue;
    float sq = std::sqrt(disc);
    float t = -b - sq;
    if (!(t > eps)) t = -b + sq;
    if (!(t > eps && t < best)) continue;
    best = t;
    any = true;
    h->t = t;
    h->p = o + d * t;
    h->n = normalize(h->p - s.c);
    h->rough = s.rough;
    hq = nullptr;
  }
  if (any && hq && hq->tex >= 0) {
    int32_t tu = (int32_t)std::floor(dot(hl, hq->u) + hq->hu);
    int32_t tv = (int32_t)std::floor(dot(hl, hq->v) + hq->hv);
    U4 r = philox4x32_10(U4{{(uint32_t)hq->tex, (uint32_t)tu, (uint32_t)tv, 9u}}, sc.seed, 0x7e87u);
    h->rough = rough_from(sc.glossy_frac, u01(r.v[0]), u01(r.v[1]));
  }
  if (any && dot(h->n, d) > 0.0f) h->n = h->n * -1.0f;
  return any;
}

}  // namespace

extern "C" {

struct synth_params {
  int32_t width, height, spp, verts;
  uint32_t seed;
  float cam[3];
  float look[3];
  float fov_y_deg;
  int32_t field;       // 0 smooth analytic, 1 constant, 2 linear
  int32_t noise;       // 0 none, 1 exponential(1), 2 lognormal(0, sigma)
  float sigma;
  float field_scale;   // smooth field evaluated at p / field_scale
  float amp[3];        // smooth field per-channel amplitude / constant value
  float lin_a[9];      // linear field: rgb_c = lin_b[c] + dot(lin_a[3c..3c+2], p)
  float lin_b[3];
  float light[3];      // glossy lobe axis
  float glossy_thr;    // vertices with roughness below this get the lobe
  int32_t glossy_lobe; // 1 multiplies glossy vertices by the lobe
};

struct synth_stats {
  uint64_t restarts;
  uint64_t fallbacks;
  uint64_t glossy;
};

void* synth_scene_create(int kind, uint32_t seed, int n_quads, int n_spheres, float glossy_frac) {
  Scene* sc = new Scene();
  if (kind == 0) {
    // open box [0,1]^3: floor, ceiling, back, left, right; sphere r=0.3
    auto add = [&](V3 c, V3 u, V3 v) {
      Quad q;
      q.c = c;
      q.u = u;
      q.v = v;
      q.n = cross(u, v);
      q.hu = 0.5f;
      q.hv = 0.5f;
      q.rough = 1.0f;
      q.tex = -1;
      sc->quads.push_back(q);
    };
    add({0.5f, 0.0f, 0.5f}, {1, 0, 0}, {0, 0, 1});
    add({0.5f, 1.0f, 0.5f}, {1, 0, 0}, {0, 0, 1});
    add({0.5f, 0.5f, 1.0f}, {1, 0, 0}, {0, 1, 0});
    add({0.0f, 0.5f, 0.5f}, {0, 1, 0}, {0, 0, 1});
    add({1.0f, 0.5f, 0.5f}, {0, 1, 0}, {0, 0, 1});
    sc->spheres.push_back({{0.5f, 0.3f, 0.5f}, 0.3f, 1.0f});
    return sc;
  }
  auto draw = [&](uint32_t prim, uint32_t purpose) {
    U4 c{{prim, 0x5ce7e000u, purpose, 0u}};
    return philox4x32_10(c, seed, 0x243f6a88u);
  };
  sc->seed = seed;
  sc->glossy_frac = glossy_frac;
  auto rough_of = [&](uint32_t prim) {
    U4 r = draw(prim, 7);
    return rough_from(glossy_frac, u01(r.v[0]), u01(r.v[1]));
  };
  for (int i = 0; i < n_quads; ++i) {
    U4 r0 = draw((uint32_t)i, 1), r1 = draw((uint32_t)i, 2);
    Quad q;
    q.c = {-4.0f + 8.0f * u01(r0.v[0]), -4.0f + 8.0f * u01(r0.v[1]), -4.0f + 8.0f * u01(r0.v[2])};
    float z = 1.0f - 2.0f * u01(r1.v[0]);
    float phi = 6.28318531f * u01(r1.v[1]);
    float s = std::sqrt(std::max(0.0f, 1.0f - z * z));
    V3 n = {s * std::cos(phi), s * std::sin(phi), z};
    V3 b1, b2;
    onb(n, &b1, &b2);
    float rot = 6.28318531f * u01(r0.v[3]);
    q.u = b1 * std::cos(rot) + b2 * std::sin(rot);
    q.v = cross(n, q.u);
    q.n = n;
    q.hu = 0.5f * (0.5f + 1.5f * u01(r1.v[2]));
    q.hv = 0.5f * (0.5f + 1.5f * u01(r1.v[3]));
    q.rough = rough_of((uint32_t)i);
    q.tex = i;
    sc->quads.push_back(q);
  }
  // enclosing room x in [-8,8], y in [-6,6], z in [-12,8], diffuse walls, so
  // that every camera ray and most bounces find a surface
  {
    const float xs = 8.0f, ys = 6.0f, z0 = -12.0f, z1 = 8.0f, zc = 0.5f * (z0 + z1),
                zh = 0.5f * (z1 - z0);
    auto wall = [&](V3 c, V3 u, V3 v, float hu, float hv, uint32_t id) {
      Quad q;
      q.c = c;
      q.u = u;
      q.v = v;
      q.n = cross(u, v);
      q.hu = hu;
      q.hv = hv;
      q.rough = rough_of(id);
      q.tex = (int32_t)id;
      sc->quads.push_back(q);
    };
    wall({0.0f, -ys, zc}, {1, 0, 0}, {0, 0, 1}, xs, zh, 2000u);
    wall({0.0f, ys, zc}, {1, 0, 0}, {0, 0, 1}, xs, zh, 2001u);
    wall({-xs, 0.0f, zc}, {0, 1, 0}, {0, 0, 1}, ys, zh, 2002u);
    wall({xs, 0.0f, zc}, {0, 1, 0}, {0, 0, 1}, ys, zh, 2003u);
    wall({0.0f, 0.0f, z0}, {1, 0, 0}, {0, 1, 0}, xs, ys, 2004u);
    wall({0.0f, 0.0f, z1}, {1, 0, 0}, {0, 1, 0}, xs, ys, 2005u);
  }
  for (int i = 0; i < n_spheres; ++i) {
    uint32_t id = 1000u + (uint32_t)i;
    U4 r0 = draw(id, 1);
    Sphere s;
    s.c = {-4.0f + 8.0f * u01(r0.v[0]), -4.0f + 8.0f * u01(r0.v[1]), -4.0f + 8.0f * u01(r0.v[2])};
    s.r = 0.2f + 0.6f * u01(r0.v[3]);
    s.rough = rough_of(id);
    sc->spheres.push_back(s);
  }
  return sc;
}

void synth_scene_destroy(void* s) { delete static_cast<Scene*>(s); }

int synth_scene_counts(void* s, int* quads, int* spheres) {
  Scene* sc = static_cast<Scene*>(s);
  *quads = (int)sc->quads.size();
  *spheres = (int)sc->spheres.size();
  return 0;
}

// out: 13 float arrays (px py pz nx ny nz ox oy oz r g b rough), each of
// width*height*spp*verts entries.  Returns 0, or -1 on bad arguments.
int synth_generate(void* scene, const synth_params* prm, uint32_t iteration, float** out,
                   int nthreads, synth_stats* stats) {
  const Scene& sc = *static_cast<Scene*>(scene);
  const synth_params P = *prm;
  if (P.width <= 0 || P.height <= 0 || P.spp <= 0 || P.verts <= 0) return -1;
  for (int i = 0; i < 13; ++i)
    if (!out[i]) return -1;
  const uint64_t pix = (uint64_t)P.width * (uint64_t)P.height;
  const uint64_t per_depth = pix * (uint64_t)P.spp;
  V3 cam = {P.cam[0], P.cam[1], P.cam[2]};
  V3 look = normalize({P.look[0], P.look[1], P.look[2]});
  V3 up0 = {0.0f, 1.0f, 0.0f};
  V3 right = normalize(cross(up0, look));
  V3 up = cross(look, right);
  float th = std::tan(0.5f * P.fov_y_deg * 3.14159265f / 180.0f);
  float aspect = (float)P.width / (float)P.height;
  V3 light = normalize({P.light[0], P.light[1], P.light[2]});
  const float two_pi = 6.28318531f;

  auto radiance = [&](V3 p, V3 wo, float rough, float noise, float* rgb) {
    float f[3];
    if (P.field == 1) {
      for (int c = 0; c < 3; ++c) f[c] = P.amp[c];
    } else if (P.field == 2) {
      for (int c = 0; c < 3; ++c)
        f[c] = P.lin_b[c] + P.lin_a[3 * c] * p.x + P.lin_a[3 * c + 1] * p.y + P.lin_a[3 * c + 2] * p.z;
    } else {
      V3 q = p * (1.0f / P.field_scale);
      float base = (1.0f + 0.5f * std::sin(two_pi * q.x) * std::cos(two_pi * q.z)) * (0.75f + 0.25f * q.y);
      for (int c = 0; c < 3; ++c) f[c] = P.amp[c] * base;
    }
    float lobe = 1.0f;
    if (P.glossy_lobe && rough < P.glossy_thr) {
      float cl = std::max(0.0f, dot(wo, light));
      float c2 = cl * cl, c4 = c2 * c2;
      lobe = 1.0f + 2.0f * c4 * c4;
    }
    for (int c = 0; c < 3; ++c) rgb[c] = f[c] * lobe * noise;
  };

  auto work = [&](uint64_t p_begin, uint64_t p_end, synth_stats* st) {
    for (uint64_t pl = p_begin; pl < p_end; ++pl) {
      for (int s = 0; s < P.spp; ++s) {
        int rec = 0;
        uint32_t attempt = 0;
        while (rec < P.verts) {
          if (attempt > 64) {
            // practically unreachable: emit degenerate records in front of the camera
            for (; rec < P.verts; ++rec) {
              uint64_t idx = (uint64_t)rec * per_depth + pl * (uint64_t)P.spp + (uint64_t)s;
              V3 p = cam + look;
              float vals[13] = {p.x, p.y, p.z, -look.x, -look.y, -look.z, -look.x, -look.y, -look.z,
                                0.0f, 0.0f, 0.0f, 1.0f};
              for (int k = 0; k < 13; ++k) out[k][idx] = vals[k];
              st->fallbacks++;
            }
            break;
          }
          U4 cr = philox4x32_10(U4{{(uint32_t)pl, (uint32_t)s, (attempt << 8) | (uint32_t)rec, 0u}},
                                P.seed, iteration);
          uint64_t src = pl;
          if (attempt >= 4) {
            uint64_t r64 = ((uint64_t)cr.v[2] << 32) | cr.v[3];
            src = r64 % pix;
          }
          float x = (float)(src % (uint64_t)P.width), y = (float)(src / (uint64_t)P.width);
          float sx = ((x + u01(cr.v[0])) / (float)P.width * 2.0f - 1.0f) * th * aspect;
          float sy = (1.0f - (y + u01(cr.v[1])) / (float)P.height * 2.0f) * th;
          V3 o = cam;
          V3 d = normalize(look + right * sx + up * sy);
          while (rec < P.verts) {
            Hit h{};
            if (!intersect(sc, o, d, &h)) break;
            U4 rb = philox4x32_10(
                U4{{(uint32_t)pl, (uint32_t)s, (attempt << 8) | (uint32_t)rec, 1u}}, P.seed, iteration);
            V3 wo = d * -1.0f;
            float noise = 1.0f;
            if (P.noise == 1) {
              noise = -std::log(u01(rb.v[2]));
            } else if (P.noise == 2) {
              float z = std::sqrt(-2.0f * std::log(u01(rb.v[2]))) * std::cos(two_pi * u01(rb.v[3]));
              noise = std::exp(P.sigma * z);
            }
            float rgb[3];
            radiance(h.p, wo, h.rough, noise, rgb);
            uint64_t idx = (uint64_t)rec * per_depth + pl * (uint64_t)P.spp + (uint64_t)s;
            float vals[13] = {h.p.x, h.p.y, h.p.z, h.n.x, h.n.y, h.n.z, wo.x, wo.y, wo.z,
                              rgb[0], rgb[1], rgb[2], h.rough};
            for (int k = 0; k < 13; ++k) out[k][idx] = vals[k];
            if (h.rough < P.glossy_thr) st->glossy++;
            ++rec;
            // scatter
            V3 b1, b2;
            float u1 = u01(rb.v[0]), u2 = u01(rb.v[1]);
            V3 nd;
            if (h.rough < 0.3f) {
              V3 m = d - h.n * (2.0f * dot(d, h.n));
              float e = std::max(1.0f, 2.0f / (h.rough * h.rough) - 2.0f);
              float ct = std::pow(u1, 1.0f / (e + 1.0f));
              float st2 = std::sqrt(std::max(0.0f, 1.0f - ct * ct));
              onb(m, &b1, &b2);
              nd = b1 * (st2 * std::cos(two_pi * u2)) + b2 * (st2 * std::sin(two_pi * u2)) + m * ct;
              if (dot(nd, h.n) <= 0.0f) nd = m;
            } else {
              float r = std::sqrt(u1);
              onb(h.n, &b1, &b2);
              nd = b1 * (r * std::cos(two_pi * u2)) + b2 * (r * std::sin(two_pi * u2)) +
                   h.n * std::sqrt(std::max(0.0f, 1.0f - u1));
            }
            o = h.p + h.n * 1e-4f;
            d = normalize(nd);
          }
          if (rec < P.verts) {
            attempt++;
            st->restarts++;
          }
        }
      }
    }
  };

  int nt = std::max(1, nthreads);
  std::vector<synth_stats> sts((size_t)nt, synth_stats{0, 0, 0});
  std::vector<std::thread> th_pool;
  uint64_t chunk = (pix + (uint64_t)nt - 1) / (uint64_t)nt;
  for (int t = 0; t < nt; ++t) {
    uint64_t b = std::min(pix, (uint64_t)t * chunk), e = std::min(pix, b + chunk);
    if (nt == 1) {
      work(b, e, &sts[0]);
    } else {
      th_pool.emplace_back(work, b, e, &sts[(size_t)t]);
    }
  }
  for (auto& t : th_pool) t.join();
  if (stats) {
    *stats = synth_stats{0, 0, 0};
    for (auto& s : sts) {
      stats->restarts += s.restarts;
      stats->fallbacks += s.fallbacks;
      stats->glossy += s.glossy;
    }
  }
  return 0;
}

// Philox known-answer access for tests.
void synth_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  U4 c{{ctr[0], ctr[1], ctr[2], ctr[3]}};
  U4 r = philox4x32_10(c, key[0], key[1]);
  std::memcpy(out, r.v, sizeof r.v);
}

}  // extern "C"

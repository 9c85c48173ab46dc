// Procedural path sampler for the progressive solver (Sec. 2.2; Algorithms
// 1 and 2): the step upstream of the hash path.  One thread traces one path
// of V vertices x_1..x_V (plus x_{V+1}, the next vertex of x_V) through a
// scene of quads and spheres with Lambertian materials, and writes, per
// vertex, what one frame of the solver consumes: the vertex as a record
// (position, normal, outgoing direction, roughness), its next vertex as a
// query, the throughput factor f G w / p of the sampled step and the
// emission argument:
//   Algorithm 1 (L_o):    L_e(x_i)
//   Algorithm 2 (L_o\e):  w_nee NEE(x_i) + t_i w_bsdf L_e(x_{i+1})
// where NEE samples a point on a randomly chosen emitter and the two ways of
// reaching an emitter are combined by the balance heuristic.  Records are
// depth-major (vertex i of every path, then vertex i + 1), as the library's
// record order expects.  A path that leaves the scene restarts from its
// origin (so every path has exactly V vertices); the vertex before the
// escape gets an invalid next vertex (its lookup finds nothing) and no
// transported emission.
//
// Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key
// (seed, frame), counter (path, vertex, purpose, 0): each path is a pure
// function of its coordinates.  Directions around a normal use the
// orthonormal basis of Duff et al. (JCGT 2017).
#include "psf_internal.h"

namespace psf {

// ------------------------------------------------------------------ Philox
struct Philox {
  uint32_t v[4];
};

__host__ __device__ __forceinline__ Philox philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                         uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u, kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kM0 * c0, p1 = (uint64_t)kM1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += kW0;
    k1 += kW1;
  }
  return Philox{{c0, c1, c2, c3}};
}

// uniform in (0, 1): the top 24 bits, centred in their interval
__device__ __forceinline__ float unit01(uint32_t x) { return ((float)(x >> 8) + 0.5f) * (1.0f / 16777216.0f); }

__global__ void k_philox(const uint32_t* ctr, const uint32_t* key, uint64_t n, uint32_t* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Philox r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[2 * i],
                                 key[2 * i + 1]);
  for (int k = 0; k < 4; ++k) out[4 * i + k] = r.v[k];
}

// ------------------------------------------------------------------ geometry
struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 normalize(V3 a) {
  const float l = sqrtf(dot(a, a));
  return l > 0.0f ? a * (1.0f / l) : v3(0.0f, 0.0f, 1.0f);
}

// direction around the normal n from local coordinates (x, y, z), z along n
__device__ __forceinline__ V3 around(V3 n, float x, float y, float z) {
  const float sgn = n.z >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sgn + n.z);
  const float b = n.x * n.y * a;
  const V3 t1 = v3(1.0f + sgn * n.x * n.x * a, sgn * b, -sgn * n.x);
  const V3 t2 = v3(b, sgn + n.y * n.y * a, -n.y);
  return normalize(t1 * x + t2 * y + n * z);
}

// Cosine-weighted direction about n (Malley's method): density cos / pi.
__device__ __forceinline__ V3 cosine_dir(V3 n, float u1, float u2) {
  const float r = sqrtf(u1), phi = 6.28318530717958647692f * u2;
  return around(n, r * cosf(phi), r * sinf(phi), sqrtf(fmaxf(0.0f, 1.0f - u1)));
}

__device__ __forceinline__ V3 uniform_sphere(float u1, float u2) {
  const float z = 1.0f - 2.0f * u1, r = sqrtf(fmaxf(0.0f, 1.0f - z * z)), phi = 6.28318530717958647692f * u2;
  return v3(r * cosf(phi), r * sinf(phi), z);
}

struct Prim {
  int32_t kind;
  V3 p, u, v;
  V3 albedo, emit;
  float rough;
};

__device__ __forceinline__ Prim load_prim(const PathPrim* ps, uint32_t i) {
  const PathPrim& s = ps[i];
  Prim q;
  q.kind = s.kind;
  q.p = v3(s.p[0], s.p[1], s.p[2]);
  q.u = v3(s.u[0], s.u[1], s.u[2]);
  q.v = v3(s.v[0], s.v[1], s.v[2]);
  q.albedo = v3(s.albedo[0], s.albedo[1], s.albedo[2]);
  q.emit = v3(s.emission[0], s.emission[1], s.emission[2]);
  q.rough = s.rough;
  return q;
}

__device__ __forceinline__ bool emissive(const Prim& q) { return q.emit.x > 0.0f || q.emit.y > 0.0f || q.emit.z > 0.0f; }

__device__ __forceinline__ float prim_area(const Prim& q) {
  if (q.kind == kPrimSphere) return 12.5663706143591729539f * q.u.x * q.u.x;
  const V3 c = cross(q.u, q.v);
  return 4.0f * sqrtf(dot(c, c));
}

// Nearest hit along o + t d with t in (t_min, t_max): primitive index or -1.
// Quads are centre p with half edges u, v; spheres centre p, radius u.x.
__device__ int32_t trace(const PathPrim* ps, uint32_t np, V3 o, V3 d, float t_min, float t_max, float& t_hit) {
  int32_t best = -1;
  t_hit = t_max;
  for (uint32_t i = 0; i < np; ++i) {
    const Prim q = load_prim(ps, i);
    if (q.kind == kPrimSphere) {
      const V3 oc = o - q.p;
      const float b = dot(oc, d), c = dot(oc, oc) - q.u.x * q.u.x;
      const float disc = b * b - c;
      if (disc < 0.0f) continue;
      const float s = sqrtf(disc);
      float t = -b - s;
      if (!(t > t_min)) t = -b + s;
      if (t > t_min && t < t_hit) {
        t_hit = t;
        best = (int32_t)i;
      }
    } else {
      const V3 n = cross(q.u, q.v);
      const float den = dot(n, d);
      if (den == 0.0f) continue;
      const float t = dot(n, q.p - o) / den;
      if (!(t > t_min && t < t_hit)) continue;
      const V3 h = o + d * t - q.p;
      const float a = dot(h, q.u) / dot(q.u, q.u), b = dot(h, q.v) / dot(q.v, q.v);
      if (fabsf(a) <= 1.0f && fabsf(b) <= 1.0f) {
        t_hit = t;
        best = (int32_t)i;
      }
    }
  }
  return best;
}

// geometric normal of primitive q at point h (not face-forwarded)
__device__ __forceinline__ V3 prim_normal(const Prim& q, V3 h) {
  return q.kind == kPrimSphere ? normalize(h - q.p) : normalize(cross(q.u, q.v));
}

// ------------------------------------------------------------------ paths
struct PathVertex {
  bool valid;
  V3 p, n, wo;  // n faces wo
  int32_t prim;
};

__device__ __forceinline__ float lum_max(V3 a) { return fmaxf(a.x, fmaxf(a.y, a.z)); }

__global__ void __launch_bounds__(256) k_sample_paths(const PathPrim* prims, uint32_t np, PathCamera cam,
                                                     PathParams prm, uint64_t n_paths, PathOut out) {
  const uint64_t path = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (path >= n_paths) return;
  const uint32_t V = prm.verts;
  constexpr float kEps = 1e-4f, kInvPi = 0.318309886183790671538f;
  // emitters, for next-event estimation
  uint32_t n_emit = 0;
  for (uint32_t i = 0; i < np; ++i) n_emit += emissive(load_prim(prims, i)) ? 1u : 0u;
  auto rnd = [&](uint32_t vertex, uint32_t purpose) {
    return philox4x32_10((uint32_t)path, (uint32_t)(path >> 32) ^ vertex, purpose, 0u, prm.seed, prm.frame);
  };
  // origin ray of attempt k (restarts after an escape draw fresh numbers)
  auto origin = [&](uint32_t vertex, V3& o, V3& d) {
    const Philox r = rnd(vertex, 0u);
    o = v3(cam.pos[0], cam.pos[1], cam.pos[2]);
    if (prm.origin == kOriginPoint) {
      d = uniform_sphere(unit01(r.v[0]), unit01(r.v[1]));
      return;
    }
    const uint64_t pix = path / cam.spp;
    const uint32_t px = (uint32_t)(pix % cam.width), py = (uint32_t)(pix / cam.width);
    const float th = tanf(0.5f * cam.fov_y), aspect = (float)cam.width / (float)cam.height;
    const float sx = (2.0f * (((float)px + unit01(r.v[0])) / (float)cam.width) - 1.0f) * th * aspect;
    const float sy = (1.0f - 2.0f * (((float)py + unit01(r.v[1])) / (float)cam.height)) * th;
    const V3 f = v3(cam.fwd[0], cam.fwd[1], cam.fwd[2]), up = v3(cam.up[0], cam.up[1], cam.up[2]);
    const V3 right = cross(f, up);
    d = normalize(f + right * sx + up * sy);
  };
  auto hit_vertex = [&](V3 o, V3 d, PathVertex& x) {
    float t;
    const int32_t pi = trace(prims, np, o, d, kEps, 1e30f, t);
    x.valid = pi >= 0;
    if (!x.valid) return;
    const Prim q = load_prim(prims, (uint32_t)pi);
    x.p = o + d * t;
    x.wo = d * -1.0f;
    V3 n = prim_normal(q, x.p);
    x.n = dot(n, x.wo) < 0.0f ? n * -1.0f : n;
    x.prim = pi;
  };
  // density, per solid angle at x, of reaching point y of emitter q by NEE
  auto nee_pdf = [&](const Prim& q, V3 x, V3 y, V3 ny) {
    const V3 dxy = y - x;
    const float d2 = dot(dxy, dxy);
    const float cy = fabsf(dot(ny, normalize(dxy)));
    return cy > 0.0f ? d2 / (cy * prim_area(q) * (float)n_emit) : 0.0f;
  };

  V3 o, d;
  origin(0u, o, d);
  PathVertex cur;
  hit_vertex(o, d, cur);
  for (uint32_t attempt = 1; !cur.valid && attempt < 64; ++attempt) {
    origin(attempt << 16, o, d);
    hit_vertex(o, d, cur);
  }
  for (uint32_t i = 1; i <= V; ++i) {
    const uint64_t idx = (uint64_t)(i - 1) * n_paths + path;
    // x_i (a path that cannot reach the scene at all leaves NaN records)
    const float nan = __builtin_nanf("");
    const Prim q = cur.valid ? load_prim(prims, (uint32_t)cur.prim) : Prim{};
    out.px[idx] = cur.valid ? cur.p.x : nan;
    out.py[idx] = cur.valid ? cur.p.y : nan;
    out.pz[idx] = cur.valid ? cur.p.z : nan;
    out.nx[idx] = cur.valid ? cur.n.x : nan;
    out.ny[idx] = cur.valid ? cur.n.y : nan;
    out.nz[idx] = cur.valid ? cur.n.z : nan;
    out.ox[idx] = cur.valid ? cur.wo.x : nan;
    out.oy[idx] = cur.valid ? cur.wo.y : nan;
    out.oz[idx] = cur.valid ? cur.wo.z : nan;
    out.rough[idx] = cur.valid ? q.rough : nan;
    V3 le = v3(0.0f, 0.0f, 0.0f), tp = v3(0.0f, 0.0f, 0.0f);
    PathVertex nxt;
    nxt.valid = false;
    if (cur.valid) {
      if (prm.mode == kPathsLo) le = q.emit;
      const V3 f = q.albedo * kInvPi;  // Lambertian BSDF
      if (prm.mode == kPathsLoe && n_emit > 0) {
        // next-event estimation: a uniformly chosen emitter, a uniform point on it
        const Philox r = rnd(i, 2u);
        uint32_t pick = (uint32_t)(((uint64_t)r.v[0] * n_emit) >> 32), k = 0, e = 0;
        for (; k < np; ++k)
          if (emissive(load_prim(prims, k)) && e++ == pick) break;
        const Prim L = load_prim(prims, k);
        V3 y, ny;
        if (L.kind == kPrimSphere) {
          ny = uniform_sphere(unit01(r.v[1]), unit01(r.v[2]));
          y = L.p + ny * L.u.x;
        } else {
          y = L.p + L.u * (2.0f * unit01(r.v[1]) - 1.0f) + L.v * (2.0f * unit01(r.v[2]) - 1.0f);
          ny = prim_normal(L, y);
        }
        const V3 dxy = y - cur.p;
        const float dist = sqrtf(dot(dxy, dxy));
        const V3 w = dxy * (1.0f / dist);
        const float cx = dot(cur.n, w);
        float t_occ;
        if (cx > 0.0f && dist > 2.0f * kEps && trace(prims, np, cur.p, w, kEps, dist * (1.0f - 1e-4f), t_occ) < 0) {
          const float p_nee = nee_pdf(L, cur.p, y, ny);
          const float p_bsdf = cx * kInvPi;
          if (p_nee > 0.0f) {
            const float wn = p_nee / (p_nee + p_bsdf);
            const float g = wn * cx / p_nee;
            le = le + v3(f.x * L.emit.x, f.y * L.emit.y, f.z * L.emit.z) * g;
          }
        }
      }
      // the scattering event: cosine-weighted, so f cos / p = albedo
      const Philox r = rnd(i, 1u);
      const V3 wi = cosine_dir(cur.n, unit01(r.v[0]), unit01(r.v[1]));
      hit_vertex(cur.p, wi, nxt);
      if (nxt.valid) {
        tp = q.albedo;
        const Prim qn = load_prim(prims, (uint32_t)nxt.prim);
        if (prm.mode == kPathsLoe && emissive(qn)) {
          // emission reached by the scattering event, balance-weighted
          const float p_bsdf = dot(cur.n, wi) * kInvPi;
          const float p_nee = nee_pdf(qn, cur.p, nxt.p, prim_normal(qn, nxt.p));
          const float wb = p_bsdf / (p_bsdf + p_nee);
          le = le + v3(tp.x * qn.emit.x, tp.y * qn.emit.y, tp.z * qn.emit.z) * wb;
        }
      }
    }
    out.t_r[idx] = tp.x;
    out.t_g[idx] = tp.y;
    out.t_b[idx] = tp.z;
    out.le_r[idx] = le.x;
    out.le_g[idx] = le.y;
    out.le_b[idx] = le.z;
    const Prim qn = nxt.valid ? load_prim(prims, (uint32_t)nxt.prim) : Prim{};
    out.qx[idx] = nxt.valid ? nxt.p.x : nan;
    out.qy[idx] = nxt.valid ? nxt.p.y : nan;
    out.qz[idx] = nxt.valid ? nxt.p.z : nan;
    out.qnx[idx] = nxt.valid ? nxt.n.x : nan;
    out.qny[idx] = nxt.valid ? nxt.n.y : nan;
    out.qnz[idx] = nxt.valid ? nxt.n.z : nan;
    out.qox[idx] = nxt.valid ? nxt.wo.x : nan;
    out.qoy[idx] = nxt.valid ? nxt.wo.y : nan;
    out.qoz[idx] = nxt.valid ? nxt.wo.z : nan;
    out.qrough[idx] = nxt.valid ? qn.rough : nan;
    if (i == V) break;
    if (nxt.valid) {
      cur = nxt;
    } else {
      // escaped: restart from the origin with fresh numbers
      cur.valid = false;
      for (uint32_t attempt = 0; !cur.valid && attempt < 64; ++attempt) {
        origin((i << 8) | (attempt << 16) | 1u, o, d);
        hit_vertex(o, d, cur);
      }
    }
  }
}

hipError_t launch_sample_paths(const PathPrim* prims, uint32_t np, const PathCamera& cam, const PathParams& prm,
                               uint64_t n_paths, const PathOut& out, hipStream_t s) {
  if (n_paths == 0) return hipSuccess;
  const uint64_t blocks = (n_paths + 255) / 256;
  k_sample_paths<<<(unsigned)blocks, 256, 0, s>>>(prims, np, cam, prm, n_paths, out);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint64_t n, uint32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_philox<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ctr, key, n, out);
  return hipGetLastError();
}

}  // namespace psf

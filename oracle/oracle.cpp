// FP64 CPU oracle of the differentiable face render.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
// baseline leg of the benchmark load this library.  It shares no code with the
// HIP path: it has its own counter-based generator, its own brute-force
// intersection (every triangle, no acceleration structure), its own shading
// and its own derivatives (forward-mode dual numbers, not a hand-written
// adjoint).
//
// What it computes (Dib et al. 2021, "Practical Face Reconstruction via
// Differentiable Ray Tracing"):
//   * pixel colours p^S = F(chi), a Monte-Carlo estimate of the rendering
//     equation with direct light only and shadows from shadow rays
//     (Sec. 3.3 "Shadows approximation", Sec. 4 Eq. energy);
//   * the Cook-Torrance BRDF of Appendix A (Eq. brdf, brdf_diffuse,
//     brdf_spec, brdf_d, halfVector, brdf_g, brdf_g1, brdf_g1_a, brdf_g1_chi,
//     brdf_f);
//   * the derivative of the estimate with every discrete decision held fixed
//     (the "interior" gradient that back-propagation through a ray tracer
//     gives, Sec. 4), and the primary-visibility boundary term of edge
//     sampling (Sec. 4 "Edge Sampling").
// Readings of points the paper leaves open (sampling, normals, epsilons,
// half vector, Fresnel exponent, D normalisation) are listed where they are
// used.
//
// All scene inputs are FP32 arrays, promoted exactly to FP64.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <thread>
#include <utility>
#include <vector>

extern "C" {

// Mirrors the ctypes structure in oracle/__init__.py.
struct OrScene {
  int32_t n_verts, n_tris, n_lights, width, height, spp;
  const float* verts;      // [N*3] world-space positions
  const int32_t* tris;     // [F*3]
  const float* diffuse;    // [N*3]
  const float* specular;   // [N*3]
  const float* roughness;  // [N]
  const float* light_p0;   // [L*3]
  const float* light_e1;   // [L*3]
  const float* light_e2;   // [L*3]
  const float* light_rad;  // [L*3]
  const int32_t* light_shape;  // [L] 0 parallelogram, 1 triangle, 2 at infinity (direction p0)
  const float* cam_R;      // [9] camera-to-world, row-major
  const float* cam_T;      // [3]
  float fov_y;
  int32_t brdf_variant;    // 0 = as printed, 1 = normalised D + Schlick^5
  int32_t components;      // bit 0 diffuse, bit 1 specular
  int32_t pad_;
  uint64_t seed;
  uint32_t step;
  uint32_t pad2_;
  // reflectance maps (tex_size > 0): per-corner texture coordinates and
  // M x M maps, read at the interpolated coordinates of the shading point
  const float* uv;         // [F*3*2] (u, v) of each triangle corner
  const float* tex_c;      // [M*M*3] diffuse
  const float* tex_s;      // [M*M*3] specular
  const float* tex_r;      // [M*M] roughness
  int32_t tex_size;        // M (0: per-vertex reflectance)
  int32_t pad3_;
  // spherical-harmonics lighting (sh_bands B > 0): coefficients L_lm of the
  // distant radiance, [B*B][3] (index l(l+1)+m, RGB inner)
  const float* sh;
  int32_t sh_bands;
  int32_t pad4_;
};

}  // extern "C"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kShadowTmin = 1e-4;   // shadow-ray start offset (reading)
constexpr double kFlagEps = 1e-6;      // decision-ambiguity band (world units)
constexpr double kRoughMin = 1e-3, kRoughMax = 1.0;
// Film offset (pixels) of the boundary term's two side rays from the edge point.
constexpr double kEdgeSide = 1e-2;
constexpr double kMissFar = 1e4;       // length of a primary-ray segment that hits nothing

// Flag bits.
constexpr uint8_t FLAG_EDGE = 1;    // ray passes within kFlagEps of a triangle boundary
constexpr uint8_t FLAG_TIE = 2;     // two hits within kFlagEps in t
constexpr uint8_t FLAG_TRANGE = 4;  // a crossing within kFlagEps of the segment ends
constexpr uint8_t FLAG_COSO = 8;    // |n_s . o| < kFlagEps
constexpr uint8_t FLAG_COSL = 16;   // |n_s . l| or |n_j . l| < kFlagEps
constexpr uint8_t FLAG_G1 = 32;     // a G1 argument within kFlagEps of its 1.6 branch point

// Visibility codes of one (sample, light) pair.
constexpr uint8_t VIS_OCCLUDED = 0, VIS_VISIBLE = 1, VIS_CULLED = 2, VIS_NONE = 3;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// -> 64-bit multiplies, with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
struct Rand4 { uint32_t x[4]; };

Rand4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key) {
  uint32_t k0 = (uint32_t)(key & 0xffffffffu), k1 = (uint32_t)(key >> 32);
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Rand4{{x0, x1, x2, x3}};
}

// 24 high bits -> [0,1): exact in both FP32 and FP64.
inline double unit24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

// Counter layout: (pixel = y*W + x, sample, purpose, step); purpose 0 is the
// pixel jitter, 1 + j the point on light j; edge samples use purpose
// 0x80000000 (edge pick) and 0x80000001 + j (light j), with pixel = sample id.
constexpr uint32_t PURPOSE_JITTER = 0u;
constexpr uint32_t PURPOSE_EDGE = 0x80000000u;

// ---------------------------------------------------------------------------
// Forward-mode dual numbers: value + K directional derivatives.
// ---------------------------------------------------------------------------
template <int K>
struct Dual {
  double v;
  double d[K];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: implicit constant
  static Dual seed(double x, int k) { Dual r(x); r.d[k] = 1.0; return r; }
};

template <int K> Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v + b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int K> Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v - b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int K> Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r; r.v = -a.v; for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
template <int K> Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v * b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int K> Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v / b.v; const double ib = 1.0 / b.v;
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib; return r; }
template <int K> Dual<K> operator+(const Dual<K>& a, double b) { Dual<K> r = a; r.v += b; return r; }
template <int K> Dual<K> operator+(double a, const Dual<K>& b) { return b + a; }
template <int K> Dual<K> operator-(const Dual<K>& a, double b) { Dual<K> r = a; r.v -= b; return r; }
template <int K> Dual<K> operator-(double a, const Dual<K>& b) { return (-b) + a; }
template <int K> Dual<K> operator*(const Dual<K>& a, double b) {
  Dual<K> r; r.v = a.v * b; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b; return r; }
template <int K> Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K> Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> Dual<K> sqrt(const Dual<K>& a) {
  Dual<K> r; r.v = std::sqrt(a.v); const double g = 0.5 / r.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * g; return r; }
template <int K> Dual<K> exp(const Dual<K>& a) {
  Dual<K> r; r.v = std::exp(a.v); for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * r.v; return r; }
template <int K> Dual<K> log(const Dual<K>& a) {
  Dual<K> r; r.v = std::log(a.v); for (int k = 0; k < K; ++k) r.d[k] = a.d[k] / a.v; return r; }
// x^y for x > 0
template <int K> Dual<K> pow(const Dual<K>& x, const Dual<K>& y) { return exp(y * log(x)); }

inline double val(double x) { return x; }
template <int K> double val(const Dual<K>& x) { return x.v; }
inline double pow(double x, double y) { return std::pow(x, y); }
using std::sqrt;

template <class S>
struct Vec3 {
  S x, y, z;
  Vec3() : x(0.0), y(0.0), z(0.0) {}
  Vec3(S a, S b, S c) : x(a), y(b), z(c) {}
};
template <class S> Vec3<S> operator+(const Vec3<S>& a, const Vec3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> Vec3<S> operator-(const Vec3<S>& a, const Vec3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S, class T> Vec3<S> operator*(const Vec3<S>& a, const T& s) { return {a.x * s, a.y * s, a.z * s}; }
template <class S> S dot(const Vec3<S>& a, const Vec3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> Vec3<S> cross(const Vec3<S>& a, const Vec3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
template <class S> S norm(const Vec3<S>& a) { return sqrt(dot(a, a)); }
template <class S> Vec3<S> normalize(const Vec3<S>& a) { S n = norm(a); return {a.x / n, a.y / n, a.z / n}; }
template <class S> Vec3<S> mul3(const S R[9], const Vec3<S>& v) {  // row-major R @ v
  return {R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
          R[6] * v.x + R[7] * v.y + R[8] * v.z}; }
template <class S> Vec3<S> mul3T(const S R[9], const Vec3<S>& v) {  // R^T @ v
  return {R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z,
          R[2] * v.x + R[5] * v.y + R[8] * v.z}; }

using V3 = Vec3<double>;

inline V3 load3(const float* p, int i) { return V3(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

// ---------------------------------------------------------------------------
// Vertex normals: area-weighted sum of incident face normals, normalised.
// (The paper only names "the normal at vertex v_i", Sec. 3.2.)
// ---------------------------------------------------------------------------
template <class S>
Vec3<S> face_cross(const Vec3<S>& a, const Vec3<S>& b, const Vec3<S>& c) { return cross(b - a, c - a); }

std::vector<V3> vertex_normals(const OrScene& sc) {
  std::vector<V3> acc(sc.n_verts);
  for (int f = 0; f < sc.n_tris; ++f) {
    const int i0 = sc.tris[3 * f], i1 = sc.tris[3 * f + 1], i2 = sc.tris[3 * f + 2];
    V3 n = face_cross(load3(sc.verts, i0), load3(sc.verts, i1), load3(sc.verts, i2));
    acc[i0] = acc[i0] + n; acc[i1] = acc[i1] + n; acc[i2] = acc[i2] + n;
  }
  for (auto& n : acc) n = normalize(n);
  return acc;
}

// ---------------------------------------------------------------------------
// Brute-force ray casting with decision flags.
// ---------------------------------------------------------------------------
struct TriGeo { V3 a, b, c, centre; double radius; };

std::vector<TriGeo> tri_geometry(const OrScene& sc) {
  std::vector<TriGeo> g(sc.n_tris);
  for (int f = 0; f < sc.n_tris; ++f) {
    TriGeo& t = g[f];
    t.a = load3(sc.verts, sc.tris[3 * f]);
    t.b = load3(sc.verts, sc.tris[3 * f + 1]);
    t.c = load3(sc.verts, sc.tris[3 * f + 2]);
    t.centre = (t.a + t.b + t.c) * (1.0 / 3.0);
    t.radius = std::max({norm(t.a - t.centre), norm(t.b - t.centre), norm(t.c - t.centre)});
  }
  return g;
}

// Distance between segments [p1,q1] and [p2,q2]: minimise |p1 + s d1 - p2 - t d2|
// over s, t in [0,1] (closed form of the 2x2 normal equations, then clamping).
double segment_distance(const V3& p1, const V3& q1, const V3& p2, const V3& q2) {
  const V3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
  const double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  double s, t;
  if (a <= 0.0 && e <= 0.0) return norm(r);
  if (a <= 0.0) {
    s = 0.0; t = std::clamp(f / e, 0.0, 1.0);
  } else {
    const double c = dot(d1, r);
    if (e <= 0.0) {
      t = 0.0; s = std::clamp(-c / a, 0.0, 1.0);
    } else {
      const double b = dot(d1, d2), den = a * e - b * b;
      s = den > 0.0 ? std::clamp((b * f - c * e) / den, 0.0, 1.0) : 0.0;
      t = (b * s + f) / e;
      if (t < 0.0) { t = 0.0; s = std::clamp(-c / a, 0.0, 1.0); }
      else if (t > 1.0) { t = 1.0; s = std::clamp((b - c) / a, 0.0, 1.0); }
    }
  }
  return norm((p1 + d1 * s) - (p2 + d2 * t));
}

// Moller-Trumbore solve of o + t d = a + u (b - a) + v (c - a); det == 0 -> no solution.
struct Crossing { bool ok; double t, u, v; };
Crossing cross_plane(const V3& o, const V3& d, const TriGeo& g) {
  const V3 e1 = g.b - g.a, e2 = g.c - g.a;
  const V3 p = cross(d, e2);
  const double det = dot(e1, p);
  if (det == 0.0) return {false, 0, 0, 0};
  const double inv = 1.0 / det;
  const V3 s = o - g.a;
  const double u = dot(s, p) * inv;
  const V3 q = cross(s, e1);
  const double v = dot(d, q) * inv;
  const double t = dot(e2, q) * inv;
  return {true, t, u, v};
}

inline bool inside(const Crossing& c) { return c.ok && c.u >= 0.0 && c.v >= 0.0 && c.u + c.v <= 1.0; }

bool near_boundary(const V3& o, const V3& d, double t0, double t1, const TriGeo& g) {
  const V3 p = o + d * t0, q = o + d * t1;
  return segment_distance(p, q, g.a, g.b) < kFlagEps || segment_distance(p, q, g.b, g.c) < kFlagEps ||
         segment_distance(p, q, g.c, g.a) < kFlagEps;
}

// Conservative reject: can the segment [t0,t1] come within `slack` of the triangle?
bool may_touch(const V3& o, const V3& d, double t0, double t1, const TriGeo& g, double slack) {
  const double tc = std::clamp(dot(g.centre - o, d), t0, t1);
  const V3 p = o + d * tc;
  return norm(p - g.centre) <= g.radius + slack;
}

struct HitResult { int id; double t, u, v; uint8_t flags; };

// Closest hit along o + t d, t > 0; ties in t go to the lowest triangle id.
HitResult closest_hit(const std::vector<TriGeo>& tg, const V3& o, const V3& d) {
  struct Cand { int id; Crossing c; };
  std::vector<Cand> cand;
  for (int f = 0; f < (int)tg.size(); ++f) {
    if (!may_touch(o, d, 0.0, kMissFar, tg[f], 1e-5)) continue;
    cand.push_back({f, cross_plane(o, d, tg[f])});
  }
  HitResult h{-1, kMissFar, 0, 0, 0};
  for (const Cand& c : cand)
    if (inside(c.c) && c.c.t > 0.0 && (c.c.t < h.t || (c.c.t == h.t && c.id < h.id)))
      h = {c.id, c.c.t, c.c.u, c.c.v, 0};
  const double tend = (h.id >= 0 ? h.t : kMissFar) + kFlagEps;
  for (const Cand& c : cand) {
    if (near_boundary(o, d, 0.0, tend, tg[c.id])) h.flags |= FLAG_EDGE;
    if (h.id >= 0 && c.id != h.id && inside(c.c) && c.c.t > 0.0 && std::fabs(c.c.t - h.t) < kFlagEps)
      h.flags |= FLAG_TIE;
  }
  return h;
}

// Is any triangle other than `exclude` crossed strictly inside (tmin, tmax)?
bool occluded(const std::vector<TriGeo>& tg, const V3& o, const V3& d, double tmin, double tmax,
              int exclude, uint8_t* flags) {
  bool occ = false;
  for (int f = 0; f < (int)tg.size(); ++f) {
    if (f == exclude) continue;
    if (!may_touch(o, d, tmin, tmax, tg[f], 1e-5)) continue;
    const Crossing c = cross_plane(o, d, tg[f]);
    if (inside(c) && c.t > tmin && c.t < tmax) occ = true;
    if (near_boundary(o, d, tmin, tmax, tg[f])) *flags |= FLAG_EDGE;
    if (inside(c) && (std::fabs(c.t - tmin) < kFlagEps || std::fabs(c.t - tmax) < kFlagEps))
      *flags |= FLAG_TRANGE;
  }
  return occ;
}

// ---------------------------------------------------------------------------
// Camera and light sampling.
// ---------------------------------------------------------------------------
struct CamConst { double tan_half, aspect; int W, H; };

CamConst cam_const(const OrScene& sc) {
  return {std::tan(0.5 * (double)sc.fov_y), (double)sc.width / (double)sc.height, sc.width, sc.height};
}

// Film point (fx, fy) in pixel units -> camera-space direction (unnormalised).
V3 film_dir(const CamConst& cc, double fx, double fy) {
  return V3((2.0 * fx / cc.W - 1.0) * cc.tan_half * cc.aspect, (1.0 - 2.0 * fy / cc.H) * cc.tan_half, -1.0);
}

// Point on light j from two uniforms: parallelogram p0 + u0 e1 + u1 e2;
// triangle p0 + sqrt(u0)(1-u1) e1 + sqrt(u0) u1 e2 (uniform area density).
// A light at infinity (shape 2) has no point: the weights go unused.
inline void light_weights(int shape, double u0, double u1, double* w1, double* w2) {
  if (shape == 1) { const double su = std::sqrt(u0); *w1 = su * (1.0 - u1); *w2 = su * u1; }
  else { *w1 = u0; *w2 = u1; }
}

// ---------------------------------------------------------------------------
// Shading: everything downstream of the decisions, templated so that the
// same code gives values (S = double) and derivatives (S = Dual<K>).
// ---------------------------------------------------------------------------
template <class S>
struct SampleParams {     // what one camera sample depends on
  Vec3<S> v[3], n[3], c[3], s[3];
  S r[3];
  S R[9];
  Vec3<S> T;
  // reflectance maps (M > 0): corner coordinates, the maps, and offsets added
  // to the looked-up values (zero; seeded to differentiate w.r.t. the texels)
  double uv[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  const float* tc = nullptr;
  const float* ts = nullptr;
  const float* tr = nullptr;
  int M = 0;
  Vec3<S> dc{S(0.0), S(0.0), S(0.0)}, ds{S(0.0), S(0.0), S(0.0)};
  S dr = S(0.0);
};

// Bilinear footprint of texture coordinates (u, v) on an M x M map: texel
// (i, j) is centred at ((i + 1/2) / M, (j + 1/2) / M) and stored at j M + i;
// addressing clamps to the border texels.  Returns the four texel indices and
// weights (a weight may repeat a clamped index).
template <class S>
void tex_footprint(const S& u, const S& v, int M, int idx[4], S w[4]) {
  const S x = u * double(M) - 0.5, y = v * double(M) - 0.5;
  const double x0 = std::floor(val(x)), y0 = std::floor(val(y));
  const S fx = x - x0, fy = y - y0;
  auto cl = [M](double t) { return (int)std::min(std::max(t, 0.0), (double)(M - 1)); };
  const int i0 = cl(x0), i1 = cl(x0 + 1.0), j0 = cl(y0), j1 = cl(y0 + 1.0);
  idx[0] = j0 * M + i0; idx[1] = j0 * M + i1; idx[2] = j1 * M + i0; idx[3] = j1 * M + i1;
  w[0] = (S(1.0) - fx) * (S(1.0) - fy);
  w[1] = fx * (S(1.0) - fy);
  w[2] = (S(1.0) - fx) * fy;
  w[3] = fx * fy;
}

template <class S>
struct LightParams { Vec3<S> p0, e1, e2, rad; int shape; };

template <class S>
struct Frame { Vec3<S> x, ns, wo, c, s; S r; };

// Shading frame of a camera sample through film point (fx, fy) that hits the
// (fixed) triangle of `p`: barycentrics recomputed as smooth functions of the
// triangle, the ray origin and direction.
template <class S>
Frame<S> shading_frame(const SampleParams<S>& p, const CamConst& cc, double fx, double fy) {
  const V3 dc = film_dir(cc, fx, fy);
  const Vec3<S> dcs(S(dc.x), S(dc.y), S(dc.z));
  const Vec3<S> d = normalize(mul3(p.R, dcs));
  const Vec3<S>& o = p.T;
  const Vec3<S> e1 = p.v[1] - p.v[0], e2 = p.v[2] - p.v[0];
  const Vec3<S> pv = cross(d, e2);
  const S det = dot(e1, pv);
  const Vec3<S> sv = o - p.v[0];
  const S b1 = dot(sv, pv) / det;
  const Vec3<S> qv = cross(sv, e1);
  const S b2 = dot(d, qv) / det;
  const S b0 = S(1.0) - b1 - b2;
  Frame<S> f;
  f.x = p.v[0] * b0 + p.v[1] * b1 + p.v[2] * b2;
  f.ns = normalize(p.n[0] * b0 + p.n[1] * b1 + p.n[2] * b2);
  f.wo = Vec3<S>(-d.x, -d.y, -d.z);
  S r;
  if (p.M > 0) {
    // reflectance maps read at the interpolated corner coordinates
    const S u = b0 * p.uv[0][0] + b1 * p.uv[1][0] + b2 * p.uv[2][0];
    const S v = b0 * p.uv[0][1] + b1 * p.uv[1][1] + b2 * p.uv[2][1];
    int idx[4];
    S w[4];
    tex_footprint(u, v, p.M, idx, w);
    f.c = p.dc;
    f.s = p.ds;
    r = p.dr;
    for (int q = 0; q < 4; ++q) {
      const int t = idx[q];
      f.c = f.c + Vec3<S>(w[q] * (double)p.tc[3 * t], w[q] * (double)p.tc[3 * t + 1], w[q] * (double)p.tc[3 * t + 2]);
      f.s = f.s + Vec3<S>(w[q] * (double)p.ts[3 * t], w[q] * (double)p.ts[3 * t + 1], w[q] * (double)p.ts[3 * t + 2]);
      r = r + w[q] * (double)p.tr[t];
    }
  } else {
    f.c = p.c[0] * b0 + p.c[1] * b1 + p.c[2] * b2;
    f.s = p.s[0] * b0 + p.s[1] * b1 + p.s[2] * b2;
    r = p.r[0] * b0 + p.r[1] * b1 + p.r[2] * b2;
  }
  if (val(r) < kRoughMin) r = S(kRoughMin);      // clamp: the gradient passes only inside
  if (val(r) > kRoughMax) r = S(kRoughMax);
  f.r = r;
  return f;
}

// Barycentrics of the camera sample through (fx, fy) on the triangle of `p`
// (the same solve as in shading_frame, values only).
void bary_of(const SampleParams<double>& p, const CamConst& cc, double fx, double fy, double b[3]) {
  const V3 d = normalize(mul3(p.R, film_dir(cc, fx, fy)));
  const V3 e1 = p.v[1] - p.v[0], e2 = p.v[2] - p.v[0];
  const V3 pv = cross(d, e2);
  const double det = dot(e1, pv);
  const V3 sv = p.T - p.v[0];
  b[1] = dot(sv, pv) / det;
  b[2] = dot(d, cross(sv, e1)) / det;
  b[0] = 1.0 - b[1] - b[2];
}

// Walter et al.'s rational approximation of the Smith G1 for a Beckmann-like
// lobe, with a = 1 / (r tan(acos(n.v))) = n.v / (r sqrt(1 - (n.v)^2)).
template <class S>
S smith_g1(const S& nv, const S& hv, const S& r, uint8_t* flags) {
  if (!(val(hv) / val(nv) > 0.0)) return S(0.0);
  const double s2 = 1.0 - val(nv) * val(nv);
  if (s2 <= 0.0) return S(1.0);
  const S a = nv / (r * sqrt(S(1.0) - nv * nv));
  if (flags && std::fabs(val(a) - 1.6) < kFlagEps * 1.6) *flags |= FLAG_G1;
  if (val(a) < 1.6) return (3.535 * a + 2.181 * a * a) / (1.0 + 2.276 * a + 2.577 * a * a);
  return S(1.0);
}

// Cook-Torrance f_r = c/pi + D G F / (4 (o.n)(l.n)) (Appendix A).
//   variant 0 (as printed): D = (2/r + 2)/(2 pi) (n.h)^(2/r - 2), F = s + (1-s)(1 - o.h)
//   variant 1: D = 1/(pi r) (n.h)^(2/r - 2) (unit projected integral),
//              F = s + (1-s)(1 - o.h)^5 (Schlick)
// The half vector is normalize(l + o): the printed denominator |l . o| is read
// as the norm of l + o, which the text's "normalized halfway vector" requires.
template <class S>
Vec3<S> brdf(const Frame<S>& f, const Vec3<S>& l, const S& cos_o, const S& cos_l, int variant,
             int components, uint8_t* flags) {
  Vec3<S> out(S(0.0), S(0.0), S(0.0));
  if (components & 1) out = f.c * (1.0 / kPi);
  if (components & 2) {
    const Vec3<S> h = normalize(l + f.wo);
    const S nh = dot(f.ns, h);
    const S ex = 2.0 / f.r - 2.0;
    const S nd = variant == 1 ? 1.0 / (kPi * f.r) : (2.0 / f.r + 2.0) / (2.0 * kPi);
    const S D = nd * pow(nh, ex);
    const S oh = dot(f.wo, h), lh = dot(l, h);
    const S G = smith_g1(cos_o, oh, f.r, flags) * smith_g1(cos_l, lh, f.r, flags);
    const S om = 1.0 - oh;
    S fw = om;
    if (variant == 1) fw = om * om * om * om * om;
    const S spec = D * G / (4.0 * cos_o * cos_l);
    const Vec3<S> F(f.s.x + (1.0 - f.s.x) * fw, f.s.y + (1.0 - f.s.y) * fw, f.s.z + (1.0 - f.s.z) * fw);
    out = out + F * spec;
  }
  return out;
}

// Contribution of light j to one camera sample (radiance, before the 1/S
// weight): V L_j * f_r * (n_s . l) * (-n_j . l) A_j / |q - x|^2.
// With A_j (-n_j . l) = -kappa (e1 x e2) . l, kappa = 1 (parallelogram) or
// 1/2 (triangle).  `vis` is the frozen decision; culled pairs give zero.
// A light at infinity (the environment-map pixels of Sec. 6, "Environment
// Map vs. Light Stage") shines along l = p0 / |p0| with L_j the irradiance
// it delivers to a surface facing it (radiance times the pixel's solid
// angle): V L_j * f_r * (n_s . l).
template <class S>
Vec3<S> light_contribution(const Frame<S>& f, const LightParams<S>& L, double w1, double w2, uint8_t vis,
                           int variant, int components, uint8_t* flags) {
  if (vis != VIS_VISIBLE) return Vec3<S>(S(0.0), S(0.0), S(0.0));
  if (L.shape == 2) {
    const Vec3<S> l = normalize(L.p0);
    const S cos_s = dot(f.ns, l);
    const S cos_o = dot(f.ns, f.wo);
    const Vec3<S> fr = brdf(f, l, cos_o, cos_s, variant, components, flags);
    return Vec3<S>(L.rad.x * fr.x * cos_s, L.rad.y * fr.y * cos_s, L.rad.z * fr.z * cos_s);
  }
  const Vec3<S> q = L.p0 + L.e1 * S(w1) + L.e2 * S(w2);
  const Vec3<S> dq = q - f.x;
  const S dist2 = dot(dq, dq);
  const Vec3<S> l = dq * (1.0 / sqrt(dist2));
  const S cos_s = dot(f.ns, l);
  const S cos_o = dot(f.ns, f.wo);
  const double kappa = L.shape == 1 ? 0.5 : 1.0;
  const S cosA = -(kappa * dot(cross(L.e1, L.e2), l));
  const Vec3<S> fr = brdf(f, l, cos_o, cos_s, variant, components, flags);
  const S g = cos_s * cosA / dist2;
  return Vec3<S>(L.rad.x * fr.x * g, L.rad.y * fr.y * g, L.rad.z * fr.z * g);
}

// ---------------------------------------------------------------------------
// Spherical-harmonics lighting (Sec. 6, "Spherical Harmonics (SH) vs. Light
// Stage": distant light as a B-band SH expansion, no visibility).  Reading:
// the SH light reaches the diffuse term only, as the irradiance
// E(n) = sum_l A_l sum_m L_lm Y_lm(n), with A_l the coefficients of the
// clamped cosine max(0, n . w) (Ramamoorthi and Hanrahan 2001); a sample
// receives (c / pi) E(n_s).
// ---------------------------------------------------------------------------
constexpr int kMaxShBands = 11;

// Normalisation of the real SH: sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
double sh_norm(int l, int m) {
  double r = 1.0;
  for (int k = l - m + 1; k <= l + m; ++k) r /= k;
  return std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * r);
}

// A_l: pi, 2 pi / 3, 0 for odd l > 1, and for even l
// 2 pi (-1)^(l/2 - 1) / ((l + 2)(l - 1)) * l! / (2^l ((l/2)!)^2).
double sh_cosine_coeff(int l) {
  if (l == 0) return kPi;
  if (l == 1) return 2.0 * kPi / 3.0;
  if (l % 2) return 0.0;
  double c = 1.0;                      // l! / (2^l ((l/2)!)^2) = C(l, l/2) / 2^l
  for (int k = 1; k <= l / 2; ++k) c *= (double)(l / 2 + k) / (double)k;
  c /= std::ldexp(1.0, l);
  const double sg = ((l / 2 - 1) % 2) ? -1.0 : 1.0;
  return 2.0 * kPi * sg / ((l + 2.0) * (l - 1.0)) * c;
}

// Real SH up to band B-1 at the unit vector n (z the polar axis), Y[l(l+1)+m]:
// Y_l0 = K_l0 P_l(z); Y_l,+m = sqrt2 K_lm Pbar_lm(z) Re (x + i y)^m;
// Y_l,-m = sqrt2 K_lm Pbar_lm(z) Im (x + i y)^m, where Pbar_lm is the
// associated Legendre function (Condon-Shortley phase) divided by
// (1 - z^2)^(m/2), from its three-term recurrence in l.
template <class S>
void sh_basis(int B, const Vec3<S>& n, S* Y) {
  S cr[kMaxShBands], ci[kMaxShBands];
  cr[0] = S(1.0); ci[0] = S(0.0);
  for (int m = 1; m < B; ++m) {
    cr[m] = n.x * cr[m - 1] - n.y * ci[m - 1];
    ci[m] = n.x * ci[m - 1] + n.y * cr[m - 1];
  }
  for (int m = 0; m < B; ++m) {
    double pmm = 1.0;                  // (-1)^m (2m - 1)!!
    for (int k = 1; k <= m; ++k) pmm *= -(2.0 * k - 1.0);
    auto put = [&](int l, const S& p) {
      if (m == 0) { Y[l * (l + 1)] = p * sh_norm(l, 0); return; }
      const double k = std::sqrt(2.0) * sh_norm(l, m);
      Y[l * (l + 1) + m] = p * cr[m] * k;
      Y[l * (l + 1) - m] = p * ci[m] * k;
    };
    S pa = S(pmm);
    put(m, pa);
    if (m + 1 >= B) continue;
    S pb = n.z * ((2.0 * m + 1.0) * pmm);
    put(m + 1, pb);
    for (int l = m + 2; l < B; ++l) {
      const S pc = (n.z * pb * (2.0 * l - 1.0) - pa * (double)(l + m - 1)) / (double)(l - m);
      put(l, pc);
      pa = pb; pb = pc;
    }
  }
}

// The SH light's contribution to a sample: (c / pi) E(n_s), diffuse only.
template <class S>
Vec3<S> sh_contribution(const Frame<S>& f, const float* sh, int B, int components) {
  if (B <= 0 || !(components & 1)) return Vec3<S>(S(0.0), S(0.0), S(0.0));
  S Y[kMaxShBands * kMaxShBands];
  sh_basis(B, f.ns, Y);
  S e[3] = {S(0.0), S(0.0), S(0.0)};
  for (int l = 0; l < B; ++l) {
    const double a = sh_cosine_coeff(l);
    if (a == 0.0) continue;
    for (int m = -l; m <= l; ++m) {
      const int i = l * (l + 1) + m;
      for (int ch = 0; ch < 3; ++ch) e[ch] = e[ch] + Y[i] * (a * (double)sh[3 * i + ch]);
    }
  }
  return Vec3<S>(f.c.x * e[0] * (1.0 / kPi), f.c.y * e[1] * (1.0 / kPi), f.c.z * e[2] * (1.0 / kPi));
}

// ---------------------------------------------------------------------------
// Scene access helpers.
// ---------------------------------------------------------------------------
struct Prepared {
  const OrScene* sc;
  CamConst cc;
  std::vector<V3> normals;
  std::vector<TriGeo> tg;
  double R[9];
  V3 T;
};

Prepared prepare(const OrScene* sc) {
  Prepared p;
  p.sc = sc;
  p.cc = cam_const(*sc);
  p.normals = vertex_normals(*sc);
  p.tg = tri_geometry(*sc);
  for (int i = 0; i < 9; ++i) p.R[i] = sc->cam_R[i];
  p.T = V3(sc->cam_T[0], sc->cam_T[1], sc->cam_T[2]);
  return p;
}

SampleParams<double> sample_params_d(const Prepared& P, int tri) {
  const OrScene& sc = *P.sc;
  SampleParams<double> sp;
  for (int k = 0; k < 3; ++k) {
    const int vi = sc.tris[3 * tri + k];
    sp.v[k] = load3(sc.verts, vi);
    sp.n[k] = P.normals[vi];
    sp.c[k] = load3(sc.diffuse, vi);
    sp.s[k] = load3(sc.specular, vi);
    sp.r[k] = sc.roughness[vi];
  }
  for (int i = 0; i < 9; ++i) sp.R[i] = P.R[i];
  sp.T = P.T;
  if (sc.tex_size > 0) {
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 2; ++a) sp.uv[k][a] = sc.uv[6 * tri + 2 * k + a];
    sp.tc = sc.tex_c; sp.ts = sc.tex_s; sp.tr = sc.tex_r; sp.M = sc.tex_size;
  }
  return sp;
}

LightParams<double> light_params_d(const OrScene& sc, int j) {
  return {load3(sc.light_p0, j), load3(sc.light_e1, j), load3(sc.light_e2, j), load3(sc.light_rad, j),
          sc.light_shape[j]};
}

// Decision pass of one light for a shading frame (FP64): cull tests, then the
// shadow ray from x towards q over t in (1e-4, |q - x|), excluding the hit
// triangle.  A light at infinity: the one cosine test, then the ray along
// p0 / |p0| over t in (1e-4, 1e4) (the scene lies well within 1e4).
uint8_t light_decision(const Prepared& P, const Frame<double>& f, int j, double w1, double w2, int hit,
                       uint8_t* flags) {
  const OrScene& sc = *P.sc;
  const LightParams<double> L = light_params_d(sc, j);
  if (L.shape == 2) {
    const V3 l = normalize(L.p0);
    const double cs = dot(f.ns, l);
    if (std::fabs(cs) < kFlagEps) *flags |= FLAG_COSL;
    if (cs <= 0.0) return VIS_CULLED;
    return occluded(P.tg, f.x, l, kShadowTmin, kMissFar, hit, flags) ? VIS_OCCLUDED : VIS_VISIBLE;
  }
  const V3 q = L.p0 + L.e1 * w1 + L.e2 * w2;
  const V3 dq = q - f.x;
  const double dist = norm(dq);
  const V3 l = dq * (1.0 / dist);
  const double cs = dot(f.ns, l);
  const double cl = -dot(normalize(cross(L.e1, L.e2)), l);
  if (std::fabs(cs) < kFlagEps || std::fabs(cl) < kFlagEps) *flags |= FLAG_COSL;
  if (cs <= 0.0 || cl <= 0.0) return VIS_CULLED;
  const bool occ = occluded(P.tg, f.x, l, kShadowTmin, dist, hit, flags);
  return occ ? VIS_OCCLUDED : VIS_VISIBLE;
}

template <class Fn>
void parallel_for(int n, int nthreads, Fn fn) {
  if (nthreads <= 1 || n < 2) { for (int i = 0; i < n; ++i) fn(i, 0); return; }
  nthreads = std::min(nthreads, n);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&, t]() { for (int i = t; i < n; i += nthreads) fn(i, t); });
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// Gradient slots of one (sample, light) evaluation.
// ---------------------------------------------------------------------------
constexpr int SLOT_V = 0, SLOT_N = 9, SLOT_C = 18, SLOT_S = 27, SLOT_R = 36;
constexpr int SLOT_LP0 = 39, SLOT_LE1 = 42, SLOT_LE2 = 45, SLOT_LRAD = 48;
constexpr int SLOT_CR = 51, SLOT_CT = 60, NSLOT = 63;
using D63 = Dual<NSLOT>;

Vec3<D63> seed3(const V3& v, int slot) {
  return Vec3<D63>(D63::seed(v.x, slot), D63::seed(v.y, slot + 1), D63::seed(v.z, slot + 2));
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

// Philox outputs for n counters (c0,c1,c2,c3) = ctr[4*i..4*i+3].
void oracle_philox(uint64_t key, int64_t n, const uint32_t* ctr, uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) {
    Rand4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = r.x[k];
  }
}

void oracle_vertex_normals(const OrScene* sc, double* out) {
  std::vector<V3> n = vertex_normals(*sc);
  for (int i = 0; i < sc->n_verts; ++i) { out[3 * i] = n[i].x; out[3 * i + 1] = n[i].y; out[3 * i + 2] = n[i].z; }
}

// Vector-Jacobian product of the vertex normals: g_v += (dn/dv)^T g_n, by
// forward-mode duals over each vertex's one-ring.
void oracle_normals_vjp(const OrScene* sc, const double* g_n, double* g_v) {
  using D3 = Dual<3>;
  const int N = sc->n_verts, F = sc->n_tris;
  std::vector<std::vector<int>> faces(N);
  for (int f = 0; f < F; ++f) for (int k = 0; k < 3; ++k) faces[sc->tris[3 * f + k]].push_back(f);
  for (int i = 0; i < N; ++i) {
    std::vector<int> ring;
    for (int f : faces[i]) for (int k = 0; k < 3; ++k) ring.push_back(sc->tris[3 * f + k]);
    std::sort(ring.begin(), ring.end());
    ring.erase(std::unique(ring.begin(), ring.end()), ring.end());
    const V3 gni(g_n[3 * i], g_n[3 * i + 1], g_n[3 * i + 2]);
    for (int m : ring) {
      auto pos = [&](int vi) {
        const V3 p = load3(sc->verts, vi);
        if (vi == m) return Vec3<D3>(D3::seed(p.x, 0), D3::seed(p.y, 1), D3::seed(p.z, 2));
        return Vec3<D3>(D3(p.x), D3(p.y), D3(p.z));
      };
      Vec3<D3> acc(D3(0.0), D3(0.0), D3(0.0));
      for (int f : faces[i])
        acc = acc + face_cross(pos(sc->tris[3 * f]), pos(sc->tris[3 * f + 1]), pos(sc->tris[3 * f + 2]));
      const Vec3<D3> n = normalize(acc);
      for (int k = 0; k < 3; ++k) g_v[3 * m + k] += gni.x * n.x.d[k] + gni.y * n.y.d[k] + gni.z * n.z.d[k];
    }
  }
}

// Forward render of a pixel subset (all pixels when pix == nullptr).
//   force_hit [n_pix*S]   : -2 = decide here, else the hit id (-1 = miss) to use
//   force_vis [n_pix*S*L] : 0xFF = decide here, else a VIS_* code to use
// Outputs (nullable): rgb [n_pix*3], hit [n_pix*S], pflag [n_pix*S],
// vis [n_pix*S*L], sflag [n_pix*S*L].
int oracle_render(const OrScene* sc, int32_t n_pix, const int32_t* pix, const int32_t* force_hit,
                  const uint8_t* force_vis, double* out_rgb, int32_t* out_hit, uint8_t* out_pflag,
                  uint8_t* out_vis, uint8_t* out_sflag, int32_t nthreads) {
  const Prepared P = prepare(sc);
  const int S = sc->spp, L = sc->n_lights, W = sc->width;
  if (!pix) n_pix = sc->width * sc->height;
  parallel_for(n_pix, nthreads, [&](int ip, int) {
    const int pid = pix ? pix[ip] : ip;
    const int px = pid % W, py = pid / W;
    double acc[3] = {0, 0, 0};
    for (int s = 0; s < S; ++s) {
      const size_t rs = (size_t)ip * S + s;
      const Rand4 rj = philox4x32_10((uint32_t)pid, (uint32_t)s, PURPOSE_JITTER, sc->step, sc->seed);
      const double fx = px + unit24(rj.x[0]), fy = py + unit24(rj.x[1]);
      const V3 d = normalize(mul3(P.R, film_dir(P.cc, fx, fy)));
      HitResult h = closest_hit(P.tg, P.T, d);
      if (force_hit && force_hit[rs] != -2) h.id = force_hit[rs];
      uint8_t pflag = h.flags;
      if (out_hit) out_hit[rs] = h.id;
      uint8_t* vis_row = out_vis ? out_vis + rs * L : nullptr;
      uint8_t* sf_row = out_sflag ? out_sflag + rs * L : nullptr;
      if (h.id < 0) {
        if (out_pflag) out_pflag[rs] = pflag;
        for (int j = 0; j < L; ++j) { if (vis_row) vis_row[j] = VIS_NONE; if (sf_row) sf_row[j] = 0; }
        continue;
      }
      const SampleParams<double> sp = sample_params_d(P, h.id);
      const Frame<double> fr = shading_frame(sp, P.cc, fx, fy);
      const double cos_o = dot(fr.ns, fr.wo);
      if (std::fabs(cos_o) < kFlagEps) pflag |= FLAG_COSO;
      if (out_pflag) out_pflag[rs] = pflag;
      for (int j = 0; j < L; ++j) {
        const Rand4 rl = philox4x32_10((uint32_t)pid, (uint32_t)s, 1u + (uint32_t)j, sc->step, sc->seed);
        double w1, w2;
        light_weights(sc->light_shape[j], unit24(rl.x[0]), unit24(rl.x[1]), &w1, &w2);
        uint8_t sflag = 0;
        uint8_t vis = VIS_NONE;
        if (cos_o > 0.0) vis = light_decision(P, fr, j, w1, w2, h.id, &sflag);
        if (force_vis && force_vis[rs * L + j] != 0xFF) vis = force_vis[rs * L + j];
        const Vec3<double> c = light_contribution(fr, light_params_d(*sc, j), w1, w2, vis, sc->brdf_variant,
                                                  sc->components, &sflag);
        acc[0] += c.x; acc[1] += c.y; acc[2] += c.z;
        if (vis_row) vis_row[j] = vis;
        if (sf_row) sf_row[j] = sflag;
      }
      if (cos_o > 0.0) {
        const Vec3<double> c = sh_contribution(fr, sc->sh, sc->sh_bands, sc->components);
        acc[0] += c.x; acc[1] += c.y; acc[2] += c.z;
      }
    }
    if (out_rgb) for (int k = 0; k < 3; ++k) out_rgb[3 * ip + k] = acc[k] / S;
  });
  return 0;
}

// Interior gradient of sum_p dEdp[p] . rgb[p] over a pixel subset, with the
// decisions (hit [n_pix*S], vis [n_pix*S*L], as produced by oracle_render and
// possibly replaced) held fixed.  All outputs are accumulated (+=):
//   g_verts [N*3] (direct path only), g_normals [N*3], g_diffuse [N*3],
//   g_specular [N*3], g_rough [N], g_light [L*9] (p0, e1, e2), g_rad [L*3],
//   g_cam [12] (R row-major, then T).
// abs_terms != 0 accumulates the magnitude of every (sample, light) term
// instead of the term: the condition measure of each sum (test tolerance
// only; not a gradient).  g_sh [B*B*3] (nullable): the SH coefficients'
// gradient (the SH term is linear in them: (g . c / pi) A_l Y_lm(n_s)).
int oracle_grad(const OrScene* sc, int32_t n_pix, const int32_t* pix, const int32_t* hit, const uint8_t* vis,
                const double* dEdp, double* g_verts, double* g_normals, double* g_diffuse, double* g_specular,
                double* g_rough, double* g_light, double* g_rad, double* g_cam, double* g_tex_c, double* g_tex_s,
                double* g_tex_r, int32_t nthreads, int32_t abs_terms, double* g_sh) {
  const Prepared P = prepare(sc);
  const int S = sc->spp, L = sc->n_lights, W = sc->width, N = sc->n_verts;
  if (!pix) n_pix = sc->width * sc->height;
  nthreads = std::max(1, std::min<int>(nthreads, n_pix));
  const int M = sc->tex_size, MM = M > 0 ? M * M : 0;
  const int B = sc->sh_bands;
  struct Acc { std::vector<double> v, n, c, s, r, l, rad, cam, tc, ts, tr, sh; };
  std::vector<Acc> accs(nthreads);
  for (auto& a : accs) {
    a.v.assign(3 * N, 0); a.n.assign(3 * N, 0); a.c.assign(3 * N, 0); a.s.assign(3 * N, 0);
    a.r.assign(N, 0); a.l.assign(9 * L, 0); a.rad.assign(3 * L, 0); a.cam.assign(12, 0);
    a.tc.assign(3 * (size_t)MM, 0); a.ts.assign(3 * (size_t)MM, 0); a.tr.assign(MM, 0);
    a.sh.assign(3 * (size_t)B * B, 0);
  }
  parallel_for(n_pix, nthreads, [&](int ip, int tid) {
    Acc& A = accs[tid];
    const int pid = pix ? pix[ip] : ip;
    const int px = pid % W, py = pid / W;
    const double g[3] = {dEdp[3 * ip] / S, dEdp[3 * ip + 1] / S, dEdp[3 * ip + 2] / S};
    if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) return;
    for (int s = 0; s < S; ++s) {
      const size_t rs = (size_t)ip * S + s;
      const int tri = hit[rs];
      if (tri < 0) continue;
      const Rand4 rj = philox4x32_10((uint32_t)pid, (uint32_t)s, PURPOSE_JITTER, sc->step, sc->seed);
      const double fx = px + unit24(rj.x[0]), fy = py + unit24(rj.x[1]);
      const SampleParams<double> spd = sample_params_d(P, tri);
      SampleParams<D63> sp;
      for (int k = 0; k < 3; ++k) {
        sp.v[k] = seed3(spd.v[k], SLOT_V + 3 * k);
        sp.n[k] = seed3(spd.n[k], SLOT_N + 3 * k);
        sp.c[k] = seed3(spd.c[k], SLOT_C + 3 * k);
        sp.s[k] = seed3(spd.s[k], SLOT_S + 3 * k);
        sp.r[k] = D63::seed(spd.r[k], SLOT_R + k);
      }
      for (int i = 0; i < 9; ++i) sp.R[i] = D63::seed(P.R[i], SLOT_CR + i);
      sp.T = seed3(P.T, SLOT_CT);
      int tidx[4] = {0, 0, 0, 0};
      double tw[4] = {0, 0, 0, 0};
      if (M > 0) {
        // with maps, the reflectance slots hold the offsets of the looked-up values
        for (int k = 0; k < 3; ++k)
          for (int a = 0; a < 2; ++a) sp.uv[k][a] = spd.uv[k][a];
        sp.tc = spd.tc; sp.ts = spd.ts; sp.tr = spd.tr; sp.M = M;
        sp.dc = seed3(V3(0.0, 0.0, 0.0), SLOT_C);
        sp.ds = seed3(V3(0.0, 0.0, 0.0), SLOT_S);
        sp.dr = D63::seed(0.0, SLOT_R);
        // footprint at the (value of the) shading point, for the texel scatter
        double b[3];
        bary_of(spd, P.cc, fx, fy, b);
        const double u = b[0] * spd.uv[0][0] + b[1] * spd.uv[1][0] + b[2] * spd.uv[2][0];
        const double v = b[0] * spd.uv[0][1] + b[1] * spd.uv[1][1] + b[2] * spd.uv[2][1];
        tex_footprint(u, v, M, tidx, tw);
      }
      const Frame<D63> fr = shading_frame(sp, P.cc, fx, fy);
      int vid[3];
      for (int k = 0; k < 3; ++k) vid[k] = sc->tris[3 * tri + k];
      // one term (a light's or the SH light's contribution) into the sums;
      // j < 0: no light slots
      auto scatter = [&](const Vec3<D63>& c, int j) {
        double gs[NSLOT];
        for (int k = 0; k < NSLOT; ++k) gs[k] = g[0] * c.x.d[k] + g[1] * c.y.d[k] + g[2] * c.z.d[k];
        if (abs_terms)
          for (int k = 0; k < NSLOT; ++k) gs[k] = std::fabs(gs[k]);
        for (int k = 0; k < 3; ++k)
          for (int a = 0; a < 3; ++a) {
            A.v[3 * vid[k] + a] += gs[SLOT_V + 3 * k + a];
            A.n[3 * vid[k] + a] += gs[SLOT_N + 3 * k + a];
          }
        if (M > 0) {
          for (int q = 0; q < 4; ++q) {
            const size_t t = (size_t)tidx[q];
            for (int a = 0; a < 3; ++a) {
              A.tc[3 * t + a] += tw[q] * gs[SLOT_C + a];
              A.ts[3 * t + a] += tw[q] * gs[SLOT_S + a];
            }
            A.tr[t] += tw[q] * gs[SLOT_R];
          }
        } else {
          for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
              A.c[3 * vid[k] + a] += gs[SLOT_C + 3 * k + a];
              A.s[3 * vid[k] + a] += gs[SLOT_S + 3 * k + a];
            }
          for (int k = 0; k < 3; ++k) A.r[vid[k]] += gs[SLOT_R + k];
        }
        if (j >= 0) {
          for (int a = 0; a < 9; ++a) A.l[9 * j + a] += gs[SLOT_LP0 + a];
          for (int a = 0; a < 3; ++a) A.rad[3 * j + a] += gs[SLOT_LRAD + a];
        }
        for (int a = 0; a < 12; ++a) A.cam[a] += gs[SLOT_CR + a];
      };
      for (int j = 0; j < L; ++j) {
        const uint8_t vs = vis[rs * L + j];
        if (vs != VIS_VISIBLE) continue;
        const Rand4 rl = philox4x32_10((uint32_t)pid, (uint32_t)s, 1u + (uint32_t)j, sc->step, sc->seed);
        double w1, w2;
        light_weights(sc->light_shape[j], unit24(rl.x[0]), unit24(rl.x[1]), &w1, &w2);
        const LightParams<double> ld = light_params_d(*sc, j);
        LightParams<D63> lp{seed3(ld.p0, SLOT_LP0), seed3(ld.e1, SLOT_LE1), seed3(ld.e2, SLOT_LE2),
                            seed3(ld.rad, SLOT_LRAD), ld.shape};
        scatter(light_contribution(fr, lp, w1, w2, vs, sc->brdf_variant, sc->components, nullptr), j);
      }
      if (B > 0 && (sc->components & 1) && val(dot(fr.ns, fr.wo)) > 0.0) {
        scatter(sh_contribution(fr, sc->sh, B, sc->components), -1);
        // the coefficients: (g . c / pi) A_l Y_lm(n_s), in values
        Vec3<double> ns(val(fr.ns.x), val(fr.ns.y), val(fr.ns.z));
        double Y[kMaxShBands * kMaxShBands];
        sh_basis(B, ns, Y);
        const double w[3] = {g[0] * val(fr.c.x) / kPi, g[1] * val(fr.c.y) / kPi, g[2] * val(fr.c.z) / kPi};
        for (int l = 0; l < B; ++l)
          for (int m = -l; m <= l; ++m) {
            const int i = l * (l + 1) + m;
            for (int ch = 0; ch < 3; ++ch) {
              const double t = w[ch] * sh_cosine_coeff(l) * Y[i];
              A.sh[3 * i + ch] += abs_terms ? std::fabs(t) : t;
            }
          }
      }
    }
  });
  auto add = [](double* dst, const std::vector<double>& src) { if (dst) for (size_t i = 0; i < src.size(); ++i) dst[i] += src[i]; };
  for (const Acc& a : accs) {
    add(g_verts, a.v); add(g_normals, a.n); add(g_diffuse, a.c); add(g_specular, a.s);
    add(g_rough, a.r); add(g_light, a.l); add(g_rad, a.rad); add(g_cam, a.cam);
    add(g_tex_c, a.tc); add(g_tex_s, a.ts); add(g_tex_r, a.tr); add(g_sh, a.sh);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Primary-visibility boundary term (edge sampling, Sec. 4).
//
// Silhouette edges: interior edges whose two faces differ in facing w.r.t. the
// camera centre, plus every edge with one face.  Facing of a face is the sign
// of ((v1 - v0) x (v2 - v0)) . (T - v0), evaluated in FP64 in that order.
// Each silhouette edge gets probability proportional to its length on the
// film (pixel units); a sample picks the edge by the running sum, a point
// y = a + u (b - a) on it, and shades two rays through y -/+ eps m, with m the
// unit film normal perp(b - a) and eps = 1e-2 pixel.  The pick is stratified:
// sample k draws its position in the running sum from [k, k+1)/n_samples.
// The estimate
//     sum_k  (ltot / n_samples) (f_minus - f_plus) . dEdp[pixel(y)] (m . dy/dtheta)
// is added to the two edge vertices and the camera.  dy/dtheta is the film
// velocity of the 3D edge point that projects to y (perspective-correct
// parameter held fixed).
//   edge_out [n_sel*4] per selected sample: edge id, pixel id (-1 outside),
//   hit id of the minus ray, hit id of the plus ray;  flag_out [n_sel].
//   sel: sample ids to evaluate (nullptr = all).  dEdp is the full [H*W*3].
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct EdgeList { std::vector<int> a, b, f0, f1; };

EdgeList build_edges(const OrScene& sc) {
  std::map<std::pair<int, int>, std::vector<int>> m;
  for (int f = 0; f < sc.n_tris; ++f)
    for (int k = 0; k < 3; ++k) {
      int i = sc.tris[3 * f + k], j = sc.tris[3 * f + (k + 1) % 3];
      if (i > j) std::swap(i, j);
      m[{i, j}].push_back(f);
    }
  EdgeList e;
  for (auto& kv : m) {
    e.a.push_back(kv.first.first); e.b.push_back(kv.first.second);
    e.f0.push_back(kv.second[0]); e.f1.push_back(kv.second.size() > 1 ? kv.second[1] : -1);
  }
  return e;
}

template <class S>
struct FilmPt { S x, y, depth; };

// Pixel coordinates of world point X: camera frame R^T (X - T), pinhole.
template <class S>
FilmPt<S> project(const Vec3<S>& X, const S R[9], const Vec3<S>& T, const CamConst& cc) {
  const Vec3<S> pc = mul3T(R, X - T);
  const S z = -pc.z;
  FilmPt<S> f;
  f.x = (pc.x / z / (cc.tan_half * cc.aspect) + 1.0) * (0.5 * cc.W);
  f.y = (1.0 - pc.y / z / cc.tan_half) * (0.5 * cc.H);
  f.depth = z;
  return f;
}

}  // namespace

extern "C" {

int oracle_edge_grad(const OrScene* sc, int32_t n_samples, int32_t n_sel, const int32_t* sel,
                     const double* dEdp, double* g_verts, double* g_cam, int32_t* edge_out, uint8_t* flag_out,
                     double* ltot_out, int32_t nthreads, int32_t abs_terms) {
  // abs_terms != 0: accumulate, per element, (|f-| + |f+|) . |dEdp| times the
  // magnitude of the velocity instead: the size of the two shaded values whose
  // difference each term carries (the condition of that difference; a test
  // tolerance, not a gradient)
  const Prepared P = prepare(sc);
  const OrScene& s = *sc;
  const EdgeList E = build_edges(s);
  const int nE = (int)E.a.size(), W = s.width, H = s.height, L = s.n_lights;
  // Facing of each face.
  std::vector<uint8_t> front(s.n_tris);
  for (int f = 0; f < s.n_tris; ++f) {
    const V3 v0 = load3(s.verts, s.tris[3 * f]), v1 = load3(s.verts, s.tris[3 * f + 1]),
             v2 = load3(s.verts, s.tris[3 * f + 2]);
    const V3 n = cross(v1 - v0, v2 - v0);
    const V3 w = P.T - v0;
    front[f] = (n.x * w.x + n.y * w.y + n.z * w.z) > 0.0;
  }
  // Film length of each silhouette edge and the running sum.
  std::vector<double> len(nE, 0.0), cdf(nE + 1, 0.0);
  for (int e = 0; e < nE; ++e) {
    const bool sil = E.f1[e] < 0 || front[E.f0[e]] != front[E.f1[e]];
    if (!sil) continue;
    const FilmPt<double> pa = project(load3(s.verts, E.a[e]), P.R, P.T, P.cc);
    const FilmPt<double> pb = project(load3(s.verts, E.b[e]), P.R, P.T, P.cc);
    if (pa.depth <= 0.0 || pb.depth <= 0.0) continue;
    len[e] = std::hypot(pb.x - pa.x, pb.y - pa.y);
  }
  for (int e = 0; e < nE; ++e) cdf[e + 1] = cdf[e] + len[e];
  const double ltot = cdf[nE];
  if (ltot_out) *ltot_out = ltot;
  if (ltot <= 0.0 || n_samples <= 0) return 0;
  if (!sel) n_sel = n_samples;
  nthreads = std::max(1, std::min<int>(nthreads, n_sel));
  std::vector<std::vector<double>> gv(nthreads, std::vector<double>(3 * s.n_verts, 0.0));
  std::vector<std::vector<double>> gc(nthreads, std::vector<double>(12, 0.0));
  parallel_for(n_sel, nthreads, [&](int is, int tid) {
    const int k = sel ? sel[is] : is;
    const Rand4 re = philox4x32_10((uint32_t)k, 0u, PURPOSE_EDGE, s.step, s.seed);
    // stratified pick over the running sum: sample k covers [k, k+1)/n_samples
    const double target = ((double)k + unit24(re.x[0])) / (double)n_samples * ltot;
    const double u = unit24(re.x[1]);
    // first e with cdf[e+1] > target
    const int e = (int)(std::upper_bound(cdf.begin() + 1, cdf.end(), target) - (cdf.begin() + 1));
    uint8_t flag = 0;
    if (std::fabs(target - cdf[e]) < 1e-9 * ltot || std::fabs(target - cdf[e + 1]) < 1e-9 * ltot) flag |= FLAG_TIE;
    const V3 A = load3(s.verts, E.a[e]), B = load3(s.verts, E.b[e]);
    const FilmPt<double> pa = project(A, P.R, P.T, P.cc), pb = project(B, P.R, P.T, P.cc);
    const double yx = pa.x + u * (pb.x - pa.x), yy = pa.y + u * (pb.y - pa.y);
    const double lx = pb.x - pa.x, ly = pb.y - pa.y, ll = std::hypot(lx, ly);
    const double mx = -ly / ll, my = lx / ll;
    const int pxi = (int)std::floor(yx), pyi = (int)std::floor(yy);
    const bool in_img = pxi >= 0 && pxi < W && pyi >= 0 && pyi < H;
    const int pid = in_img ? pyi * W + pxi : -1;
    int hits[2] = {-1, -1};
    double fpm[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (in_img) {
      for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? -1.0 : 1.0;
        const double fx = yx + sg * kEdgeSide * mx, fy = yy + sg * kEdgeSide * my;
        const V3 d = normalize(mul3(P.R, film_dir(P.cc, fx, fy)));
        const HitResult h = closest_hit(P.tg, P.T, d);
        flag |= h.flags;
        hits[side] = h.id;
        if (h.id < 0) continue;
        const Frame<double> fr = shading_frame(sample_params_d(P, h.id), P.cc, fx, fy);
        const double cos_o = dot(fr.ns, fr.wo);
        if (std::fabs(cos_o) < kFlagEps) flag |= FLAG_COSO;
        if (cos_o <= 0.0) continue;
        for (int j = 0; j < L; ++j) {
          const Rand4 rl = philox4x32_10((uint32_t)k, 0u, PURPOSE_EDGE + 1u + (uint32_t)j, s.step, s.seed);
          double w1, w2;
          light_weights(s.light_shape[j], unit24(rl.x[0]), unit24(rl.x[1]), &w1, &w2);
          const uint8_t vis = light_decision(P, fr, j, w1, w2, h.id, &flag);
          const Vec3<double> c = light_contribution(fr, light_params_d(s, j), w1, w2, vis, s.brdf_variant,
                                                    s.components, &flag);
          fpm[side][0] += c.x; fpm[side][1] += c.y; fpm[side][2] += c.z;
        }
        const Vec3<double> c = sh_contribution(fr, s.sh, s.sh_bands, s.components);
        fpm[side][0] += c.x; fpm[side][1] += c.y; fpm[side][2] += c.z;
      }
    }
    if (edge_out) { edge_out[4 * is] = e; edge_out[4 * is + 1] = pid; edge_out[4 * is + 2] = hits[0]; edge_out[4 * is + 3] = hits[1]; }
    if (flag_out) flag_out[is] = flag;
    if (!in_img) return;
    double dlt = 0.0;
    for (int c = 0; c < 3; ++c)
      dlt += abs_terms ? (std::fabs(fpm[0][c]) + std::fabs(fpm[1][c])) * std::fabs(dEdp[3 * pid + c])
                       : (fpm[0][c] - fpm[1][c]) * dEdp[3 * pid + c];
    const double wgt = ltot / n_samples * dlt;
    const auto T = [abs_terms](double x) { return abs_terms ? std::fabs(x) : x; };
    if (wgt == 0.0) return;
    // Film velocity of the edge point: X(w) = (1-w) A + w B, w perspective-correct.
    const double w = (u / pb.depth) / ((1.0 - u) / pa.depth + u / pb.depth);
    using D18 = Dual<18>;
    Vec3<D18> Ad(D18::seed(A.x, 0), D18::seed(A.y, 1), D18::seed(A.z, 2));
    Vec3<D18> Bd(D18::seed(B.x, 3), D18::seed(B.y, 4), D18::seed(B.z, 5));
    D18 Rd[9];
    for (int i = 0; i < 9; ++i) Rd[i] = D18::seed(P.R[i], 6 + i);
    Vec3<D18> Td(D18::seed(P.T.x, 15), D18::seed(P.T.y, 16), D18::seed(P.T.z, 17));
    const Vec3<D18> X = Ad * D18(1.0 - w) + Bd * D18(w);
    const FilmPt<D18> y = project(X, Rd, Td, P.cc);
    double vn[18];
    for (int i = 0; i < 18; ++i) vn[i] = mx * y.x.d[i] + my * y.y.d[i];
    std::vector<double>& G = gv[tid];
    for (int a = 0; a < 3; ++a) { G[3 * E.a[e] + a] += T(wgt * vn[a]); G[3 * E.b[e] + a] += T(wgt * vn[3 + a]); }
    for (int i = 0; i < 12; ++i) gc[tid][i] += T(wgt * vn[6 + i]);
  });
  for (int t = 0; t < nthreads; ++t) {
    if (g_verts) for (int i = 0; i < 3 * s.n_verts; ++i) g_verts[i] += gv[t][i];
    if (g_cam) for (int i = 0; i < 12; ++i) g_cam[i] += gc[t][i];
  }
  return 0;
}

// Number of unique edges (for sizing).
int32_t oracle_edge_count(const OrScene* sc) { return (int32_t)build_edges(*sc).a.size(); }

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Shadow-edge (secondary visibility) boundary term, Sec. 4 "Edge Sampling":
// the gradient must include the visibility discontinuities, and those of the
// shadow rays (Sec. 3.3) lie on the lights.  Light j seen from the shading
// point x contributes I = kappa^-1 int int h(w1, w2) V(x, y) dw1 dw2 over the
// light's parameter domain (unit square; triangle: w1 + w2 <= 1), y = p0 +
// w1 e1 + w2 e2, h the render's per-sample value of the light at y (pdf 1/A,
// A = kappa |e1 x e2|).  On the line w2 = v the visibility V is piecewise
// constant in w1, so d/dtheta of the inner integral is the interior term plus
// sum_k h(w1_k) J_k dw1_k/dtheta over the jumps w1_k, J_k = V(w1_k-) -
// V(w1_k+) (Leibniz).  A jump is where an occluder edge (a, b) crosses the
// wedge {x + tau (y(w1, v) - x)}, the edge's faces (other than the shading
// point's own triangle, which never occludes) all lie on one side as seen
// from x, and no other triangle blocks x -> y(w1_k).  Its position solves
// D(w1) = det[a - x, b - x, y(w1, v) - x] = 0, linear in w1; implicit
// differentiation gives dw1/dtheta = -(dD/dtheta) / (dD/dw1).
// ---------------------------------------------------------------------------
constexpr uint32_t PURPOSE_SHADOW_EDGE = 0xC0000000u;

// Index in [0, n) from 32 random bits, floor(r n / 2^32), and its exact
// probability (the number of r mapping to i, over 2^32).
inline int64_t pick_index(uint32_t r, int64_t n) { return (int64_t)(((uint64_t)r * (uint64_t)n) >> 32); }
inline double pick_prob(int64_t i, int64_t n) {
  const auto cdiv = [n](uint64_t x) { return (x + (uint64_t)n - 1) / (uint64_t)n; };
  return (double)(cdiv((uint64_t)(i + 1) << 32) - cdiv((uint64_t)i << 32)) * (1.0 / 4294967296.0);
}

// Neighbour of triangle f across its edge k (tris[3f+k], tris[3f+(k+1)%3]), -1 if none.
std::vector<int> face_neighbours(const OrScene& sc) {
  const EdgeList E = build_edges(sc);
  std::map<std::pair<int, int>, int> id;
  for (size_t e = 0; e < E.a.size(); ++e) id[{E.a[e], E.b[e]}] = (int)e;
  std::vector<int> nb(3 * (size_t)sc.n_tris, -1);
  for (int f = 0; f < sc.n_tris; ++f)
    for (int k = 0; k < 3; ++k) {
      int i = sc.tris[3 * f + k], j = sc.tris[3 * f + (k + 1) % 3];
      if (i > j) std::swap(i, j);
      const int e = id[{i, j}];
      nb[3 * f + k] = E.f0[e] == f ? E.f1[e] : E.f0[e];
    }
  return nb;
}

// Occlusion of o + t d, t in (tmin, tmax), by any triangle but ex[0..2].
bool occluded3(const std::vector<TriGeo>& tg, const V3& o, const V3& d, double tmin, double tmax, const int ex[3],
               uint8_t* flags) {
  bool occ = false;
  for (int f = 0; f < (int)tg.size(); ++f) {
    if (f == ex[0] || f == ex[1] || f == ex[2]) continue;
    if (!may_touch(o, d, tmin, tmax, tg[f], 1e-5)) continue;
    const Crossing c = cross_plane(o, d, tg[f]);
    if (inside(c) && c.t > tmin && c.t < tmax) occ = true;
    if (near_boundary(o, d, tmin, tmax, tg[f])) *flags |= FLAG_EDGE;
    if (inside(c) && (std::fabs(c.t - tmin) < kFlagEps || std::fabs(c.t - tmax) < kFlagEps)) *flags |= FLAG_TRANGE;
  }
  return occ;
}

// One jump of V along the line w2 = v of light j, seen from x.
struct ShadowJump { int a, b, f0, f1; int J; double w1; };

// Jumps of V(x, y(w1, v)), w1 in (0, l), l = 1 (parallelogram) or 1 - v
// (triangle), with `self` the shading point's triangle (never an occluder),
// in increasing w1 (ties by edge).  Every near-ambiguous decision sets a bit
// of *flags.
std::vector<ShadowJump> shadow_jumps(const OrScene& sc, const std::vector<TriGeo>& tg, const std::vector<int>& nb,
                                     const V3& x, int self, int j, double v, uint8_t* flags) {
  std::vector<ShadowJump> out;
  const LightParams<double> L = light_params_d(sc, j);
  if (L.shape == 2) return out;
  const double ell = L.shape == 1 ? 1.0 - v : 1.0;
  const V3 y0 = L.p0 + L.e2 * v, y1 = y0 + L.e1 * ell;
  const V3 Nw = cross(y0 - x, y1 - x);
  const double nN = norm(Nw);
  if (!(nN > 0.0)) return out;
  const auto sgn = [&](int vi) { return dot(Nw, load3(sc.verts, vi) - x); };
  const auto near_plane = [&](double s) { return std::fabs(s) < kFlagEps * nN; };
  // side (+1: towards larger w1) of face f, whose edge (a, b) crosses the
  // plane at P: the direction from P to the face's other crossing, seen from x
  const auto side = [&](int f, int ia, int ib, const V3& P) -> int {
    int ic = -1;
    for (int k = 0; k < 3; ++k) {
      const int t = sc.tris[3 * f + k];
      if (t != ia && t != ib) ic = t;
    }
    const double sa = sgn(ia), sb = sgn(ib), sc_ = sgn(ic);
    if (near_plane(sc_)) *flags |= FLAG_EDGE;
    const V3 A = load3(sc.verts, ia), B = load3(sc.verts, ib), C = load3(sc.verts, ic);
    const bool with_a = (sc_ > 0.0) == (sa > 0.0);        // c on a's side: the other crossing is on (b, c)
    const V3 Q = with_a ? B + (C - B) * (sb / (sb - sc_)) : A + (C - A) * (sa / (sa - sc_));
    const double o = dot(cross(P - x, Q - x), Nw);
    if (std::fabs(o) < kFlagEps * norm(P - x) * norm(Q - P) * nN) *flags |= FLAG_EDGE;
    return o > 0.0 ? 1 : -1;
  };
  for (int f = 0; f < sc.n_tris; ++f)
    for (int k = 0; k < 3; ++k) {
      const int g = nb[3 * f + k];
      if (g >= 0 && g < f) continue;                      // each edge once, from its lower face
      int ia = sc.tris[3 * f + k], ib = sc.tris[3 * f + (k + 1) % 3];
      if (ia > ib) std::swap(ia, ib);
      const double sa = sgn(ia), sb = sgn(ib);
      // an end on the wedge plane is flagged once the crossing is in range
      // (below); an edge with no crossing and an end near the plane is
      // flagged when that end lies inside the wedge's range
      const V3 A = load3(sc.verts, ia), B = load3(sc.verts, ib);
      if (near_plane(sa) || near_plane(sb)) {
        // E - x ~ alpha (y0 - x) + beta (y1 - x) (least squares): in front of
        // x and within the line's span, with a margin
        const V3 E = near_plane(sa) ? A : B, u0 = y0 - x, u1 = y1 - x, e = E - x;
        const double g00 = dot(u0, u0), g01 = dot(u0, u1), g11 = dot(u1, u1);
        const double r0 = dot(u0, e), r1 = dot(u1, e), det = g00 * g11 - g01 * g01;
        const double al = (g11 * r0 - g01 * r1) / det, be = (g00 * r1 - g01 * r0) / det;
        const double tot = al + be;
        if (tot > 0.0 && be > -0.01 * tot && be < 1.01 * tot && tot < 1.01) *flags |= FLAG_EDGE;
      }
      if (!((sa > 0.0 && sb < 0.0) || (sa < 0.0 && sb > 0.0))) continue;
      const V3 P = A + (B - A) * (sa / (sa - sb));
      const V3 ax = A - x, bx = B - x, nab = cross(ax, bx);
      const double D1 = dot(nab, L.e1);
      if (D1 == 0.0) continue;
      const double w1 = -dot(nab, y0 - x) / D1;
      // an edge nearly parallel to the line: the jump's position (and its
      // derivative, ~1/D1) is ill-conditioned; flagged when in range
      const bool ill = std::fabs(D1) < 1e-3 * norm(nab) * norm(L.e1);
      const V3 yk = L.p0 + L.e1 * w1 + L.e2 * v;
      const V3 dy = yk - x;
      const double dist = norm(dy);
      const double tau = dot(P - x, dy) / (dist * dist);
      if (!(tau > 0.0)) continue;
      const double dP = tau * dist;
      const bool in_w = w1 > 0.0 && w1 < ell, in_t = dP > kShadowTmin && tau < 1.0;
      const bool near_w = std::fabs(w1) < kFlagEps || std::fabs(w1 - ell) < kFlagEps;
      const bool near_t = std::fabs(dP - kShadowTmin) < kFlagEps || std::fabs(dist - dP) < kFlagEps;
      if (near_w || near_t) *flags |= FLAG_TRANGE;
      if (!(in_w && in_t)) continue;
      if (ill) *flags |= FLAG_EDGE;
      int faces[2] = {f, g}, n = 0, right = 0;
      for (int q = 0; q < 2; ++q) {
        if (faces[q] < 0 || faces[q] == self) continue;
        ++n;
        right += side(faces[q], ia, ib, P) > 0 ? 1 : 0;
      }
      if (n == 0 || (right != 0 && right != n)) continue;   // no face, or faces on both sides
      const int ex[3] = {f, g, self};
      const V3 l = dy * (1.0 / dist);
      if (occluded3(tg, x, l, kShadowTmin, dist, ex, flags)) continue;
      out.push_back({ia, ib, f, g, right == n ? 1 : -1, w1});
    }
  std::sort(out.begin(), out.end(), [](const ShadowJump& p, const ShadowJump& q) {
    return p.w1 < q.w1 || (p.w1 == q.w1 && (p.a < q.a || (p.a == q.a && p.b < q.b)));
  });
  return out;
}

// dw1/dtheta of a jump, theta = (a, b, x, p0, e1, e2) as 18 directional
// derivatives, from D(w1) = det[a - x, b - x, p0 + w1 e1 + v e2 - x] = 0.
using D18 = Dual<18>;
void jump_gradient(const V3& a, const V3& b, const Vec3<D18>& x, const LightParams<double>& L, double v,
                   D18* w1_out) {
  const Vec3<D18> A(D18::seed(a.x, 0), D18::seed(a.y, 1), D18::seed(a.z, 2));
  const Vec3<D18> B(D18::seed(b.x, 3), D18::seed(b.y, 4), D18::seed(b.z, 5));
  const Vec3<D18> p0(D18::seed(L.p0.x, 9), D18::seed(L.p0.y, 10), D18::seed(L.p0.z, 11));
  const Vec3<D18> e1(D18::seed(L.e1.x, 12), D18::seed(L.e1.y, 13), D18::seed(L.e1.z, 14));
  const Vec3<D18> e2(D18::seed(L.e2.x, 15), D18::seed(L.e2.y, 16), D18::seed(L.e2.z, 17));
  const Vec3<D18> nab = cross(A - x, B - x);
  *w1_out = -(dot(nab, p0 + e2 * D18(v) - x) / dot(nab, e1));
}

}  // namespace

extern "C" {

// Jumps of the visibility along the line w2 = v of light j seen from point x
// (triangle `self` excluded as an occluder): returns their count; up to cap
// of them are written as w1[k], J[k], edge[2k..2k+1] (vertex ids, lower
// first) and grad[18k..18k+17] = dw1/d(a, b, x, p0, e1, e2).  *flags gets
// the ambiguity bits.  A probe for the oracle's own pins.
int32_t oracle_shadow_jumps(const OrScene* sc, const double* xp, int32_t self, int32_t j, double v, int32_t cap,
                            double* w1, int32_t* J, int32_t* edge, double* grad, uint8_t* flags) {
  const std::vector<TriGeo> tg = tri_geometry(*sc);
  const std::vector<int> nb = face_neighbours(*sc);
  const V3 x(xp[0], xp[1], xp[2]);
  uint8_t fl = 0;
  const std::vector<ShadowJump> js = shadow_jumps(*sc, tg, nb, x, self, j, v, &fl);
  const LightParams<double> L = light_params_d(*sc, j);
  const Vec3<D18> X(D18::seed(x.x, 6), D18::seed(x.y, 7), D18::seed(x.z, 8));
  for (int k = 0; k < (int)js.size() && k < cap; ++k) {
    w1[k] = js[k].w1;
    J[k] = js[k].J;
    edge[2 * k] = js[k].a;
    edge[2 * k + 1] = js[k].b;
    if (grad) {
      D18 w;
      jump_gradient(load3(sc->verts, js[k].a), load3(sc->verts, js[k].b), X, L, v, &w);
      for (int q = 0; q < 18; ++q) grad[18 * k + q] = w.d[q];
    }
  }
  if (flags) *flags = fl;
  return (int32_t)js.size();
}

// Shadow-edge boundary term of sum_p dEdp[p] . rgb[p] (dEdp [H*W*3]) from
// n_samples line samples in groups of 64: group g draws, from Philox
// counter (g, 0, 0xC0000000, step), an 8 x 8 pixel tile uniformly over the
// tiles (word 0; edge tiles are clipped to the image) and a light uniformly
// (word 1); sample i of the group draws, from counter (i, 1, 0xC0000000,
// step), a camera sample uniformly over the tile's pixels and samples (word
// 0) and the line w2 = v (word 1, 24 bits).  Each sample contributes, per jump,
//   kappa^-1 (1/S) (dEdp . h(w1_k, v)) J_k dw1_k/dtheta / (n_samples p_cs p_j)
// with p_cs = p(tile) p(camera sample | tile) and p_j the exact marginal
// probabilities of its draws (a group's samples share their tile and light,
// so that a wave's wedges are coherent; each sample's marginal is what the
// weight uses, so the sum stays unbiased).  The shading
// point x is the camera ray's hit, a function of the hit triangle and the
// camera (Sec. 3.1), as in the render.  Accumulated (+=): g_verts [N*3],
// g_light [L*9] (p0, e1, e2), g_cam [12].  rec [n*4] = (camera sample,
// light, jumps that passed the occlusion test, sum of their lower vertex ids
// * N + upper ids mod 2^31); flag [n] the ambiguity bits (camera ray, edge
// tests, occlusion tests, cosines at the jump points).
int oracle_shadow_edge_grad(const OrScene* sc, int32_t n_samples, const double* dEdp, double* g_verts,
                            double* g_light, double* g_cam, int32_t* rec, uint8_t* flag_out, int32_t nthreads,
                            int32_t abs_terms) {
  // abs_terms != 0: accumulate the magnitude of every term instead (the
  // condition measure of each element's sum; a test tolerance, not a gradient)
  const auto T = [abs_terms](double x) { return abs_terms ? std::fabs(x) : x; };
  const Prepared P = prepare(sc);
  const OrScene& s = *sc;
  const std::vector<int> nb = face_neighbours(s);
  const int N = s.n_verts, L = s.n_lights, W = s.width, S = s.spp;
  if (n_samples <= 0) return 0;
  nthreads = std::max(1, std::min<int>(nthreads, n_samples));
  std::vector<std::vector<double>> gv(nthreads, std::vector<double>(3 * (size_t)N, 0.0)),
      gl(nthreads, std::vector<double>(9 * (size_t)std::max(L, 1), 0.0)), gc(nthreads, std::vector<double>(12, 0.0));
  const int tx = (W + 7) / 8, ty = (s.height + 7) / 8;
  parallel_for(n_samples, nthreads, [&](int i, int th) {
    // group draw (tile, light) shared by samples 64 g .. 64 g + 63, then the
    // sample's camera sample within the tile and its line
    const Rand4 rg = philox4x32_10((uint32_t)(i / 64), 0u, PURPOSE_SHADOW_EDGE, s.step, s.seed);
    const Rand4 r = philox4x32_10((uint32_t)i, 1u, PURPOSE_SHADOW_EDGE, s.step, s.seed);
    const int tile = (int)pick_index(rg.x[0], (int64_t)tx * ty);
    const int x0 = 8 * (tile % tx), y0 = 8 * (tile / tx);
    const int tw = std::min(8, W - x0), tht = std::min(8, s.height - y0);
    const int64_t n_in = (int64_t)tw * tht * S;
    const int64_t k = pick_index(r.x[0], n_in);
    const int64_t cs = ((int64_t)(y0 + (int)(k / S) / tw) * W + x0 + (int)(k / S) % tw) * S + k % S;
    const int j = L > 0 ? (int)pick_index(rg.x[1], L) : -1;
    const double v = unit24(r.x[1]);
    const double p_cs = pick_prob(tile, (int64_t)tx * ty) * pick_prob(k, n_in);
    int32_t* rr = rec ? rec + 4 * (size_t)i : nullptr;
    if (rr) { rr[0] = (int32_t)cs; rr[1] = j; rr[2] = 0; rr[3] = 0; }
    uint8_t fl = 0;
    const auto done = [&]() { if (flag_out) flag_out[i] = fl; };
    if (j < 0 || s.light_shape[j] == 2) { done(); return; }
    const int pid = (int)(cs / S), smp = (int)(cs % S);
    const int px = pid % W, py = pid / W;
    const Rand4 rj = philox4x32_10((uint32_t)pid, (uint32_t)smp, PURPOSE_JITTER, s.step, s.seed);
    const double fx = px + unit24(rj.x[0]), fy = py + unit24(rj.x[1]);
    const V3 d = normalize(mul3(P.R, film_dir(P.cc, fx, fy)));
    const HitResult h = closest_hit(P.tg, P.T, d);
    fl |= h.flags;
    if (h.id < 0) { done(); return; }
    const SampleParams<double> sp = sample_params_d(P, h.id);
    const Frame<double> fr = shading_frame(sp, P.cc, fx, fy);
    const double cos_o = dot(fr.ns, fr.wo);
    if (std::fabs(cos_o) < kFlagEps) fl |= FLAG_COSO;
    if (!(cos_o > 0.0)) { done(); return; }
    // a light wholly below the tangent plane at x (every corner lower than
    // 1e-4), or x behind the light's emitting plane (by more than 1e-3 of the
    // light's area-normal size): h = 0 on the whole line, the sample is skipped
    {
      const LightParams<double> Lc = light_params_d(s, j);
      const V3 d0 = Lc.p0 - fr.x;
      const double ca = dot(fr.ns, d0), cb = dot(fr.ns, Lc.e1), cc = dot(fr.ns, Lc.e2);
      double top = std::max({ca, ca + cb, ca + cc});
      if (Lc.shape != 1) top = std::max(top, ca + cb + cc);
      const double kap = Lc.shape == 1 ? 0.5 : 1.0;
      const V3 na = cross(Lc.e1, Lc.e2) * (-kap);
      const double side = dot(na, d0), alen = std::fabs(na.x) + std::fabs(na.y) + std::fabs(na.z);
      if (std::fabs(top + 1e-4) < 1e-6 || std::fabs(side + 1e-3 * alen) < 1e-6 * (1.0 + alen)) fl |= FLAG_COSL;
      if (top < -1e-4 || side < -1e-3 * alen) { done(); return; }
    }
    const std::vector<ShadowJump> js = shadow_jumps(s, P.tg, nb, fr.x, h.id, j, v, &fl);
    if (js.empty()) { done(); return; }
    // the shading point as a function of the hit triangle and the camera
    using D36 = Dual<36>;
    SampleParams<D36> spd;
    for (int k = 0; k < 3; ++k) {
      spd.v[k] = Vec3<D36>(D36::seed(sp.v[k].x, 3 * k), D36::seed(sp.v[k].y, 3 * k + 1), D36::seed(sp.v[k].z, 3 * k + 2));
      spd.n[k] = Vec3<D36>(D36(sp.n[k].x), D36(sp.n[k].y), D36(sp.n[k].z));
      spd.c[k] = Vec3<D36>(D36(sp.c[k].x), D36(sp.c[k].y), D36(sp.c[k].z));
      spd.s[k] = Vec3<D36>(D36(sp.s[k].x), D36(sp.s[k].y), D36(sp.s[k].z));
      spd.r[k] = D36(0.5);
    }
    for (int q = 0; q < 9; ++q) spd.R[q] = D36::seed(P.R[q], 9 + q);
    spd.T = Vec3<D36>(D36::seed(P.T.x, 18), D36::seed(P.T.y, 19), D36::seed(P.T.z, 20));
    const Vec3<D36> xd = shading_frame(spd, P.cc, fx, fy).x;
    // x's 18-slot seeds for jump_gradient carry x's own value; its slots 6..8
    // are chained below through dx/d(triangle, camera)
    const Vec3<D18> X(D18::seed(xd.x.v, 6), D18::seed(xd.y.v, 7), D18::seed(xd.z.v, 8));
    const LightParams<double> Lp = light_params_d(s, j);
    const double kinv = Lp.shape == 1 ? 2.0 : 1.0;
    const double wgt = 1.0 / ((double)n_samples * p_cs * pick_prob(j, L));
    int n_ok = 0;
    int64_t key = 0;
    for (const ShadowJump& q : js) {
      ++n_ok;
      key = (key + (int64_t)q.a * N + q.b) % 2147483648LL;
      // h at the jump: the render's value of the light sample there (cosine
      // culls included), with the ambiguity bits of its tests
      const V3 yk = Lp.p0 + Lp.e1 * q.w1 + Lp.e2 * v;
      const V3 dy = yk - fr.x;
      const V3 l = dy * (1.0 / norm(dy));
      const double cs_ = dot(fr.ns, l), cl = -dot(normalize(cross(Lp.e1, Lp.e2)), l);
      if (std::fabs(cs_) < kFlagEps || std::fabs(cl) < kFlagEps) fl |= FLAG_COSL;
      if (!(cs_ > 0.0 && cl > 0.0)) continue;
      const Vec3<double> hv = light_contribution(fr, Lp, q.w1, v, VIS_VISIBLE, s.brdf_variant, s.components, &fl);
      const double* g = dEdp + 3 * (size_t)pid;
      const double coef = wgt * kinv / S * q.J * (g[0] * hv.x + g[1] * hv.y + g[2] * hv.z);
      if (coef == 0.0) continue;
      D18 w;
      jump_gradient(load3(s.verts, q.a), load3(s.verts, q.b), X, Lp, v, &w);
      for (int c = 0; c < 3; ++c) {
        gv[th][3 * (size_t)q.a + c] += T(coef * w.d[c]);
        gv[th][3 * (size_t)q.b + c] += T(coef * w.d[3 + c]);
        gl[th][9 * (size_t)j + c] += T(coef * w.d[9 + c]);
        gl[th][9 * (size_t)j + 3 + c] += T(coef * w.d[12 + c]);
        gl[th][9 * (size_t)j + 6 + c] += T(coef * w.d[15 + c]);
      }
      // chain dw1/dx through x(triangle, camera)
      const double gx[3] = {coef * w.d[6], coef * w.d[7], coef * w.d[8]};
      const D36* xc[3] = {&xd.x, &xd.y, &xd.z};
      for (int c = 0; c < 3; ++c) {
        for (int k = 0; k < 3; ++k)
          for (int e = 0; e < 3; ++e) gv[th][3 * (size_t)s.tris[3 * h.id + k] + e] += T(gx[c] * xc[c]->d[3 * k + e]);
        for (int q2 = 0; q2 < 12; ++q2) gc[th][q2] += T(gx[c] * xc[c]->d[9 + q2]);
      }
    }
    if (rr) { rr[2] = n_ok; rr[3] = (int32_t)key; }
    done();
  });
  for (int t = 0; t < nthreads; ++t) {
    for (size_t k = 0; k < 3 * (size_t)N; ++k) g_verts[k] += gv[t][k];
    for (size_t k = 0; k < 9 * (size_t)L; ++k) g_light[k] += gl[t][k];
    for (int k = 0; k < 12; ++k) g_cam[k] += gc[t][k];
  }
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Probes of single stages, used by the oracle's own pins.
// ---------------------------------------------------------------------------
extern "C" {

// Exact probability of the index floor(r n / 2^32) == i over the 2^32
// values of r, as the shadow-edge estimator weights its draws.
double oracle_pick_prob(int64_t i, int64_t n) { return pick_prob(i, n); }

// World-space unit direction of the camera ray through film point (fx, fy).
void oracle_camera_ray(const OrScene* sc, double fx, double fy, double* out_d) {
  const Prepared P = prepare(sc);
  const V3 d = normalize(mul3(P.R, film_dir(P.cc, fx, fy)));
  out_d[0] = d.x; out_d[1] = d.y; out_d[2] = d.z;
}

// Closest hit of ray o + t d (d unit): out_i = {id, flags}, out_d = {t, u, v}.
void oracle_closest_hit(const OrScene* sc, const double* o, const double* d, int32_t* out_i, double* out_d) {
  const std::vector<TriGeo> tg = tri_geometry(*sc);
  const HitResult h = closest_hit(tg, V3(o[0], o[1], o[2]), V3(d[0], d[1], d[2]));
  out_i[0] = h.id; out_i[1] = h.flags;
  out_d[0] = h.t; out_d[1] = h.u; out_d[2] = h.v;
}

// All plane crossings of the full line o + t d, t in (-inf, inf), that fall
// inside a triangle: returns the count; ts[] receives their t (up to cap).
int32_t oracle_line_crossings(const OrScene* sc, const double* o, const double* d, double* ts, int32_t cap) {
  const std::vector<TriGeo> tg = tri_geometry(*sc);
  const V3 O(o[0], o[1], o[2]), D(d[0], d[1], d[2]);
  int32_t n = 0;
  for (const TriGeo& g : tg) {
    const Crossing c = cross_plane(O, D, g);
    if (inside(c)) { if (n < cap) ts[n] = c.t; ++n; }
  }
  return n;
}

// Occlusion of segment o + t d, t in (tmin, tmax), excluding triangle `exclude`.
int32_t oracle_occluded(const OrScene* sc, const double* o, const double* d, double tmin, double tmax,
                        int32_t exclude, uint8_t* flags) {
  const std::vector<TriGeo> tg = tri_geometry(*sc);
  uint8_t f = 0;
  const bool occ = occluded(tg, V3(o[0], o[1], o[2]), V3(d[0], d[1], d[2]), tmin, tmax, exclude, &f);
  if (flags) *flags = f;
  return occ ? 1 : 0;
}

// Cook-Torrance f_r for unit n, l, o (all pointing away from the surface) and
// reflectances c, s (RGB), roughness r (clamped as in shading).
//   out_rgb [3]; out_terms = {D, G1(o), G1(l), Fresnel weight (1 - o.h)^k}.
void oracle_brdf(int32_t variant, int32_t components, const double* n, const double* l, const double* o,
                 const double* c, const double* s, double r, double* out_rgb, double* out_terms) {
  Frame<double> f;
  f.ns = V3(n[0], n[1], n[2]);
  f.wo = V3(o[0], o[1], o[2]);
  f.c = V3(c[0], c[1], c[2]);
  f.s = V3(s[0], s[1], s[2]);
  f.r = std::min(std::max(r, kRoughMin), kRoughMax);
  const V3 L(l[0], l[1], l[2]);
  const double cos_o = dot(f.ns, f.wo), cos_l = dot(f.ns, L);
  const V3 fr = brdf(f, L, cos_o, cos_l, variant, components, nullptr);
  out_rgb[0] = fr.x; out_rgb[1] = fr.y; out_rgb[2] = fr.z;
  if (out_terms) {
    const V3 h = normalize(L + f.wo);
    const double nh = dot(f.ns, h);
    const double nd = variant == 1 ? 1.0 / (kPi * f.r) : (2.0 / f.r + 2.0) / (2.0 * kPi);
    out_terms[0] = nd * std::pow(nh, 2.0 / f.r - 2.0);
    out_terms[1] = smith_g1(cos_o, dot(f.wo, h), f.r, (uint8_t*)nullptr);
    out_terms[2] = smith_g1(cos_l, dot(L, h), f.r, (uint8_t*)nullptr);
    const double om = 1.0 - dot(f.wo, h);
    out_terms[3] = variant == 1 ? om * om * om * om * om : om;
  }
}

// G1 as a function of a directly (branch included), for the pins of Eq. brdf_g1.
double oracle_g1_of_a(double a) {
  if (a < 1.6) return (3.535 * a + 2.181 * a * a) / (1.0 + 2.276 * a + 2.577 * a * a);
  return 1.0;
}

// The real SH basis Y [B*B] at the unit vector (x, y, z), and A_l, for the
// pins of the SH lighting.
int oracle_sh_basis(int32_t B, double x, double y, double z, double* Y) {
  if (B < 1 || B > kMaxShBands) return -1;
  sh_basis(B, Vec3<double>(x, y, z), Y);
  return 0;
}

double oracle_sh_cosine_coeff(int32_t l) { return sh_cosine_coeff(l); }

}  // extern "C"

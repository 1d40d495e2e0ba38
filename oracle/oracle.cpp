// Reference oracle for the tetrahedral cone-beam projector.
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously-correct CPU
// implementation used to check the GPU library.  Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// product path never does.  It shares no code, header, table or helper with
// the GPU library.
//
// What it computes (paper, Section II-A, Eqs. 1-3): the system matrix entry
// a_ij is the length of ray j inside tetrahedron i; the forward projection is
// b_j = sum_i a_ij x_i (Eq. 2) and the backprojection is
// xhat_i = sum_j a_ij y_j (Eq. 3, with the detector index j on y).
// The ray of pixel j runs from the source point to the pixel centre
// (Algorithm 2 takes l = |R2 - R1| and lengths l (t2 - t1)).
//
// How (Sections II-C, II-D, II-E): the ray enters the convex mesh through a
// boundary face and walks from tetrahedron to face-neighbour tetrahedron
// through the face it leaves by, visiting zero-length passages too (Fig. 3).
// The paper makes the walk robust by widening faces with an escalating
// epsilon in FP64; here every decision is taken with exact arithmetic
// instead, and ties (rays through vertices, along edges, inside face planes)
// are resolved by the limit of a translated ray S + delta, P + delta with
// delta = eps U + eps^2 V, eps -> 0+, where U, V are the detector axes.  For
// the edge (p, q) the sign that decides everything is
//   E(p, q) = det[P - S, p - S, q - S]                 (level 0)
//   then det[P - S, U, p - q], then det[P - S, V, p - q] (levels 1, 2)
// taken at the first level that is non-zero.  A face (a, b, c) whose normal
// (b - a) x (c - a) points out of its tetrahedron is left by the ray when all
// three of E(a,b), E(b,c), E(c,a) are +1 and entered when all three are -1
// (because E(a,b)+E(b,c)+E(c,a) = (P-S).((b-a)x(c-a)) and the line meets the
// triangle exactly when the three agree).
//
// Arithmetic: signs are exact.  A float64 evaluation with an error bound
// decides the clear cases; otherwise the determinant is recomputed exactly
// with dyadic big integers (value = m * 2^e, m an arbitrary-size integer).
// Ray parameters t and lengths are float64; sums use Neumaier compensation.

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Exact dyadic arithmetic: sign-magnitude big integers times a power of two.
// ---------------------------------------------------------------------------
typedef std::vector<uint32_t> Mag;  // little-endian base-2^32 digits, no leading zeros

void trim(Mag& a) {
  while (!a.empty() && a.back() == 0) a.pop_back();
}

int cmp_mag(const Mag& a, const Mag& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

Mag add_mag(const Mag& a, const Mag& b) {
  Mag r(std::max(a.size(), b.size()) + 1, 0);
  uint64_t carry = 0;
  for (size_t i = 0; i < r.size(); ++i) {
    uint64_t s = carry;
    if (i < a.size()) s += a[i];
    if (i < b.size()) s += b[i];
    r[i] = (uint32_t)s;
    carry = s >> 32;
  }
  trim(r);
  return r;
}

Mag sub_mag(const Mag& a, const Mag& b) {  // requires a >= b
  Mag r(a.size(), 0);
  int64_t borrow = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    int64_t s = (int64_t)a[i] - borrow - (i < b.size() ? (int64_t)b[i] : 0);
    if (s < 0) {
      s += (int64_t)1 << 32;
      borrow = 1;
    } else {
      borrow = 0;
    }
    r[i] = (uint32_t)s;
  }
  trim(r);
  return r;
}

Mag mul_mag(const Mag& a, const Mag& b) {
  if (a.empty() || b.empty()) return Mag();
  Mag r(a.size() + b.size() + 1, 0);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      uint64_t cur = (uint64_t)a[i] * b[j] + r[i + j] + carry;
      r[i + j] = (uint32_t)cur;
      carry = cur >> 32;
    }
    size_t k = i + b.size();
    while (carry) {
      uint64_t cur = (uint64_t)r[k] + carry;
      r[k] = (uint32_t)cur;
      carry = cur >> 32;
      ++k;
    }
  }
  trim(r);
  return r;
}

Mag shl_mag(const Mag& a, int bits) {
  if (a.empty() || bits == 0) return a;
  int limbs = bits / 32, rem = bits % 32;
  Mag r(a.size() + limbs + 1, 0);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t v = (uint64_t)a[i] << rem;
    r[i + limbs] |= (uint32_t)v;
    r[i + limbs + 1] |= (uint32_t)(v >> 32);
  }
  trim(r);
  return r;
}

struct Dy {  // s * m * 2^e, s in {-1, 0, 1}
  int s = 0;
  Mag m;
  int e = 0;
};

Dy dy_from_double(double v) {
  Dy r;
  if (v == 0.0) return r;
  int ex = 0;
  double fr = std::frexp(std::fabs(v), &ex);  // |v| = fr * 2^ex, fr in [0.5, 1)
  uint64_t mant = (uint64_t)std::ldexp(fr, 53);  // exact: a 53-bit integer
  r.s = v < 0 ? -1 : 1;
  r.m = {(uint32_t)mant, (uint32_t)(mant >> 32)};
  trim(r.m);
  r.e = ex - 53;
  return r;
}

Dy dy_neg(Dy a) {
  a.s = -a.s;
  return a;
}

Dy dy_add(const Dy& a, const Dy& b) {
  if (a.s == 0) return b;
  if (b.s == 0) return a;
  int e = std::min(a.e, b.e);
  Mag am = shl_mag(a.m, a.e - e), bm = shl_mag(b.m, b.e - e);
  Dy r;
  r.e = e;
  if (a.s == b.s) {
    r.s = a.s;
    r.m = add_mag(am, bm);
    return r;
  }
  int c = cmp_mag(am, bm);
  if (c == 0) return Dy();
  if (c > 0) {
    r.s = a.s;
    r.m = sub_mag(am, bm);
  } else {
    r.s = b.s;
    r.m = sub_mag(bm, am);
  }
  return r;
}

Dy dy_sub(const Dy& a, const Dy& b) { return dy_add(a, dy_neg(b)); }

Dy dy_mul(const Dy& a, const Dy& b) {
  Dy r;
  if (a.s == 0 || b.s == 0) return r;
  r.s = a.s * b.s;
  r.m = mul_mag(a.m, b.m);
  r.e = a.e + b.e;
  return r;
}

// ---------------------------------------------------------------------------
// Sign of det[A1 - A0, B1 - B0, C1 - C0] for float32 points.
// ---------------------------------------------------------------------------
std::atomic<long long> g_exact_calls{0};

int det_sign_exact(const float* A1, const float* A0, const float* B1, const float* B0,
                   const float* C1, const float* C0) {
  g_exact_calls.fetch_add(1, std::memory_order_relaxed);
  Dy A[3], B[3], C[3];
  for (int i = 0; i < 3; ++i) {
    A[i] = dy_sub(dy_from_double(A1[i]), dy_from_double(A0[i]));
    B[i] = dy_sub(dy_from_double(B1[i]), dy_from_double(B0[i]));
    C[i] = dy_sub(dy_from_double(C1[i]), dy_from_double(C0[i]));
  }
  // det = A0 (B1 C2 - B2 C1) - A1 (B0 C2 - B2 C0) + A2 (B0 C1 - B1 C0)
  Dy m0 = dy_sub(dy_mul(B[1], C[2]), dy_mul(B[2], C[1]));
  Dy m1 = dy_sub(dy_mul(B[0], C[2]), dy_mul(B[2], C[0]));
  Dy m2 = dy_sub(dy_mul(B[0], C[1]), dy_mul(B[1], C[0]));
  Dy d = dy_add(dy_sub(dy_mul(A[0], m0), dy_mul(A[1], m1)), dy_mul(A[2], m2));
  return d.s;
}

// Float64 evaluation first.  Each of the six monomials of the determinant
// passes through at most eight roundings (three input differences, two
// products, one difference inside the 2x2 minor, two additions), so the
// computed value differs from the exact one by at most
// gamma_8 * sum|monomials| <= 9 u * perm with u = 2^-53; 16 u is used.  Inputs
// are float32, so no intermediate can underflow in float64.
int det_sign(const float* A1, const float* A0, const float* B1, const float* B0,
             const float* C1, const float* C0) {
  double A[3], B[3], C[3];
  for (int i = 0; i < 3; ++i) {
    A[i] = (double)A1[i] - (double)A0[i];
    B[i] = (double)B1[i] - (double)B0[i];
    C[i] = (double)C1[i] - (double)C0[i];
  }
  double m0 = B[1] * C[2] - B[2] * C[1];
  double m1 = B[0] * C[2] - B[2] * C[0];
  double m2 = B[0] * C[1] - B[1] * C[0];
  double det = A[0] * m0 - A[1] * m1 + A[2] * m2;
  double perm = std::fabs(A[0]) * (std::fabs(B[1] * C[2]) + std::fabs(B[2] * C[1])) +
                std::fabs(A[1]) * (std::fabs(B[0] * C[2]) + std::fabs(B[2] * C[0])) +
                std::fabs(A[2]) * (std::fabs(B[0] * C[1]) + std::fabs(B[1] * C[0]));
  double bound = 16.0 * std::ldexp(1.0, -53) * perm;
  if (det > bound) return 1;
  if (det < -bound) return -1;
  return det_sign_exact(A1, A0, B1, B0, C1, C0);
}

const float kZero3[3] = {0.f, 0.f, 0.f};

// orient3d(a, b, c, d) = det[b - a, c - a, d - a]: positive when d lies on the
// side of plane (a, b, c) that (b - a) x (c - a) points to.
int orient3d(const float* a, const float* b, const float* c, const float* d) {
  return det_sign(b, a, c, a, d, a);
}

struct Ray {
  float S[3], P[3], U[3], V[3];
};

struct SignStats {
  long long perturbed = 0;  // signs decided at level 1 or 2
  long long parallel = 0;   // all three levels zero (edge parallel to the ray)
};

// Perturbed sign of the edge (p, q) against the ray (see the header comment).
int edge_sign(const Ray& r, const float* p, const float* q, SignStats* st) {
  int s = det_sign(r.P, r.S, p, r.S, q, r.S);
  if (s != 0) return s;
  s = det_sign(r.P, r.S, r.U, kZero3, p, q);
  if (s == 0) s = det_sign(r.P, r.S, r.V, kZero3, p, q);
  if (st) {
    if (s != 0)
      ++st->perturbed;
    else
      ++st->parallel;
  }
  return s;
}

// ---------------------------------------------------------------------------
// Cone-beam frame (circular orbit about +z, equispaced angles).
// ---------------------------------------------------------------------------
struct Cone {
  double dso, dsd;
  int nu, nv;
  double du, dv, off_u, off_v;
};

struct Frame {
  std::vector<float> S, D, U, V;  // [na][3]
  std::vector<float> ut, vt;      // pixel-centre coordinates along U and V
  int na = 0, nu = 0, nv = 0;
};

// cos and sin of theta in float64; at quarter turns (|theta - k pi/2| < 1e-12)
// the exact values 0 and +-1 are used, since the library functions return
// 6e-17 instead of 0 there.  Every frame vector is then rounded to float32.
void cos_sin_snapped(double th, double* c, double* s) {
  double k = std::nearbyint(th / (M_PI / 2.0));
  if (std::fabs(th - k * (M_PI / 2.0)) < 1e-12) {
    long q = ((long)k % 4 + 4) % 4;
    const double cs[4][2] = {{1.0, 0.0}, {0.0, 1.0}, {-1.0, 0.0}, {0.0, -1.0}};
    *c = cs[q][0];
    *s = cs[q][1];
    return;
  }
  *c = std::cos(th);
  *s = std::sin(th);
}

Frame make_frame(const Cone& g, const double* angles, int na) {
  Frame f;
  f.na = na;
  f.nu = g.nu;
  f.nv = g.nv;
  f.S.resize(3 * na);
  f.D.resize(3 * na);
  f.U.resize(3 * na);
  f.V.resize(3 * na);
  for (int a = 0; a < na; ++a) {
    double c, s;
    cos_sin_snapped(angles[a], &c, &s);
    // Source on the orbit, detector centre opposite it, U tangent, V = +z.
    f.S[3 * a + 0] = (float)(g.dso * c);
    f.S[3 * a + 1] = (float)(g.dso * s);
    f.S[3 * a + 2] = 0.f;
    f.D[3 * a + 0] = (float)(-(g.dsd - g.dso) * c);
    f.D[3 * a + 1] = (float)(-(g.dsd - g.dso) * s);
    f.D[3 * a + 2] = 0.f;
    f.U[3 * a + 0] = (float)(-s);
    f.U[3 * a + 1] = (float)(c);
    f.U[3 * a + 2] = 0.f;
    f.V[3 * a + 0] = 0.f;
    f.V[3 * a + 1] = 0.f;
    f.V[3 * a + 2] = 1.f;
  }
  f.ut.resize(g.nu);
  f.vt.resize(g.nv);
  for (int i = 0; i < g.nu; ++i) f.ut[i] = (float)((i - (g.nu - 1) / 2.0) * g.du + g.off_u);
  for (int j = 0; j < g.nv; ++j) f.vt[j] = (float)((j - (g.nv - 1) / 2.0) * g.dv + g.off_v);
  return f;
}

// Ray of pixel (a, j, i): from the source to the pixel centre
// P = D + u_i U + v_j V, every operation rounded to float32 in this order.
Ray make_ray(const Frame& f, int64_t rid) {
  int64_t i = rid % f.nu;
  int64_t j = (rid / f.nu) % f.nv;
  int64_t a = rid / ((int64_t)f.nu * f.nv);
  Ray r;
  float u = f.ut[i], v = f.vt[j];
  for (int k = 0; k < 3; ++k) {
    r.S[k] = f.S[3 * a + k];
    r.U[k] = f.U[3 * a + k];
    r.V[k] = f.V[3 * a + k];
    volatile float uu = u * r.U[k];
    volatile float vv = v * r.V[k];
    volatile float t = f.D[3 * a + k] + uu;
    r.P[k] = t + vv;
  }
  return r;
}

// ---------------------------------------------------------------------------
// Mesh: oriented tetrahedra, face neighbours, outward faces, boundary.
// ---------------------------------------------------------------------------
enum Status {
  OK = 0,
  E_ARG = -1,
  E_DEGENERATE = -2,
  E_NONMANIFOLD = -3,
  E_NONCONVEX = -4,
  E_DISCONNECTED = -5,
  E_CAPACITY = -10,
  E_WALK = -9,
};

thread_local std::string g_err;

struct Mesh {
  int nv = 0, nt = 0;
  std::vector<float> V;                       // [nv][3]
  std::vector<std::array<int, 4>> T;          // positively oriented
  std::vector<std::array<int, 4>> N;          // neighbour across face k (opposite vertex k)
  std::vector<std::array<std::array<int, 3>, 4>> F;  // face k, outward vertex order
  std::vector<std::array<int, 2>> bfaces;     // (tet, face) of boundary faces
  int flips = 0;
  const float* p(int v) const { return &V[3 * (size_t)v]; }
};

int build_mesh(const float* verts, int nv, const int* tets, int nt, Mesh* m) {
  m->nv = nv;
  m->nt = nt;
  m->V.assign(verts, verts + 3 * (size_t)nv);
  m->T.resize(nt);
  m->N.assign(nt, {-1, -1, -1, -1});
  m->F.resize(nt);
  for (int t = 0; t < nt; ++t) {
    std::array<int, 4> v = {tets[4 * t], tets[4 * t + 1], tets[4 * t + 2], tets[4 * t + 3]};
    for (int k = 0; k < 4; ++k)
      if (v[k] < 0 || v[k] >= nv) {
        g_err = "tetrahedron " + std::to_string(t) + " references a vertex out of range";
        return E_ARG;
      }
    int o = orient3d(m->p(v[0]), m->p(v[1]), m->p(v[2]), m->p(v[3]));
    if (o == 0) {
      g_err = "tetrahedron " + std::to_string(t) + " has zero volume";
      return E_DEGENERATE;
    }
    if (o < 0) {
      std::swap(v[2], v[3]);
      ++m->flips;
    }
    m->T[t] = v;
  }
  // Faces keyed by their sorted vertex triple.
  std::map<std::array<int, 3>, std::vector<std::array<int, 2>>> owners;
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < 4; ++k) {
      std::array<int, 3> key;
      int n = 0;
      for (int j = 0; j < 4; ++j)
        if (j != k) key[n++] = m->T[t][j];
      std::sort(key.begin(), key.end());
      owners[key].push_back({t, k});
      // Outward order: the other three in local order, swapped if the normal
      // (b - a) x (c - a) points towards the opposite vertex.
      std::array<int, 3> f;
      n = 0;
      for (int j = 0; j < 4; ++j)
        if (j != k) f[n++] = m->T[t][j];
      if (orient3d(m->p(f[0]), m->p(f[1]), m->p(f[2]), m->p(m->T[t][k])) > 0) std::swap(f[1], f[2]);
      m->F[t][k] = f;
    }
  }
  for (auto& kv : owners) {
    const auto& own = kv.second;
    if (own.size() > 2) {
      g_err = "face shared by more than two tetrahedra";
      return E_NONMANIFOLD;
    }
    if (own.size() == 2) {
      if (own[0][0] == own[1][0]) {
        g_err = "tetrahedron with a repeated face";
        return E_NONMANIFOLD;
      }
      m->N[own[0][0]][own[0][1]] = own[1][0];
      m->N[own[1][0]][own[1][1]] = own[0][0];
    } else {
      m->bfaces.push_back(own[0]);
    }
  }
  std::sort(m->bfaces.begin(), m->bfaces.end());
  // Convexity (the method requires a convex mesh, Section II-D): at every
  // boundary edge the far vertex of the other boundary face must not lie
  // outside this face's plane; the boundary must also be one connected,
  // closed, consistently oriented surface.
  std::map<std::pair<int, int>, int> dir_edge;  // directed edge -> boundary face index
  const int nb = (int)m->bfaces.size();
  for (int i = 0; i < nb; ++i) {
    const auto& f = m->F[m->bfaces[i][0]][m->bfaces[i][1]];
    for (int e = 0; e < 3; ++e) {
      auto key = std::make_pair(f[e], f[(e + 1) % 3]);
      if (dir_edge.count(key)) {
        g_err = "boundary edge used twice in the same direction";
        return E_NONMANIFOLD;
      }
      dir_edge[key] = i;
    }
  }
  std::vector<int> parent(nb);
  for (int i = 0; i < nb; ++i) parent[i] = i;
  auto find = [&](int x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  for (int i = 0; i < nb; ++i) {
    const auto& f = m->F[m->bfaces[i][0]][m->bfaces[i][1]];
    for (int e = 0; e < 3; ++e) {
      int a = f[e], b = f[(e + 1) % 3], c = f[(e + 2) % 3];
      auto it = dir_edge.find(std::make_pair(b, a));
      if (it == dir_edge.end()) {
        g_err = "boundary edge without an opposite boundary face";
        return E_NONMANIFOLD;
      }
      const auto& g = m->F[m->bfaces[it->second][0]][m->bfaces[it->second][1]];
      int d = -1;
      for (int j = 0; j < 3; ++j)
        if (g[j] != a && g[j] != b) d = g[j];
      if (orient3d(m->p(a), m->p(b), m->p(c), m->p(d)) > 0) {
        g_err = "mesh is not convex";
        return E_NONCONVEX;
      }
      parent[find(i)] = find(it->second);
    }
  }
  for (int i = 0; i < nb; ++i)
    if (find(i) != find(0)) {
      g_err = "boundary surface is not connected";
      return E_DISCONNECTED;
    }
  return OK;
}

// Parameter t where the ray S + t (P - S) meets the plane of face (a, b, c).
double plane_t(const Ray& r, const float* a, const float* b, const float* c) {
  double e1[3], e2[3], n[3], as[3], d[3];
  for (int k = 0; k < 3; ++k) {
    e1[k] = (double)b[k] - a[k];
    e2[k] = (double)c[k] - a[k];
    as[k] = (double)a[k] - r.S[k];
    d[k] = (double)r.P[k] - r.S[k];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  return (as[0] * n[0] + as[1] * n[1] + as[2] * n[2]) / (d[0] * n[0] + d[1] * n[1] + d[2] * n[2]);
}

// +1 exit, -1 entry, 0 not crossed, for an outward-oriented face.
int face_cross(const Mesh& m, const Ray& r, const std::array<int, 3>& f, SignStats* st) {
  int s0 = edge_sign(r, m.p(f[0]), m.p(f[1]), st);
  if (s0 == 0) return 0;
  int s1 = edge_sign(r, m.p(f[1]), m.p(f[2]), st);
  if (s1 != s0) return 0;
  int s2 = edge_sign(r, m.p(f[2]), m.p(f[0]), st);
  if (s2 != s0) return 0;
  return s0;
}

struct WalkStats {
  long long rays = 0, hits = 0, segments = 0, zero_len = 0, failed = 0, multi_entry = 0;
  SignStats sg;
  void add(const WalkStats& o) {
    rays += o.rays;
    hits += o.hits;
    segments += o.segments;
    zero_len += o.zero_len;
    failed += o.failed;
    multi_entry += o.multi_entry;
    sg.perturbed += o.sg.perturbed;
    sg.parallel += o.sg.parallel;
  }
};

struct Visit {
  int tet;
  double len;
};

// Walk one ray.  Returns OK (possibly with an empty path for a miss) or an
// error status; the visited tetrahedra (including zero-length passages) and
// their lengths are appended to `path`.
int walk(const Mesh& m, const Ray& r, std::vector<Visit>* path, WalkStats* ws) {
  ws->rays++;
  // The tie-breaking translation needs {P - S, U, V} to be a basis.
  if (det_sign(r.P, r.S, r.U, kZero3, r.V, kZero3) == 0) {
    ws->failed++;
    g_err = "ray direction, U and V are linearly dependent";
    return E_ARG;
  }
  // Entry: brute force over every boundary face (Section II-E asks for the
  // boundary element met first; for a convex hull the perturbed ray enters
  // through exactly one boundary face).
  int cur = -1, entry_face = -1, found = 0;
  for (const auto& bf : m.bfaces) {
    if (face_cross(m, r, m.F[bf[0]][bf[1]], &ws->sg) == -1) {
      if (found == 0) {
        cur = bf[0];
        entry_face = bf[1];
      }
      ++found;
    }
  }
  if (found == 0) return OK;
  if (found > 1) {
    ws->multi_entry++;
    g_err = "ray enters the hull through more than one boundary face";
    return E_WALK;
  }
  ws->hits++;
  double dlen;
  {
    double d0 = (double)r.P[0] - r.S[0], d1 = (double)r.P[1] - r.S[1], d2 = (double)r.P[2] - r.S[2];
    dlen = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  }
  const auto& ef = m.F[cur][entry_face];
  double t_in = plane_t(r, m.p(ef[0]), m.p(ef[1]), m.p(ef[2]));
  for (int step = 0; step <= m.nt; ++step) {
    int exit_face = -1, nexit = 0;
    for (int k = 0; k < 4; ++k) {
      if (k == entry_face) continue;
      if (face_cross(m, r, m.F[cur][k], &ws->sg) == 1) {
        exit_face = k;
        ++nexit;
      }
    }
    if (nexit != 1) {
      ws->failed++;
      g_err = "tetrahedron " + std::to_string(cur) + " has " + std::to_string(nexit) + " exit faces";
      return E_WALK;
    }
    const auto& xf = m.F[cur][exit_face];
    double t_out = std::max(plane_t(r, m.p(xf[0]), m.p(xf[1]), m.p(xf[2])), t_in);
    double len = dlen * (t_out - t_in);
    path->push_back({cur, len});
    ws->segments++;
    if (len == 0.0) ws->zero_len++;
    int nb = m.N[cur][exit_face];
    if (nb < 0) return OK;
    int back = -1;
    for (int k = 0; k < 4; ++k)
      if (m.N[nb][k] == cur) back = k;
    cur = nb;
    entry_face = back;
    t_in = t_out;
  }
  ws->failed++;
  g_err = "walk exceeded the tetrahedron count";
  return E_WALK;
}

struct Neumaier {
  double s = 0, c = 0;
  void add(double v) {
    double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

int nthreads_of(int want) {
#ifdef _OPENMP
  return want > 0 ? want : omp_get_max_threads();
#else
  (void)want;
  return 1;
#endif
}

int thread_id() {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

WalkStats g_last;

Cone cone_from(const double* c) {
  Cone g;
  g.dso = c[0];
  g.dsd = c[1];
  g.nu = (int)c[2];
  g.nv = (int)c[3];
  g.du = c[4];
  g.dv = c[5];
  g.off_u = c[6];
  g.off_v = c[7];
  return g;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface used by the Python test harness.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The paper's own propagation (Algorithms 1 and 2), for the comparison of
// single and double precision (Section III-C).  Written from the algorithms:
//   Algorithm 1: Moller-Trumbore on triangle (P1, P2, P3) with safety eps:
//     d = R2 - R1, E1 = P2 - P1, E2 = P3 - P1, q = d x E2, a = E1 . q;
//     reject |a| < 1e-8; f = 1 / a; s = R1 - P1; u = f (s . q), reject u < -eps;
//     r = s x E1; v = f (d . r), reject v < -eps or u + v > 1 + eps; t = f (E2 . r).
//   Algorithm 2: per tetrahedron test the four faces with eps = 1e-9, x10
//     until two faces are hit; add l (t2 - t1) x; step across the t2 face.
// Readings (the same ones the library documents): v uses the dot product d . r;
// past eps = 1 the ray halts; t1 = smallest parameter hit, the exit is the
// face with the largest parameter other than the face the ray came in by,
// lowest index on ties; 16384 steps at most (else counted as looping); the ray enters
// through the boundary face found exactly.  Local vertex order: ascending
// node ids, the last two swapped if negatively oriented; face k opposite
// vertex k, its other vertices in increasing local order.  Arithmetic in a
// fixed order without contraction (the file is built with -ffp-contract=off).
// ---------------------------------------------------------------------------
template <typename T>
struct PV {
  T x, y, z;
};
template <typename T>
PV<T> psub(const PV<T>& a, const PV<T>& b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename T>
T pdot(const PV<T>& a, const PV<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
PV<T> pcross(const PV<T>& a, const PV<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

template <typename T>
bool moller_trumbore(const PV<T>& R1, const PV<T>& d, const PV<T>& P1, const PV<T>& P2, const PV<T>& P3, T eps,
                     T* t) {
  PV<T> E1 = psub(P2, P1), E2 = psub(P3, P1);
  PV<T> q = pcross(d, E2);
  T a = pdot(E1, q);
  const T tiny = (T)1e-8;
  if (a > -tiny && a < tiny) return false;
  T f = (T)1 / a;
  PV<T> s = psub(R1, P1);
  T u = f * pdot(s, q);
  if (u < (T)0 - eps) return false;
  PV<T> r = pcross(s, E1);
  T v = f * pdot(d, r);
  if (v < (T)0 - eps || u + v > (T)1 + eps) return false;
  *t = f * pdot(E2, r);
  return true;
}

struct PaperCounts {
  long long rays = 0, steps = 0, escalations = 0, halted = 0, looped = 0;
};

// Canonical local order of tetrahedron t and the neighbour across each face.
void canonical_tet(const Mesh& m, int t, int v[4], int nb[4]) {
  int ids[4] = {m.T[t][0], m.T[t][1], m.T[t][2], m.T[t][3]};
  std::sort(ids, ids + 4);
  if (orient3d(m.p(ids[0]), m.p(ids[1]), m.p(ids[2]), m.p(ids[3])) < 0) std::swap(ids[2], ids[3]);
  for (int k = 0; k < 4; ++k) {
    v[k] = ids[k];
    nb[k] = -1;
    for (int j = 0; j < 4; ++j)
      if (m.T[t][j] == ids[k]) nb[k] = m.N[t][j];
  }
}

template <typename T>
double paper_ray(const Mesh& m, const Ray& r, const float* x, PaperCounts* pc) {
  // Exact entry (brute force over the boundary, as in walk()).
  int cur = -1, opp = -1;
  SignStats sg;
  for (const auto& bf : m.bfaces)
    if (face_cross(m, r, m.F[bf[0]][bf[1]], &sg) == -1) {
      cur = bf[0];
      opp = m.T[bf[0]][bf[1]];
      break;
    }
  if (cur < 0) return 0.0;
  pc->rays++;
  PV<T> R1 = {(T)r.S[0], (T)r.S[1], (T)r.S[2]}, R2 = {(T)r.P[0], (T)r.P[1], (T)r.P[2]};
  PV<T> d = psub(R2, R1);
  T l = std::sqrt(pdot(d, d));
  T sum = 0;
  int v[4], nb[4];
  canonical_tet(m, cur, v, nb);
  int prev = 0;
  for (int k = 0; k < 4; ++k)
    if (v[k] == opp) prev = k;
  static const int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
  for (int step = 0;; ++step) {
    if (step >= 16384) {
      pc->looped++;
      break;
    }
    pc->steps++;
    PV<T> P[4];
    for (int k = 0; k < 4; ++k) P[k] = {(T)m.p(v[k])[0], (T)m.p(v[k])[1], (T)m.p(v[k])[2]};
    T eps = (T)1e-9, t1 = 0, t2 = 0;
    int exit = -1;
    bool halted = false;
    for (;;) {
      T th[4];
      bool hit[4];
      int nhit = 0;
      for (int k = 0; k < 4; ++k) {
        hit[k] = moller_trumbore(R1, d, P[kFace[k][0]], P[kFace[k][1]], P[kFace[k][2]], eps, &th[k]);
        nhit += hit[k] ? 1 : 0;
      }
      if (nhit >= 2) {
        bool first = true;
        for (int k = 0; k < 4; ++k)
          if (hit[k] && (first || th[k] < t1)) {
            t1 = th[k];
            first = false;
          }
        for (int k = 0; k < 4; ++k)
          if (hit[k] && k != prev && (exit < 0 || th[k] > t2)) {
            t2 = th[k];
            exit = k;
          }
        if (exit >= 0) break;
      }
      eps = eps * (T)10;
      pc->escalations++;
      if (eps > (T)1) {
        halted = true;
        break;
      }
    }
    if (halted) {
      pc->halted++;
      break;
    }
    sum = sum + l * (t2 - t1) * (T)x[cur];
    int next = nb[exit];
    if (next < 0) break;
    int nv[4], nnb[4];
    canonical_tet(m, next, nv, nnb);
    int back = 0;
    for (int k = 0; k < 4; ++k)
      if (nnb[k] == cur) back = k;
    cur = next;
    std::memcpy(v, nv, sizeof v);
    std::memcpy(nb, nnb, sizeof nb);
    prev = back;
  }
  return (double)sum;
}

extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

long long orc_exact_calls(void) { return g_exact_calls.load(); }

// Threads the parallel loops use when nthreads = 0.
int orc_max_threads(void) { return nthreads_of(0); }

// Last operation's walk statistics: rays, hits, segments, zero-length,
// failed, multi-entry, perturbed signs, parallel-edge signs.
void orc_last_stats(long long* out8) {
  const WalkStats& w = g_last;
  long long v[8] = {w.rays, w.hits, w.segments, w.zero_len, w.failed, w.multi_entry, w.sg.perturbed, w.sg.parallel};
  std::memcpy(out8, v, sizeof(v));
}

int orc_orient3d(const float* a, const float* b, const float* c, const float* d) { return orient3d(a, b, c, d); }

int orc_det_sign(const float* A1, const float* A0, const float* B1, const float* B0, const float* C1, const float* C0) {
  return det_sign(A1, A0, B1, B0, C1, C0);
}

int orc_det_sign_exact(const float* A1, const float* A0, const float* B1, const float* B0, const float* C1,
                       const float* C0) {
  return det_sign_exact(A1, A0, B1, B0, C1, C0);
}

// The same sign for n triples of difference vectors ([n][3] arrays), for
// checking other code's sign decisions in bulk.
void orc_det_sign_batch(long long n, const float* A1, const float* A0, const float* B1, const float* B0,
                        const float* C1, const float* C0, int* out) {
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < n; ++i)
    out[i] = det_sign(A1 + 3 * i, A0 + 3 * i, B1 + 3 * i, B0 + 3 * i, C1 + 3 * i, C0 + 3 * i);
}

int orc_edge_sign(const float* S, const float* P, const float* U, const float* V, const float* p, const float* q) {
  Ray r;
  std::memcpy(r.S, S, 12);
  std::memcpy(r.P, P, 12);
  std::memcpy(r.U, U, 12);
  std::memcpy(r.V, V, 12);
  return edge_sign(r, p, q, nullptr);
}

int orc_mesh_create(const float* verts, int nv, const int* tets, int nt, void** out) {
  if (!verts || !tets || nv <= 0 || nt <= 0 || !out) {
    g_err = "bad arguments";
    return E_ARG;
  }
  Mesh* m = new Mesh();
  int st = build_mesh(verts, nv, tets, nt, m);
  if (st != OK) {
    delete m;
    *out = nullptr;
    return st;
  }
  *out = m;
  return OK;
}

void orc_mesh_destroy(void* h) { delete (Mesh*)h; }

int orc_mesh_nboundary(void* h) { return (int)((Mesh*)h)->bfaces.size(); }

int orc_mesh_flips(void* h) { return ((Mesh*)h)->flips; }

// Oriented tetrahedra [nt][4], neighbours [nt][4] and outward boundary faces
// [nb][3] with their owners [nb][2] = (tet, face).
void orc_mesh_tables(void* h, int* tets, int* nbrs, int* bfaces, int* bowner) {
  const Mesh* m = (const Mesh*)h;
  for (int t = 0; t < m->nt; ++t)
    for (int k = 0; k < 4; ++k) {
      if (tets) tets[4 * t + k] = m->T[t][k];
      if (nbrs) nbrs[4 * t + k] = m->N[t][k];
    }
  for (size_t i = 0; i < m->bfaces.size(); ++i) {
    const auto& f = m->F[m->bfaces[i][0]][m->bfaces[i][1]];
    for (int k = 0; k < 3; ++k)
      if (bfaces) bfaces[3 * i + k] = f[k];
    if (bowner) {
      bowner[2 * i] = m->bfaces[i][0];
      bowner[2 * i + 1] = m->bfaces[i][1];
    }
  }
}

// Source, detector centre, U and V per angle [na][3] and pixel-centre tables.
void orc_frame(const double* cone, const double* angles, int na, float* S, float* D, float* U, float* V, float* ut,
               float* vt) {
  Cone g = cone_from(cone);
  Frame f = make_frame(g, angles, na);
  std::memcpy(S, f.S.data(), 12 * (size_t)na);
  std::memcpy(D, f.D.data(), 12 * (size_t)na);
  std::memcpy(U, f.U.data(), 12 * (size_t)na);
  std::memcpy(V, f.V.data(), 12 * (size_t)na);
  std::memcpy(ut, f.ut.data(), 4 * (size_t)g.nu);
  std::memcpy(vt, f.vt.data(), 4 * (size_t)g.nv);
}

// Endpoints of the listed rays: S [n][3], P [n][3], U [n][3], V [n][3].
void orc_rays(const double* cone, const double* angles, int na, const long long* ids, long long n, float* S,
              float* P, float* U, float* V) {
  Frame f = make_frame(cone_from(cone), angles, na);
  for (long long i = 0; i < n; ++i) {
    Ray r = make_ray(f, ids[i]);
    std::memcpy(S + 3 * i, r.S, 12);
    std::memcpy(P + 3 * i, r.P, 12);
    std::memcpy(U + 3 * i, r.U, 12);
    std::memcpy(V + 3 * i, r.V, 12);
  }
}

// Forward projection b_j = sum_i a_ij x_i for the listed rays (all rays when
// ids is NULL).  Output float64 per listed ray; nseg[j] gets the number of
// visited tetrahedra (may be NULL).
int orc_forward(void* h, const double* cone, const double* angles, int na, const float* x, const long long* ids,
                long long n, double* out, long long* nseg, int nthreads) {
  const Mesh& m = *(const Mesh*)h;
  Frame f = make_frame(cone_from(cone), angles, na);
  long long total = (long long)na * f.nu * f.nv;
  if (!ids) n = total;
  int nth = nthreads_of(nthreads);
  std::vector<WalkStats> ws(nth);
  std::atomic<int> status{OK};
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
  for (long long i = 0; i < n; ++i) {
    std::vector<Visit> path;
    long long rid = ids ? ids[i] : i;
    Ray r = make_ray(f, rid);
    int st = walk(m, r, &path, &ws[thread_id()]);
    if (st != OK) status = st;
    Neumaier acc;
    for (const auto& v : path) acc.add(v.len * (double)x[v.tet]);
    out[i] = acc.value();
    if (nseg) nseg[i] = (long long)path.size();
  }
  g_last = WalkStats();
  for (auto& w : ws) g_last.add(w);
  return status.load();
}

// Backprojection xhat_i = sum_j a_ij y_j over the listed rays; y is given per
// listed ray.  Per-thread float64 partial sums, added in thread order.
int orc_backproject(void* h, const double* cone, const double* angles, int na, const float* y, const long long* ids,
                    long long n, double* xhat, int nthreads) {
  const Mesh& m = *(const Mesh*)h;
  Frame f = make_frame(cone_from(cone), angles, na);
  long long total = (long long)na * f.nu * f.nv;
  if (!ids) n = total;
  int nth = nthreads_of(nthreads);
  std::vector<std::vector<double>> part(nth, std::vector<double>(m.nt, 0.0));
  std::vector<WalkStats> ws(nth);
  std::atomic<int> status{OK};
#pragma omp parallel for schedule(static) num_threads(nth)
  for (long long i = 0; i < n; ++i) {
    std::vector<Visit> path;
    long long rid = ids ? ids[i] : i;
    Ray r = make_ray(f, rid);
    int tid = thread_id();
    int st = walk(m, r, &path, &ws[tid]);
    if (st != OK) status = st;
    for (const auto& v : path) part[tid][v.tet] += v.len * (double)y[i];
  }
  for (int t = 0; t < m.nt; ++t) {
    double s = 0.0;
    for (int k = 0; k < nth; ++k) s += part[k][t];
    xhat[t] = s;
  }
  g_last = WalkStats();
  for (auto& w : ws) g_last.add(w);
  return status.load();
}

// Backprojection with the quantities tests bound its errors by, in one pass
// over the listed rays: xhat_i = sum_j a_ij y_j, support_i = the sum of y_j
// over the rays that cross tetrahedron i with positive length, count_i =
// the number of those rays.  Any output may be NULL.
int orc_backproject_ext(void* h, const double* cone, const double* angles, int na, const float* y,
                        const long long* ids, long long n, double* xhat, double* support, double* count,
                        int nthreads) {
  const Mesh& m = *(const Mesh*)h;
  Frame f = make_frame(cone_from(cone), angles, na);
  long long total = (long long)na * f.nu * f.nv;
  if (!ids) n = total;
  int nth = nthreads_of(nthreads);
  std::vector<std::vector<double>> part(nth, std::vector<double>(3 * (size_t)m.nt, 0.0));
  std::vector<WalkStats> ws(nth);
  std::atomic<int> status{OK};
#pragma omp parallel for schedule(static) num_threads(nth)
  for (long long i = 0; i < n; ++i) {
    std::vector<Visit> path;
    long long rid = ids ? ids[i] : i;
    Ray r = make_ray(f, rid);
    int tid = thread_id();
    int st = walk(m, r, &path, &ws[tid]);
    if (st != OK) status = st;
    double* p = part[tid].data();
    for (const auto& v : path) {
      p[3 * (size_t)v.tet] += v.len * (double)y[i];
      if (v.len > 0.0) {
        p[3 * (size_t)v.tet + 1] += (double)y[i];
        p[3 * (size_t)v.tet + 2] += 1.0;
      }
    }
  }
  for (int t = 0; t < m.nt; ++t) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nth; ++k)
      for (int c = 0; c < 3; ++c) s[c] += part[k][3 * (size_t)t + c];
    if (xhat) xhat[t] = s[0];
    if (support) support[t] = s[1];
    if (count) count[t] = s[2];
  }
  g_last = WalkStats();
  for (auto& w : ws) g_last.add(w);
  return status.load();
}

// One pass over the listed rays that gives a parity test both the
// oracle's values and the quantities its error bounds are made of.
// x and w are per tetrahedron (w: a weight such as the element size), y per
// listed ray.  Per listed ray i: b[i] = sum_k L_k x_{t_k} (Eq. 2),
// babs[i] = sum_k L_k |x_{t_k}|, chord[i] = sum_k L_k, wx[i] = the largest
// w_t |x_t| over the tetrahedra its walk visits.  Per tetrahedron t:
// xhat[t] = sum_j a_tj y_j (Eq. 3), xabs[t] = sum_j a_tj |y_j|, supp[t] = sum
// of |y_j| over the rays whose walk visits t (zero-length passages
// included), suppc[t] = the same sum weighted by each ray's chord, cnt[t] =
// the number of those visits.  Per-thread float64 partials, added in thread
// order.
int orc_check_pass(void* h, const double* cone, const double* angles, int na, const float* x, const double* w,
                   const float* y, const long long* ids, long long n, double* b, double* babs, double* chord, double* wx,
                   double* xhat, double* xabs, double* supp, double* suppc, double* cnt, int nthreads) {
  const Mesh& m = *(const Mesh*)h;
  Frame f = make_frame(cone_from(cone), angles, na);
  int nth = nthreads_of(nthreads);
  const size_t nt = (size_t)m.nt;
  std::vector<std::vector<double>> part(nth, std::vector<double>(5 * nt, 0.0));
  std::vector<WalkStats> ws(nth);
  std::atomic<int> status{OK};
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
  for (long long i = 0; i < n; ++i) {
    std::vector<Visit> path;
    Ray r = make_ray(f, ids[i]);
    int tid = thread_id();
    int st = walk(m, r, &path, &ws[tid]);
    if (st != OK) status = st;
    Neumaier sb, sa, sc;
    double mx = 0.0;
    for (const auto& v : path) {
      const double xv = (double)x[v.tet];
      sb.add(v.len * xv);
      sa.add(v.len * std::fabs(xv));
      sc.add(v.len);
      mx = std::max(mx, w[v.tet] * std::fabs(xv));
    }
    b[i] = sb.value();
    babs[i] = sa.value();
    chord[i] = sc.value();
    wx[i] = mx;
    const double yv = (double)y[i], ya = std::fabs(yv), c = chord[i];
    double* p = part[tid].data();
    for (const auto& v : path) {
      double* q = p + 5 * (size_t)v.tet;
      q[0] += v.len * yv;
      q[1] += v.len * ya;
      q[2] += ya;
      q[3] += c * ya;
      q[4] += 1.0;
    }
  }
  double* outs[5] = {xhat, xabs, supp, suppc, cnt};
  for (size_t t = 0; t < nt; ++t)
    for (int c = 0; c < 5; ++c) {
      double s = 0.0;
      for (int k = 0; k < nth; ++k) s += part[k][5 * t + c];
      outs[c][t] = s;
    }
  g_last = WalkStats();
  for (auto& x : ws) g_last.add(x);
  return status.load();
}

namespace {
int trace_common(const Mesh& m, const std::vector<Ray>& rays, long long* offsets, int* tets, double* lens,
                 long long cap) {
  long long n = (long long)rays.size();
  std::vector<std::vector<Visit>> paths(n);
  int nth = nthreads_of(0);
  std::vector<WalkStats> ws(nth);
  std::atomic<int> status{OK};
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
  for (long long i = 0; i < n; ++i) {
    int st = walk(m, rays[i], &paths[i], &ws[thread_id()]);
    if (st != OK) status = st;
  }
  g_last = WalkStats();
  for (auto& w : ws) g_last.add(w);
  long long off = 0;
  offsets[0] = 0;
  for (long long i = 0; i < n; ++i) {
    off += (long long)paths[i].size();
    offsets[i + 1] = off;
  }
  if (off > cap) return E_CAPACITY;
  for (long long i = 0; i < n; ++i) {
    long long o = offsets[i];
    for (size_t k = 0; k < paths[i].size(); ++k) {
      tets[o + k] = paths[i][k].tet;
      lens[o + k] = paths[i][k].len;
    }
  }
  return status.load();
}
}  // namespace

// Visited tetrahedra (user ids, zero-length passages included) and lengths of
// the listed rays, in CSR form: ray i owns entries offsets[i]..offsets[i+1].
// Returns E_CAPACITY (offsets filled) when cap is too small.
int orc_trace(void* h, const double* cone, const double* angles, int na, const long long* ids, long long n,
              long long* offsets, int* tets, double* lens, long long cap) {
  Frame f = make_frame(cone_from(cone), angles, na);
  std::vector<Ray> rays(n);
  for (long long i = 0; i < n; ++i) rays[i] = make_ray(f, ids[i]);
  return trace_common(*(const Mesh*)h, rays, offsets, tets, lens, cap);
}

// Same for caller-given rays: S, P, U, V are [n][3] float32.
int orc_trace_rays(void* h, const float* S, const float* P, const float* U, const float* V, long long n,
                   long long* offsets, int* tets, double* lens, long long cap) {
  std::vector<Ray> rays(n);
  for (long long i = 0; i < n; ++i) {
    std::memcpy(rays[i].S, S + 3 * i, 12);
    std::memcpy(rays[i].P, P + 3 * i, 12);
    std::memcpy(rays[i].U, U + 3 * i, 12);
    std::memcpy(rays[i].V, V + 3 * i, 12);
  }
  return trace_common(*(const Mesh*)h, rays, offsets, tets, lens, cap);
}


// The paper's propagation (see paper_ray) for the listed rays (all when ids
// is NULL) in float32 (precision 32) or float64 (64).  out[i] is the ray's
// sum rounded to float32 and widened; counts = {rays, steps, escalations,
// halted, looped}.
int orc_forward_paper(void* h, const double* cone, const double* angles, int na, const float* x, const long long* ids,
                      long long n, int precision, double* out, long long* counts, int nthreads) {
  const Mesh& m = *(const Mesh*)h;
  if (precision != 32 && precision != 64) {
    g_err = "precision must be 32 or 64";
    return E_ARG;
  }
  Frame f = make_frame(cone_from(cone), angles, na);
  long long total = (long long)na * f.nu * f.nv;
  if (!ids) n = total;
  int nth = nthreads_of(nthreads);
  std::vector<PaperCounts> pc(nth);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
  for (long long i = 0; i < n; ++i) {
    long long rid = ids ? ids[i] : i;
    Ray r = make_ray(f, rid);
    PaperCounts& c = pc[thread_id()];
    double v = precision == 64 ? paper_ray<double>(m, r, x, &c) : paper_ray<float>(m, r, x, &c);
    out[i] = (double)(float)v;
  }
  PaperCounts t;
  for (auto& c : pc) {
    t.rays += c.rays;
    t.steps += c.steps;
    t.escalations += c.escalations;
    t.halted += c.halted;
    t.looped += c.looped;
  }
  if (counts) {
    counts[0] = t.rays;
    counts[1] = t.steps;
    counts[2] = t.escalations;
    counts[3] = t.halted;
    counts[4] = t.looped;
  }
  return OK;
}

}  // extern "C"

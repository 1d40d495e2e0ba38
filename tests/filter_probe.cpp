// Test harness (host code): runs the library's own float32 sign filters
// (paper_1908_06909_amd/csrc/walk_filter.h, the code the walk kernels
// inline) on caller-given inputs, so that tests can compare every sign the
// filters certify with exact arithmetic.  Built by the tests with hipcc; the
// library itself never uses this file.
#include "walk_filter.h"

using namespace tct;

namespace {
float3 f3(const float* p) { return make_float3(p[0], p[1], p[2]); }

Ray make_ray(const float* S, const float* P, float extent) {
  Ray r{};
  r.S = f3(S);
  r.P = f3(P);
  finish_ray(r, extent);
  return r;
}
}  // namespace

extern "C" {

// Walk step filter for n cases: ray S -> P ([n][3]), mesh extent bound, ray
// parameter s = t - 1/2 of the ray point the offsets are taken from, vertex v
// and entry-face slots a0, a1, a2 ([n][3] each).
//   edge[3k + i]   step_edge_certified for E(v, a_i): 1, -1, or 0 (uncertain)
//   common[k]      step_exit_common: exit slot 0..3, or -1 when not settled
//   fsign[3k + i]  sign of the float32 estimate (what the common path uses)
void probe_step(long long n, const float* S, const float* P, const float* extent, const double* s, const float* v,
                const float* a0, const float* a1, const float* a2, int* edge, int* common, int* fsign) {
  for (long long k = 0; k < n; ++k) {
    const Ray r = make_ray(S + 3 * k, P + 3 * k, extent[k]);
    StepEdges g;
    step_edges(r, s[k], f3(v + 3 * k), f3(a0 + 3 * k), f3(a1 + 3 * k), f3(a2 + 3 * k), g);
    common[k] = step_exit_common(g);
    edge[3 * k + 0] = step_edge_certified(g.E0, g.m0, g.K);
    edge[3 * k + 1] = step_edge_certified(g.E1, g.m1, g.K);
    edge[3 * k + 2] = step_edge_certified(g.E2, g.m2, g.K);
    const float E[3] = {g.E0, g.E1, g.E2};
    for (int i = 0; i < 3; ++i) fsign[3 * k + i] = E[i] > 0.f ? 1 : (E[i] < 0.f ? -1 : 0);
  }
}

// Entry-test filter for n edges (p, q) of rays S -> P: 1, -1 or 2 (uncertain).
void probe_entry(long long n, const float* S, const float* P, const float* extent, const float* p, const float* q,
                 int* out) {
  for (long long k = 0; k < n; ++k) {
    const Ray r = make_ray(S + 3 * k, P + 3 * k, extent[k]);
    out[k] = entry_edge_sign(r, f3(p + 3 * k), f3(q + 3 * k));
  }
}

// Offsets D = v - Q of the walk (offset_from_ray), and the ray's R bound
// as finish_ray forms it (kB / (|d|_inf 192 u^2)).
void probe_offset(long long n, const float* S, const float* P, const float* extent, const double* s, const float* v,
                  float* D, float* kA, float* kB) {
  for (long long k = 0; k < n; ++k) {
    const Ray r = make_ray(S + 3 * k, P + 3 * k, extent[k]);
    const float3 d = offset_from_ray(r, s[k], f3(v + 3 * k));
    D[3 * k] = d.x;
    D[3 * k + 1] = d.y;
    D[3 * k + 2] = d.z;
    kA[k] = r.kA;
    kB[k] = r.kB;
  }
}

// Exit-slot table of the common path against the rule it encodes.
int probe_exit_table(int n_neg_bits) {
  const int s0 = (n_neg_bits & 1) ? -1 : 1, s1 = (n_neg_bits & 2) ? -1 : 1, s2 = (n_neg_bits & 4) ? -1 : 1;
  const int table = (int)((kExitFace >> (2 * n_neg_bits)) & 3u);
  return table == exit_slot(s0, s1, s2) ? table : -100 - table;
}
}

// XCD-aware block order (common.h) for one launch of n blocks.
extern "C" long long probe_xcd_block(long long b, long long n) { return (long long)xcd_block(b, n); }

// Entry i of the walk's local-index remap table (common.h).
extern "C" unsigned probe_loc_remap(unsigned i) { return loc_remap_entry(i); }

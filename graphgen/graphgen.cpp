// Seeded synthetic graph generators: R-MAT and stochastic block models.
//
// This module produces inputs only. It holds none of the clustering method's
// arithmetic (no neighbourhood intersection, no similarity, no ordering): it
// emits simple undirected graphs as CSR with strictly ascending rows, which
// both the CPU oracle and the GPU library consume.
//
// Random numbers come from one counter-based generator: the SplitMix64 output
// function (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) evaluated at state  mix(seed) + (ctr + 1) * gamma,
// i.e. the (ctr+1)-th output of a SplitMix64 stream seeded with mix(seed).
// Every draw is a pure function of (seed, counter), so results do not depend
// on the number of threads.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t draw(uint64_t seed, uint64_t ctr) {
  return mix64(mix64(seed) + (ctr + 1) * kGamma);
}

// Uniform double in [0, 1) from the top 53 bits.
inline double unit(uint64_t seed, uint64_t ctr) {
  return (double)(draw(seed, ctr) >> 11) * 0x1.0p-53;
}

struct EdgeList {
  std::vector<int32_t> u, v;
};

}  // namespace

extern "C" {

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *off;  // n + 1 entries, malloc'd
  int32_t *adj;  // nnz entries, malloc'd
} gg_csr;

uint64_t gg_draw(uint64_t seed, uint64_t ctr) { return draw(seed, ctr); }

// Standard normal draws g[x * k + i] (x < n, i < k) by the Box-Muller
// transform of two uniforms of the stream: u1 = 1 - unit(seed, 2c) is in
// (0, 1], u2 = unit(seed, 2c + 1), g = sqrt(-2 ln u1) cos(2 pi u2), c = x * k + i.
void gg_gaussians(int64_t n, int64_t k, uint64_t seed, double *g) {
  const double two_pi = 6.283185307179586;
  for (int64_t c = 0; c < n * k; ++c) {
    const double u1 = 1.0 - unit(seed, 2 * (uint64_t)c), u2 = unit(seed, 2 * (uint64_t)c + 1);
    g[c] = std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2);
  }
}

// A uniformly random permutation of 0..n-1 (Fisher-Yates with the stream).
void gg_permutation(int64_t n, uint64_t seed, uint32_t *p) {
  for (int64_t i = 0; i < n; ++i) p[i] = (uint32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    const int64_t j = (int64_t)(draw(seed, (uint64_t)i) % (uint64_t)(i + 1));
    std::swap(p[i], p[j]);
  }
}

// Edge weights parallel to adj, the same for both directions of an edge:
// w = lo + (hi - lo) * unit(seed, min(u, v) * n + max(u, v)).
void gg_edge_weights(int64_t n, const int64_t *off, const int32_t *adj, uint64_t seed, double lo,
                     double hi, double *w) {
  for (int64_t u = 0; u < n; ++u)
    for (int64_t s = off[u]; s < off[u + 1]; ++s) {
      const int64_t v = adj[s];
      const uint64_t key = (uint64_t)std::min<int64_t>(u, v) * (uint64_t)n + (uint64_t)std::max<int64_t>(u, v);
      w[s] = lo + (hi - lo) * unit(seed, key);
    }
}
double gg_unit(uint64_t seed, uint64_t ctr) { return unit(seed, ctr); }

void gg_free(gg_csr *g) {
  if (!g) return;
  free(g->off);
  free(g->adj);
  g->off = nullptr;
  g->adj = nullptr;
}

// Builds a simple undirected CSR from m directed pairs: drops self-loops and
// pairs with an endpoint outside [0, n), inserts both directions, sorts each
// row and removes duplicates. Returns 0 on success, -1 on allocation failure.
int gg_from_pairs(int64_t n, int64_t m, const int32_t *pu, const int32_t *pv, gg_csr *out) {
  out->n = n;
  out->nnz = 0;
  out->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  out->adj = nullptr;
  if (!out->off) return -1;
  std::vector<std::atomic<int64_t>> cnt((size_t)n + 1);
  for (int64_t i = 0; i <= n; ++i) cnt[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = pu[e], b = pv[e];
    if (a == b || a < 0 || b < 0 || a >= n || b >= n) continue;
    cnt[a].fetch_add(1, std::memory_order_relaxed);
    cnt[b].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + cnt[i].load(std::memory_order_relaxed);
  int64_t total = start[n];
  int32_t *tmp = (int32_t *)malloc((size_t)std::max<int64_t>(total, 1) * sizeof(int32_t));
  if (!tmp) return -1;
  for (int64_t i = 0; i <= n; ++i) cnt[i].store(start[i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = pu[e], b = pv[e];
    if (a == b || a < 0 || b < 0 || a >= n || b >= n) continue;
    tmp[cnt[a].fetch_add(1, std::memory_order_relaxed)] = b;
    tmp[cnt[b].fetch_add(1, std::memory_order_relaxed)] = a;
  }
  std::vector<int64_t> deg((size_t)n, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int32_t *b = tmp + start[i], *e = tmp + start[i + 1];
    std::sort(b, e);
    deg[i] = std::unique(b, e) - b;
  }
  for (int64_t i = 0; i < n; ++i) out->off[i + 1] = out->off[i] + deg[i];
  out->nnz = out->off[n];
  out->adj = (int32_t *)malloc((size_t)std::max<int64_t>(out->nnz, 1) * sizeof(int32_t));
  if (!out->adj) {
    free(tmp);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i)
    memcpy(out->adj + out->off[i], tmp + start[i], (size_t)deg[i] * sizeof(int32_t));
  free(tmp);
  return 0;
}

// R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each of `samples` edges
// descends `scale` levels of the adjacency matrix, picking quadrant
// (0,0) / (0,1) / (1,0) / (1,1) with probabilities a / b / c / 1-a-b-c.
// Level l of sample i uses draw(seed, i*scale + l). No noise, no permutation.
int gg_rmat(int32_t scale, int64_t samples, double a, double b, double c, uint64_t seed,
            gg_csr *out) {
  if (scale < 1 || scale > 30 || samples < 0) return -2;
  const double ab = a + b, abc = a + b + c;
  std::vector<int32_t> pu((size_t)samples), pv((size_t)samples);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < samples; ++i) {
    uint32_t x = 0, y = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double r = unit(seed, (uint64_t)i * (uint64_t)scale + (uint64_t)l);
      uint32_t xb, yb;
      if (r < a) { xb = 0; yb = 0; }
      else if (r < ab) { xb = 0; yb = 1; }
      else if (r < abc) { xb = 1; yb = 0; }
      else { xb = 1; yb = 1; }
      x = (x << 1) | xb;
      y = (y << 1) | yb;
    }
    pu[i] = (int32_t)x;
    pv[i] = (int32_t)y;
  }
  return gg_from_pairs((int64_t)1 << scale, samples, pu.data(), pv.data(), out);
}

// Stochastic block model with k blocks; vertex i lies in block b iff
// floor(b*n/k) <= i < floor((b+1)*n/k). Each pair i<j is an edge independently
// with p_in (same block) or p_out (different blocks). Bernoulli trials along
// row i are drawn by geometric skipping (Batagelj and Brandes, Phys. Rev. E 71,
// 2005): the gap to the next success is floor(log(1-r)/log(1-p)). Row i, block
// b2 uses the stream seed' = draw(seed, i*(k+1) + b2).
int gg_sbm(int64_t n, int32_t k, double p_in, double p_out, uint64_t seed, gg_csr *out) {
  if (n < 0 || k < 1 || k > n + (n == 0)) return -2;
  auto bstart = [&](int64_t b) { return (b * n) / k; };
  std::vector<int32_t> blk((size_t)n);
  for (int64_t b = 0; b < k; ++b)
    for (int64_t i = bstart(b); i < bstart(b + 1); ++i) blk[i] = (int32_t)b;
  std::vector<std::vector<int32_t>> rows((size_t)n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int32_t> &row = rows[i];
    int32_t bi = blk[i];
    for (int64_t b2 = bi; b2 < k; ++b2) {
      double p = (b2 == bi) ? p_in : p_out;
      int64_t lo = (b2 == bi) ? i + 1 : bstart(b2);
      int64_t hi = bstart(b2 + 1);
      if (p <= 0.0 || lo >= hi) continue;
      uint64_t s = draw(seed, (uint64_t)i * (uint64_t)(k + 1) + (uint64_t)b2);
      if (p >= 1.0) {
        for (int64_t j = lo; j < hi; ++j) row.push_back((int32_t)j);
        continue;
      }
      const double lq = std::log1p(-p);
      int64_t j = lo - 1;
      for (uint64_t t = 0;; ++t) {
        double r = unit(s, t);
        double gap = std::floor(std::log1p(-r) / lq);
        if (gap >= (double)(hi - j)) break;
        j += (int64_t)gap + 1;
        if (j >= hi) break;
        row.push_back((int32_t)j);
      }
    }
  }
  int64_t m = 0;
  for (auto &r : rows) m += (int64_t)r.size();
  std::vector<int32_t> pu((size_t)m), pv((size_t)m);
  int64_t e = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t j : rows[i]) {
      pu[e] = (int32_t)i;
      pv[e] = j;
      ++e;
    }
  rows.clear();
  return gg_from_pairs(n, m, pu.data(), pv.data(), out);
}

// Degree statistics used by the byte model: max degree, number of non-isolated
// vertices, W_min = sum over undirected edges {u,v} of min(deg u, deg v), and
// sum of deg^2. Reads CSR only.
void gg_degree_stats(int64_t n, const int64_t *off, const int32_t *adj, int64_t *dmax,
                     int64_t *nonisolated, int64_t *w_min, int64_t *sum_deg2) {
  int64_t dm = 0, ni = 0, wm = 0, s2 = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(max : dm) reduction(+ : ni, wm, s2)
  for (int64_t u = 0; u < n; ++u) {
    int64_t du = off[u + 1] - off[u];
    dm = std::max(dm, du);
    ni += du > 0;
    s2 += du * du;
    for (int64_t s = off[u]; s < off[u + 1]; ++s) {
      int64_t v = adj[s];
      if (v > u) wm += std::min(du, off[v + 1] - off[v]);
    }
  }
  *dmax = dm;
  *nonisolated = ni;
  *w_min = wm;
  *sum_deg2 = s2;
}

// Work split by edge owner: an edge belongs to its endpoint that is larger in
// (degree, id); owners of degree <= small_max form the "small" class. out[0..3]
// = edges and summed min-degree of small-owned edges, then of the others.
void gg_owner_split(int64_t n, const int64_t *off, const int32_t *adj, int64_t small_max,
                    int64_t *out) {
  int64_t es = 0, ws = 0, eb = 0, wb = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : es, ws, eb, wb)
  for (int64_t u = 0; u < n; ++u) {
    const int64_t du = off[u + 1] - off[u];
    for (int64_t s = off[u]; s < off[u + 1]; ++s) {
      const int64_t v = adj[s];
      if (v <= u) continue;
      const int64_t dv = off[v + 1] - off[v];
      const bool u_owns = du > dv || (du == dv && u > v);
      const int64_t downer = u_owns ? du : dv;
      const int64_t w = std::min(du, dv);
      if (downer <= small_max) {
        ++es;
        ws += w;
      } else {
        ++eb;
        wb += w;
      }
    }
  }
  out[0] = es;
  out[1] = ws;
  out[2] = eb;
  out[3] = wb;
}

}  // extern "C"

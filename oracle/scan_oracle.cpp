// CPU oracle for exact index-based SCAN (Tseng, Dhulipala and Shun,
// "Parallel Index-Based Structural Graph Clustering and Its Approximation",
// SIGMOD 2021).
//
// TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the test suite, the smoke check
// and the CPU-baseline leg of the benchmark may load this library. It shares
// no code, header, table or helper with the GPU library; both sides read the
// same CSR produced by the input generators and nothing else.
//
// Plain, slow and written for a reader checking it against the paper:
//   * similarities: Section 3.1 (closed neighbourhoods) and Section 2.1.1
//     (cosine / Jaccard), computed per undirected edge as in Algorithm 1;
//   * neighbour order and core order: Section 3.2 and Algorithm 2;
//   * query: Algorithms 3 (GetCores), 5 (Cluster) and 4 (AssignNonCores) with
//     the deterministic border rule of Section 7.3.4 (most similar
//     epsilon-similar core, ties to the lower vertex id);
//   * hubs and outliers among the unclustered vertices: Section 4.3;
//   * weighted cosine (Section 3.1): w(x, x) = 1, closed-neighbourhood sums
//     taken term by term in ascending vertex id, similarity =
//     dot / sqrt(S_u * S_v) with S the sums of squared weights;
//   * approximate similarities (Section 5; heuristic of Section 6.3): SimHash
//     bits are signs (>= 0 -> 1) of ascending-x dot products with the given
//     Gaussian draws, estimate cos(pi h / k); k-partition MinHash with the
//     given permutation, estimate matches / (k - bins empty in both); only
//     edges between two vertices of degree > k (cosine) or > 3k/2 (Jaccard)
//     are approximated, the rest are exact.
//
// Readings where the paper leaves a choice (each also listed in the design
// notes):
//   * ids are 0-based; the graph is simple (no loops, no multi-edges) and
//     stored with both directions, rows strictly ascending;
//   * c = |N[u] ∩ N[v]| over closed neighbourhoods = |N(u) ∩ N(v)| + 2 and
//     a(v) = |N[v]| = deg(v) + 1;
//   * cosine  = c / sqrt((double)a_u * (double)a_v)   (one IEEE sqrt, one div);
//     Jaccard = (double)c / (double)(a_u + a_v - c)  (one IEEE div);
//   * the neighbour order stores open neighbourhoods; self would rank first
//     with similarity 1, so the core threshold of v for mu is the (mu-1)-th
//     largest neighbour similarity, i.e. no_sim[off[v] + mu - 2];
//   * ties in both orders go to the lower vertex id; keys are the FP64 values;
//   * the core order has segments mu = 2 .. Dmax+1, segment mu holding every v
//     with deg(v) >= mu-1; co_off has Dmax+3 entries indexed by mu;
//   * query: mu < 2 or NaN eps is rejected; mu > Dmax+1 gives no cores;
//     clusters are labelled by their smallest core id, unclustered = -1.
//
// Compile without fast-math and with -ffp-contract=off.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <thread>
#include <utility>
#include <vector>

namespace {

// Runs body(i) for i in [0, count) on `threads` std::threads in contiguous
// chunks; threads <= 1 runs inline.
template <class F>
void parallel_for(int64_t count, int threads, F body) {
  if (threads <= 1 || count < 2) {
    for (int64_t i = 0; i < count; ++i) body(i);
    return;
  }
  std::vector<std::thread> pool;
  int64_t chunk = (count + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t lo = t * chunk, hi = std::min<int64_t>(count, lo + chunk);
    if (lo >= hi) break;
    pool.emplace_back([=]() {
      for (int64_t i = lo; i < hi; ++i) body(i);
    });
  }
  for (auto &th : pool) th.join();
}

// Same, but hands out items one at a time from a shared counter, for skewed
// per-item costs.
template <class F>
void parallel_for_dynamic(int64_t count, int threads, F body) {
  if (threads <= 1 || count < 2) {
    for (int64_t i = 0; i < count; ++i) body(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int64_t i = next.fetch_add(64);
        if (i >= count) break;
        for (int64_t j = i; j < std::min<int64_t>(count, i + 64); ++j) body(j);
      }
    });
  for (auto &th : pool) th.join();
}

inline int64_t degree(const int64_t *off, int64_t v) { return off[v + 1] - off[v]; }

// |N(u) ∩ N(v)| by a two-pointer merge of the two sorted rows.
int64_t common_open_neighbours(const int64_t *off, const int32_t *adj, int64_t u, int64_t v) {
  int64_t i = off[u], ie = off[u + 1], j = off[v], je = off[v + 1], t = 0;
  while (i < ie && j < je) {
    if (adj[i] < adj[j]) ++i;
    else if (adj[i] > adj[j]) ++j;
    else { ++t; ++i; ++j; }
  }
  return t;
}

// Similarity of adjacent u, v from c = |N[u] ∩ N[v]| and the closed sizes.
double similarity(int kind, int64_t c, int64_t a_u, int64_t a_v) {
  if (kind == 0) return (double)c / std::sqrt((double)a_u * (double)a_v);
  return (double)c / (double)(a_u + a_v - c);
}

// Weighted cosine (Section 3.1, the measure Algorithm 1 is written for).
// w(u, x) for x in N(u) is the weight in u's CSR slot for x, and w(x, x) = 1.
// N[v] as (id, weight) pairs in ascending id, v itself included.
std::vector<std::pair<int32_t, double>> closed_row(const int64_t *off, const int32_t *adj,
                                                   const double *w, int64_t v) {
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t s = off[v]; s < off[v + 1]; ++s) row.push_back({adj[s], w[s]});
  row.push_back({(int32_t)v, 1.0});
  std::sort(row.begin(), row.end());
  return row;
}

// Sum of w(v, x)^2 over N[v], terms added one by one in ascending x (the
// paper fixes no order; this one is the reading both implementations follow).
double closed_square_sum(const std::vector<std::pair<int32_t, double>> &row) {
  double acc = 0.0;
  for (const auto &e : row) acc += e.second * e.second;
  return acc;
}

// Sum of w(u, x) w(v, x) over x in N[u] ∩ N[v], in ascending x.
double closed_weighted_dot(const std::vector<std::pair<int32_t, double>> &a,
                           const std::vector<std::pair<int32_t, double>> &b) {
  double acc = 0.0;
  size_t i = 0, j = 0;
  while (i < a.size() && j < b.size()) {
    if (a[i].first < b[j].first) ++i;
    else if (a[i].first > b[j].first) ++j;
    else {
      acc += a[i].second * b[j].second;
      ++i;
      ++j;
    }
  }
  return acc;
}

// The dot product over the square root of the product of the two square sums
// (one IEEE multiply, sqrt and divide): with every weight 1 the sums are c,
// a_u and a_v exactly, so this is the unweighted cosine bit for bit.
double weighted_cosine(const int64_t *off, const int32_t *adj, const double *w, int64_t u, int64_t v) {
  const auto ru = closed_row(off, adj, w, u), rv = closed_row(off, adj, w, v);
  return closed_weighted_dot(ru, rv) / std::sqrt(closed_square_sum(ru) * closed_square_sum(rv));
}

// Approximate similarities (Section 5, with the degree heuristic of Section
// 6.3). The random draws are inputs: gauss[x * k + i] is coordinate x of the
// i-th SimHash direction, perm is the one permutation of k-partition MinHash.
//
// SimHash sketch of v: bit i is 1 iff the dot product of N[v] (weights
// w(v, x), w(v, v) = 1; all 1 without weights) with direction i is >= 0, the
// dot product summed term by term in ascending x.
std::vector<uint8_t> simhash_sketch(const int64_t *off, const int32_t *adj, const double *w, int64_t k,
                                    const double *gauss, int64_t v) {
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t s = off[v]; s < off[v + 1]; ++s) row.push_back({adj[s], w ? w[s] : 1.0});
  row.push_back({(int32_t)v, 1.0});
  std::sort(row.begin(), row.end());
  std::vector<uint8_t> bits(k);
  for (int64_t i = 0; i < k; ++i) {
    double dot = 0.0;
    for (const auto &e : row) dot += e.second * gauss[(int64_t)e.first * k + i];
    bits[i] = dot >= 0.0 ? 1 : 0;
  }
  return bits;
}

// k-partition (one permutation) MinHash sketch of v: the permuted range
// [0, n) is cut into k equal bins, bin(x) = floor(perm[x] * k / n); entry b
// is the least perm[x] over x in N[v] with bin(x) = b, or 0xffffffff if none.
std::vector<uint32_t> minhash_sketch(const int64_t *off, const int32_t *adj, int64_t n, int64_t k,
                                     const uint32_t *perm, int64_t v) {
  std::vector<uint32_t> sk(k, 0xffffffffu);
  auto take = [&](int64_t x) {
    const uint32_t p = perm[x];
    const int64_t b = (int64_t)((uint64_t)p * (uint64_t)k / (uint64_t)n);
    sk[b] = std::min(sk[b], p);
  };
  take(v);
  for (int64_t s = off[v]; s < off[v + 1]; ++s) take(adj[s]);
  return sk;
}

// cos(pi h / k) for h differing SimHash bits: the angle estimate of Section 2.1.2.
double simhash_estimate(int64_t h, int64_t k) { return std::cos(M_PI * (double)h / (double)k); }

// Matching non-empty bins over the bins not empty in both sketches (the
// one-permutation estimator of the Jaccard similarity).
double minhash_estimate(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
  int64_t match = 0, empty = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    if (a[i] == 0xffffffffu && b[i] == 0xffffffffu) ++empty;
    else if (a[i] == b[i]) ++match;
  }
  return (double)match / (double)((int64_t)a.size() - empty);
}

// Section 6.3's heuristic: a vertex is high degree when its degree exceeds k
// (the cosine kinds, 0 and 2: SimHash) or 3k/2 (Jaccard, kind 1: MinHash);
// only edges between two such vertices are approximated.
bool lsh_jaccard(int32_t kind) { return kind == 1; }
bool lsh_high(int32_t kind, int64_t deg, int64_t k) { return lsh_jaccard(kind) ? 2 * deg > 3 * k : deg > k; }

// Sort key for both orders: similarity descending, then vertex id ascending.
struct Entry {
  double key;
  int32_t id;
};
inline bool before(const Entry &x, const Entry &y) {
  if (x.key != y.key) return x.key > y.key;
  return x.id < y.id;
}

}  // namespace

extern "C" {

// 0 if (off, adj) is a simple undirected graph in CSR form with strictly
// ascending rows (Section 2.2); -2 otherwise, with *bad_vertex set to the
// first offending row.
int oracle_validate(int64_t n, const int64_t *off, const int32_t *adj, int64_t *bad_vertex) {
  *bad_vertex = -1;
  if (n < 0 || off[0] != 0) return -2;
  // every row range first, so that the symmetry search below reads valid rows
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) { *bad_vertex = v; return -2; }
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t s = off[v]; s < off[v + 1]; ++s) {
      int64_t w = adj[s];
      bool ok = w >= 0 && w < n && w != v && (s == off[v] || adj[s - 1] < w);
      if (ok) ok = std::binary_search(adj + off[w], adj + off[w + 1], (int32_t)v);
      if (!ok) { *bad_vertex = v; return -2; }
    }
  }
  return 0;
}

int64_t oracle_max_degree(int64_t n, const int64_t *off) {
  int64_t d = 0;
  for (int64_t v = 0; v < n; ++v) d = std::max(d, degree(off, v));
  return d;
}

// Algorithm 1 (unweighted): for every undirected edge {u, v}, u < v, count
// the closed-neighbourhood intersection and store c and the similarity in both
// CSR slots (u -> v and v -> u). counts may be null.
void oracle_similarities(int64_t n, const int64_t *off, const int32_t *adj, int32_t kind,
                         int32_t threads, int32_t *counts, double *sim) {
  parallel_for_dynamic(n, threads, [&](int64_t u) {
    for (int64_t s = off[u]; s < off[u + 1]; ++s) {
      int64_t v = adj[s];
      if (v < u) continue;
      int64_t c = common_open_neighbours(off, adj, u, v) + 2;
      double x = similarity(kind, c, degree(off, u) + 1, degree(off, v) + 1);
      int64_t m = std::lower_bound(adj + off[v], adj + off[v + 1], (int32_t)u) - adj;
      sim[s] = x;
      sim[m] = x;
      if (counts) {
        counts[s] = (int32_t)c;
        counts[m] = (int32_t)c;
      }
    }
  });
}

// One edge, for sampled checks at sizes where the full pass is too slow.
double oracle_edge_similarity(const int64_t *off, const int32_t *adj, int32_t kind, int64_t u,
                              int64_t v, int32_t *count) {
  int64_t c = common_open_neighbours(off, adj, u, v) + 2;
  if (count) *count = (int32_t)c;
  return similarity(kind, c, degree(off, u) + 1, degree(off, v) + 1);
}

// Hardware threads the host reports (std::thread::hardware_concurrency), for
// stating how many cores a timing used.
int32_t oracle_hardware_concurrency() { return (int32_t)std::thread::hardware_concurrency(); }

// oracle_edge_similarity over a list of edges (us[i], vs[i]), spread over
// threads: sampled checks of graphs too large for the full pass.
void oracle_edge_similarities(const int64_t *off, const int32_t *adj, int32_t kind, int64_t count,
                              const int64_t *us, const int64_t *vs, int32_t threads, int32_t *counts,
                              double *sims) {
  parallel_for_dynamic(count, threads, [&](int64_t i) {
    sims[i] = oracle_edge_similarity(off, adj, kind, us[i], vs[i], &counts[i]);
  });
}

// Algorithm 1 (weighted cosine): every undirected edge {u, v}, u < v, gets
// its similarity in both CSR slots. w is parallel to adj.
void oracle_weighted_similarities(int64_t n, const int64_t *off, const int32_t *adj, const double *w,
                                  int32_t threads, double *sim) {
  parallel_for_dynamic(n, threads, [&](int64_t u) {
    for (int64_t s = off[u]; s < off[u + 1]; ++s) {
      int64_t v = adj[s];
      if (v < u) continue;
      const double x = weighted_cosine(off, adj, w, u, v);
      int64_t m = std::lower_bound(adj + off[v], adj + off[v + 1], (int32_t)u) - adj;
      sim[s] = x;
      sim[m] = x;
    }
  });
}

double oracle_weighted_edge_similarity(const int64_t *off, const int32_t *adj, const double *w, int64_t u,
                                       int64_t v) {
  return weighted_cosine(off, adj, w, u, v);
}

// Sum of w(v, x)^2 over N[v] (the square of Algorithm 1's norm of v).
double oracle_weighted_square_sum(const int64_t *off, const int32_t *adj, const double *w, int64_t v) {
  return closed_square_sum(closed_row(off, adj, w, v));
}

// SimHash sketches of the given vertices: bits[j * k + i] for vertex vs[j].
void oracle_simhash_sketches(const int64_t *off, const int32_t *adj, const double *w, int64_t k,
                             const double *gauss, int64_t count, const int64_t *vs, uint8_t *bits) {
  for (int64_t j = 0; j < count; ++j) {
    const auto b = simhash_sketch(off, adj, w, k, gauss, vs[j]);
    std::copy(b.begin(), b.end(), bits + j * k);
  }
}

// k-partition MinHash sketches of the given vertices: sk[j * k + b].
void oracle_minhash_sketches(int64_t n, const int64_t *off, const int32_t *adj, int64_t k, const uint32_t *perm,
                             int64_t count, const int64_t *vs, uint32_t *sk) {
  for (int64_t j = 0; j < count; ++j) {
    const auto a = minhash_sketch(off, adj, n, k, perm, vs[j]);
    std::copy(a.begin(), a.end(), sk + j * k);
  }
}

// Approximate similarities of every edge, both CSR slots: kind 0 SimHash
// (cosine; weighted when w is not null), kind 1 k-partition MinHash
// (Jaccard). Edges that are not between two high-degree vertices get the
// exact similarity of the same kind.
void oracle_lsh_similarities(int64_t n, const int64_t *off, const int32_t *adj, const double *w, int32_t kind,
                             int64_t k, const double *gauss, const uint32_t *perm, int32_t threads, double *sim) {
  std::vector<std::vector<uint8_t>> sbits(n);
  std::vector<std::vector<uint32_t>> mh(n);
  parallel_for_dynamic(n, threads, [&](int64_t v) {
    if (!lsh_high(kind, degree(off, v), k)) return;
    if (!lsh_jaccard(kind)) sbits[v] = simhash_sketch(off, adj, w, k, gauss, v);
    else mh[v] = minhash_sketch(off, adj, n, k, perm, v);
  });
  parallel_for_dynamic(n, threads, [&](int64_t u) {
    for (int64_t s = off[u]; s < off[u + 1]; ++s) {
      int64_t v = adj[s];
      if (v < u) continue;
      double x;
      if (lsh_high(kind, degree(off, u), k) && lsh_high(kind, degree(off, v), k)) {
        if (!lsh_jaccard(kind)) {
          int64_t h = 0;
          for (int64_t i = 0; i < k; ++i) h += sbits[u][i] != sbits[v][i];
          x = simhash_estimate(h, k);
        } else {
          x = minhash_estimate(mh[u], mh[v]);
        }
      } else if (!lsh_jaccard(kind) && w) {
        x = weighted_cosine(off, adj, w, u, v);
      } else {
        x = similarity(lsh_jaccard(kind) ? 1 : 0, common_open_neighbours(off, adj, u, v) + 2, degree(off, u) + 1, degree(off, v) + 1);
      }
      int64_t m = std::lower_bound(adj + off[v], adj + off[v + 1], (int32_t)u) - adj;
      sim[s] = x;
      sim[m] = x;
    }
  });
}

// One edge of oracle_lsh_similarities, for sampled checks on large graphs.
double oracle_lsh_edge_similarity(int64_t n, const int64_t *off, const int32_t *adj, const double *w, int32_t kind,
                                  int64_t k, const double *gauss, const uint32_t *perm, int64_t u, int64_t v) {
  if (lsh_high(kind, degree(off, u), k) && lsh_high(kind, degree(off, v), k)) {
    if (!lsh_jaccard(kind)) {
      const auto a = simhash_sketch(off, adj, w, k, gauss, u), b = simhash_sketch(off, adj, w, k, gauss, v);
      int64_t h = 0;
      for (int64_t i = 0; i < k; ++i) h += a[i] != b[i];
      return simhash_estimate(h, k);
    }
    return minhash_estimate(minhash_sketch(off, adj, n, k, perm, u), minhash_sketch(off, adj, n, k, perm, v));
  }
  if (!lsh_jaccard(kind) && w) return weighted_cosine(off, adj, w, u, v);
  return similarity(lsh_jaccard(kind) ? 1 : 0, common_open_neighbours(off, adj, u, v) + 2, degree(off, u) + 1, degree(off, v) + 1);
}

// Algorithm 2, MakeNeighborOrder: each row sorted by non-increasing
// similarity, ties by lower id.
// One row: ids[0..d) with their similarities sim[0..d) -> sorted copy.
void oracle_neighbor_order_row(int64_t d, const int32_t *ids, const double *sim, int32_t *no_ids,
                               double *no_sim) {
  std::vector<Entry> row;
  for (int64_t i = 0; i < d; ++i) row.push_back({sim[i], ids[i]});
  std::stable_sort(row.begin(), row.end(), before);
  for (size_t i = 0; i < row.size(); ++i) {
    no_ids[i] = row[i].id;
    no_sim[i] = row[i].key;
  }
}

void oracle_neighbor_order(int64_t n, const int64_t *off, const int32_t *adj, const double *sim,
                           int32_t threads, int32_t *no_ids, double *no_sim) {
  parallel_for_dynamic(n, threads, [&](int64_t v) {
    oracle_neighbor_order_row(off[v + 1] - off[v], adj + off[v], sim + off[v], no_ids + off[v],
                              no_sim + off[v]);
  });
}

// Algorithm 2, MakeCoreOrder: for mu = 2 .. Dmax+1 the segment CO[mu] holds
// every v with |N[v]| >= mu, sorted by non-increasing core threshold
// no_sim[off[v] + mu - 2], ties by lower id. co_off has dmax + 3 entries.
void oracle_core_order(int64_t n, const int64_t *off, const double *no_sim, int64_t dmax,
                       int32_t threads, int64_t *co_off, int32_t *co_ids, double *co_thr) {
  // seg[mu - 2] collects (threshold, v) for every v with deg(v) >= mu - 1,
  // visiting v in ascending order.
  std::vector<std::vector<Entry>> seg((size_t)std::max<int64_t>(dmax, 0));
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = 0; j < degree(off, v); ++j) seg[j].push_back({no_sim[off[v] + j], (int32_t)v});
  co_off[0] = co_off[1] = co_off[2] = 0;
  for (int64_t mu = 2; mu <= dmax + 1; ++mu) co_off[mu + 1] = co_off[mu] + (int64_t)seg[mu - 2].size();
  parallel_for_dynamic(dmax, threads, [&](int64_t i) {
    int64_t mu = i + 2;
    std::stable_sort(seg[i].begin(), seg[i].end(), before);
    for (size_t k = 0; k < seg[i].size(); ++k) {
      co_ids[co_off[mu] + k] = seg[i][k].id;
      co_thr[co_off[mu] + k] = seg[i][k].key;
    }
  });
}

// Algorithm 5 (Cluster) over the index, with Algorithm 3 (GetCores) and
// Algorithm 4 (AssignNonCores) under the Section 7.3.4 border rule.
// memberships[v] = smallest core id of v's cluster, or -1. is_core may be null.
// Returns 0, or -1 for mu < 2 or NaN eps.
int oracle_query(int64_t n, const int64_t *off, const int32_t *no_ids, const double *no_sim,
                 const int64_t *co_off, const int32_t *co_ids, const double *co_thr, int64_t dmax,
                 int32_t mu, double eps, int32_t *memberships, uint8_t *is_core) {
  if (mu < 2 || std::isnan(eps)) return -1;
  std::vector<uint8_t> core((size_t)n, 0);
  std::vector<int32_t> cores;
  // GetCores: the prefix of CO[mu] whose thresholds are >= eps.
  if (mu <= dmax + 1) {
    for (int64_t k = co_off[mu]; k < co_off[mu + 1] && co_thr[k] >= eps; ++k) {
      cores.push_back(co_ids[k]);
      core[co_ids[k]] = 1;
    }
  }
  // similar_edges: the eps-prefix of NO[u] for each core u.
  struct Sim {
    int32_t u, w;
    double s;
  };
  std::vector<Sim> similar;
  for (int32_t u : cores)
    for (int64_t k = off[u]; k < off[u + 1] && no_sim[k] >= eps; ++k)
      similar.push_back({u, no_ids[k], no_sim[k]});
  // Connected components of the cores under core-core similar edges (BFS);
  // each component is labelled by its smallest member.
  std::vector<std::vector<int32_t>> nbr((size_t)n);
  for (const Sim &e : similar)
    if (core[e.w]) {
      nbr[e.u].push_back(e.w);
      nbr[e.w].push_back(e.u);
    }
  std::vector<int32_t> label((size_t)n, -1);
  std::vector<int32_t> sorted_cores = cores;
  std::sort(sorted_cores.begin(), sorted_cores.end());
  for (int32_t r : sorted_cores) {
    if (label[r] != -1) continue;
    std::deque<int32_t> q{r};
    label[r] = r;  // r is the smallest unlabelled core, so it is the minimum of its component
    while (!q.empty()) {
      int32_t x = q.front();
      q.pop_front();
      for (int32_t y : nbr[x])
        if (label[y] == -1) {
          label[y] = r;
          q.push_back(y);
        }
    }
  }
  // AssignNonCores: each non-core endpoint of a similar edge joins the cluster
  // of its most similar core neighbour, ties to the lower core id.
  std::vector<int32_t> best_core((size_t)n, -1);
  std::vector<double> best_sim((size_t)n, 0.0);
  for (const Sim &e : similar) {
    if (core[e.w]) continue;
    int32_t b = best_core[e.w];
    if (b == -1 || e.s > best_sim[e.w] || (e.s == best_sim[e.w] && e.u < b)) {
      best_core[e.w] = e.u;
      best_sim[e.w] = e.s;
    }
  }
  for (int64_t v = 0; v < n; ++v) {
    if (core[v]) memberships[v] = label[v];
    else memberships[v] = best_core[v] == -1 ? -1 : label[best_core[v]];
    if (is_core) is_core[v] = core[v];
  }
  return 0;
}

// Hubs and outliers (Section 4.3, with the definitions of Section 2): every
// vertex in a cluster gets role 0; an unclustered vertex (membership -1) is a
// hub (role 1) if its neighbours belong to at least two distinct clusters,
// and an outlier (role 2) otherwise (neighbours in one cluster or in none).
// The neighbours are the open neighbourhood N(v) of the CSR row.
void oracle_roles(int64_t n, const int64_t *off, const int32_t *adj, const int32_t *memberships,
                  uint8_t *roles) {
  for (int64_t v = 0; v < n; ++v) {
    if (memberships[v] >= 0) {
      roles[v] = 0;
      continue;
    }
    std::vector<int32_t> clusters;
    for (int64_t k = off[v]; k < off[v + 1]; ++k)
      if (memberships[adj[k]] >= 0) clusters.push_back(memberships[adj[k]]);
    std::sort(clusters.begin(), clusters.end());
    clusters.erase(std::unique(clusters.begin(), clusters.end()), clusters.end());
    roles[v] = clusters.size() >= 2 ? 1 : 2;
  }
}

// Modularity of a clustering (Section 7.2, Newman's definition), with every
// unclustered vertex (membership -1) in a cluster of its own (Section 7.3.4):
//   Q = 1/(2m) * sum over ordered pairs (u, v) of (A_uv - d_u d_v / 2m) delta_uv.
// Grouping the pairs by cluster C gives the two integers returned here:
//   s_in = sum over u of |{v in N(u) : v in C(u)}|  (ordered pairs inside clusters),
//   sd2  = sum over clusters of (sum of degrees in C)^2,
// and Q = (s_in - sd2 / 2m) / 2m with 2m = nnz; oracle_modularity_value does
// that last step in FP64 (one division inside, one outside).
void oracle_modularity_terms(int64_t n, const int64_t *off, const int32_t *adj, const int32_t *memberships,
                             int64_t *s_in, int64_t *sd2) {
  int64_t in = 0;
  for (int64_t u = 0; u < n; ++u)
    if (memberships[u] >= 0)
      for (int64_t k = off[u]; k < off[u + 1]; ++k)
        if (memberships[adj[k]] == memberships[u]) ++in;
  std::vector<int64_t> dsum((size_t)n, 0);  // labels are vertex ids
  int64_t sq = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = off[v + 1] - off[v];
    if (memberships[v] >= 0) dsum[memberships[v]] += d;
    else sq += d * d;  // a cluster of its own
  }
  for (int64_t c = 0; c < n; ++c) sq += dsum[c] * dsum[c];
  *s_in = in;
  *sd2 = sq;
}

double oracle_modularity_value(int64_t s_in, int64_t sd2, int64_t nnz) {
  if (nnz == 0) return 0.0;
  const double two_m = (double)nnz;
  return ((double)s_in - (double)sd2 / two_m) / two_m;
}

}  // extern "C"

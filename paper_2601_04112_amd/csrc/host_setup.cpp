// Host (CPU, FP64) construction of the LS-AMG-DD hierarchy, Algorithm 1 of
// the paper (sec. 3.2), for the library.  Independent of the test oracle.
//
// Per level: lattice aggregation with unknowns renumbered so that every
// aggregate omega_i is a contiguous range; one-layer overlap Omega_i =
// omega_i + Gamma_i from the rows of G touching omega_i (sec. 2.2, 3.1.1);
// multiplicities M and the SPSD splitting A~_i (Lemma, sec. 3.1.1); the
// reduced eigenproblem eq:gevp-S solved as S~ u = mu A_ww u; selection of
// sec. 3.4; smoother rows Z_i = A_i^{-1}(omega_i, Omega_i); interpolation
// eq:mg-p; G_{l+1} = G_l P_l (sec. 3.1.3) with exact row compression.
// When setup_device puts them there (setup_on_device), the dense local
// problems (Schur complement, eigenproblem, local and coarsest inverses) go
// to the HIP device in batches (setup_device.hip); everything else stays
// here.
#include <algorithm>
#include <cstdio>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <numeric>
#include <stdexcept>

#include "dense.hpp"
#include "internal.hpp"

namespace lsamg {

namespace {

struct SetupError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw SetupError{code, msg}; }

}  // namespace

int default_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 1;
  return (int)std::min<unsigned>(h, 32);
}

void parallel_for(int64_t n, const std::function<void(int64_t, int)>& body, int nthreads) {
  if (n <= 0) return;
  if (nthreads <= 0) nthreads = default_threads();
  nthreads = (int)std::min<int64_t>(nthreads, n);
  if (nthreads <= 1) {
    for (int64_t i = 0; i < n; ++i) body(i, 0);
    return;
  }
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  std::vector<std::thread> th;
  th.reserve(nthreads);
  for (int t = 0; t < nthreads; ++t) {
    th.emplace_back([&, t]() {
      try {
        for (;;) {
          int64_t i = next.fetch_add(1);
          if (i >= n) break;
          body(i, t);
        }
      } catch (...) {
        std::lock_guard<std::mutex> g(mu);
        if (!err) err = std::current_exception();
        next.store(n);
      }
    });
  }
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

namespace {

// Block id of each lattice index for block width b: a remainder narrower than
// b/2 joins the last block, otherwise it is a block of its own.
void axis_blocks(int extent, int b, std::vector<int>& id, int& nb) {
  id.assign(extent, 0);
  const int q = extent / b, r = extent % b;
  if (q == 0) {
    nb = 1;
    return;
  }
  if (r == 0 || 2 * r >= b) {
    for (int x = 0; x < extent; ++x) id[x] = x / b;
    nb = q + (r ? 1 : 0);
  } else {
    for (int x = 0; x < extent; ++x) id[x] = std::min(x / b, q - 1);
    nb = q;
  }
}

struct AggResult {
  int b = 0;
  int64_t nagg = 0;
  int aext[3] = {1, 1, 1};
  std::vector<int64_t> id;  // per point
};

// Aggregate lattice points (coordinates pc, weights w = unknowns per point):
// largest block b <= b0 with every aggregate holding at most omega_max
// unknowns.
AggResult aggregate_points(const std::vector<int32_t>& pc, const std::vector<int64_t>& w,
                           int ndim, const int ext[3], int b0, int omega_max) {
  const int64_t np = (int64_t)w.size();
  AggResult res;
  for (int b = b0; b >= 1; --b) {
    std::vector<int> ids[3];
    int nb[3] = {1, 1, 1};
    for (int d = 0; d < ndim; ++d) axis_blocks(ext[d], b, ids[d], nb[d]);
    int64_t nagg = 1;
    for (int d = 0; d < ndim; ++d) nagg *= nb[d];
    std::vector<int64_t> id(np);
    std::vector<int64_t> size(nagg, 0);
    for (int64_t i = 0; i < np; ++i) {
      int64_t a = 0, stride = 1;
      for (int d = 0; d < ndim; ++d) {
        a += (int64_t)ids[d][pc[(size_t)i * ndim + d]] * stride;
        stride *= nb[d];
      }
      id[i] = a;
      size[a] += w[i];
    }
    int64_t mx = *std::max_element(size.begin(), size.end());
    if (mx <= omega_max || b == 1) {
      res.b = b;
      res.nagg = nagg;
      for (int d = 0; d < 3; ++d) res.aext[d] = d < ndim ? nb[d] : 1;
      res.id = std::move(id);
      for (int64_t a = 0; a < nagg; ++a)
        if (size[a] == 0) fail(LSAMG_EINVAL, "empty aggregate");
      return res;
    }
  }
  return res;
}

// Standard aggregation (sec. 3.3) of a graph given by its adjacency lists
// (ptr/adj; self loops and repeats allowed, ignored), nodes visited in index
// order: (1) a node whose neighbours are all unaggregated starts an
// aggregate with them; (2) every node left over joins the aggregate (from
// step 1) of its lowest-numbered neighbour that step 1 aggregated.  A node
// step 1 skipped had an aggregated neighbour when visited, so step 2 places
// every node; a node without neighbours is an aggregate of its own.
// Aggregates are numbered in order of creation.
std::vector<int64_t> standard_aggregation(int64_t n, const std::vector<int64_t>& ptr,
                                          const std::vector<int64_t>& adj, int64_t& nagg) {
  std::vector<int64_t> agg(n, -1);
  nagg = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int64_t e = ptr[i]; e < ptr[i + 1] && free_nb; ++e)
      free_nb = adj[e] == i || agg[adj[e]] < 0;
    if (!free_nb) continue;
    agg[i] = nagg;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) agg[adj[e]] = nagg;
    ++nagg;
  }
  const std::vector<int64_t> first = agg;
  for (int64_t i = 0; i < n; ++i) {
    if (first[i] >= 0) continue;
    int64_t best = -1;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const int64_t j = adj[e];
      if (j != i && first[j] >= 0 && (best < 0 || j < best)) best = j;
    }
    if (best < 0) fail(LSAMG_EINVAL, "standard aggregation left a node unassigned");
    agg[i] = first[best];
  }
  return agg;
}

// Adjacency lists of n nodes from (u, v) edge pairs, both directions,
// sorted and without repeats.
void adjacency(int64_t n, const std::vector<std::pair<int64_t, int64_t>>& edges,
               std::vector<int64_t>& ptr, std::vector<int64_t>& adj) {
  ptr.assign(n + 1, 0);
  for (auto& e : edges) {
    ++ptr[e.first + 1];
    ++ptr[e.second + 1];
  }
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  adj.assign(ptr[n], 0);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (auto& e : edges) {
    adj[fill[e.first]++] = e.second;
    adj[fill[e.second]++] = e.first;
  }
  std::vector<int64_t> nptr(n + 1, 0);
  int64_t w = 0;
  for (int64_t i = 0; i < n; ++i) {
    auto b = adj.begin() + ptr[i], en = adj.begin() + ptr[i + 1];
    std::sort(b, en);
    const int64_t k = std::unique(b, en) - b;
    for (int64_t t = 0; t < k; ++t) adj[w + t] = adj[ptr[i] + t];
    w += k;
    nptr[i + 1] = w;
  }
  adj.resize(w);
  ptr.swap(nptr);
}

// `passes` rounds of standard aggregation (Algorithm 1's n_agg): the first on
// the given graph, each further one on the graph of the previous round's
// aggregates (two aggregates adjacent when an edge joins them), composed:
// the T_1 T_2 ... of sec. 3.3.  Returns the aggregate of every node.
std::vector<int64_t> aggregate_standard(int64_t n, std::vector<int64_t> ptr,
                                        std::vector<int64_t> adj, int passes, int64_t& nagg) {
  std::vector<int64_t> agg(n);
  std::iota(agg.begin(), agg.end(), 0);
  int64_t cur = n;
  for (int t = 0; t < std::max(1, passes); ++t) {
    int64_t na = 0;
    const std::vector<int64_t> a = standard_aggregation(cur, ptr, adj, na);
    for (int64_t i = 0; i < n; ++i) agg[i] = a[agg[i]];
    std::vector<std::pair<int64_t, int64_t>> edges;
    for (int64_t u = 0; u < cur; ++u)
      for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e)
        if (a[u] < a[adj[e]]) edges.emplace_back(a[u], a[adj[e]]);
    adjacency(na, edges, ptr, adj);
    cur = na;
  }
  nagg = cur;
  return agg;
}

int agg_passes_at(const lsamg_params& p, int level) {
  if (p.nagg_passes <= 0) return 1;
  return std::max(1, p.agg_passes[std::min(level, std::min(p.nagg_passes, 8) - 1)]);
}

struct Csr {
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// Everything a level needs transiently during setup.
struct Work {
  std::vector<int32_t> agg_of;                     // aggregate of each unknown
  std::vector<int64_t> gtouch_ptr;                 // per group: aggregates touched
  std::vector<int32_t> gtouch;
  std::vector<int64_t> nz_ptr;                     // per aggregate: groups in nz_i
  std::vector<int32_t> nz;
  std::vector<int64_t> dg_ptr;                     // per unknown: groups containing it
  std::vector<int32_t> dg;
  Csr A;                                           // A_l, structural pattern
};

int cmin_at(const lsamg_params& p, int level) {
  int nc = std::max(1, std::min(p.ncmin, 8));
  return std::max(1, p.cmin[std::min(level, nc - 1)]);
}

// Groups containing each unknown, and the sparse A_l = sum_g R_g^T R_g.
void build_A(Level& L, Work& W, int nthreads) {
  const Groups& G = L.G;
  const int64_t ng = G.ng(), n = L.n;
  W.dg_ptr.assign(n + 1, 0);
  for (int64_t g = 0; g < ng; ++g)
    for (int64_t q = G.sptr[g]; q < G.sptr[g + 1]; ++q) W.dg_ptr[G.supp[q] + 1]++;
  for (int64_t d = 0; d < n; ++d) W.dg_ptr[d + 1] += W.dg_ptr[d];
  W.dg.assign(W.dg_ptr[n], 0);
  {
    std::vector<int64_t> fill(W.dg_ptr.begin(), W.dg_ptr.end() - 1);
    for (int64_t g = 0; g < ng; ++g)
      for (int64_t q = G.sptr[g]; q < G.sptr[g + 1]; ++q) W.dg[fill[G.supp[q]]++] = (int32_t)g;
  }
  for (int64_t d = 0; d < n; ++d)
    if (W.dg_ptr[d + 1] == W.dg_ptr[d])
      fail(LSAMG_ENOTSPD, "an unknown is touched by no row of G (A is singular)");
  // rows of A, computed in parallel chunks then concatenated
  const int64_t chunk = 4096;
  const int64_t nchunk = (n + chunk - 1) / chunk;
  std::vector<std::vector<int32_t>> ccol(nchunk);
  std::vector<std::vector<double>> cval(nchunk);
  std::vector<std::vector<int64_t>> clen(nchunk);
  int nt = nthreads > 0 ? nthreads : default_threads();
  std::vector<std::vector<double>> acc(nt);
  std::vector<std::vector<int32_t>> mark(nt);
  parallel_for(nchunk, [&](int64_t c, int t) {
    if (acc[t].empty()) {
      acc[t].assign(n, 0.0);
      mark[t].assign(n, -1);
    }
    auto& a = acc[t];
    auto& mk = mark[t];
    std::vector<int32_t> touched;
    const int64_t d0 = c * chunk, d1 = std::min(n, d0 + chunk);
    for (int64_t d = d0; d < d1; ++d) {
      touched.clear();
      for (int64_t e = W.dg_ptr[d]; e < W.dg_ptr[d + 1]; ++e) {
        const int64_t g = W.dg[e];
        const int64_t s0 = G.sptr[g], ns = G.sptr[g + 1] - s0;
        const int32_t* sp = G.supp.data() + s0;
        const int64_t pd = std::lower_bound(sp, sp + ns, (int32_t)d) - sp;
        const double* R = G.val.data() + G.vptr[g];
        for (int64_t q = 0; q < ns; ++q)
          if (mk[sp[q]] != (int32_t)d) {
            mk[sp[q]] = (int32_t)d;
            touched.push_back(sp[q]);
          }
        for (int t2 = 0; t2 < G.nrows[g]; ++t2) {
          const double cf = R[t2 * ns + pd];
          if (cf == 0.0) continue;
          const double* row = R + t2 * ns;
          for (int64_t q = 0; q < ns; ++q) a[sp[q]] += cf * row[q];
        }
      }
      std::sort(touched.begin(), touched.end());
      for (int32_t e : touched) {
        ccol[c].push_back(e);
        cval[c].push_back(a[e]);
        a[e] = 0.0;
      }
      clen[c].push_back((int64_t)touched.size());
    }
  }, nthreads);
  W.A.ptr.assign(n + 1, 0);
  int64_t d = 0;
  for (int64_t c = 0; c < nchunk; ++c)
    for (int64_t len : clen[c]) {
      W.A.ptr[d + 1] = W.A.ptr[d] + len;
      ++d;
    }
  W.A.col.resize(W.A.ptr[n]);
  W.A.val.resize(W.A.ptr[n]);
  int64_t off = 0;
  for (int64_t c = 0; c < nchunk; ++c) {
    std::copy(ccol[c].begin(), ccol[c].end(), W.A.col.begin() + off);
    std::copy(cval[c].begin(), cval[c].end(), W.A.val.begin() + off);
    off += (int64_t)ccol[c].size();
  }
}

// nz_i, Gamma_i, Omega_i, M (Lemma of sec. 3.1.1), colouring, threshold.
void overlap_and_colour(Level& L, Work& W, const lsamg_params& p, int nthreads) {
  const Groups& G = L.G;
  const int64_t ng = G.ng(), n = L.n, na = L.nagg;
  W.agg_of.assign(n, 0);
  for (int64_t a = 0; a < na; ++a)
    for (int64_t d = L.astart[a]; d < L.astart[a + 1]; ++d) W.agg_of[d] = (int32_t)a;
  // aggregates touched by each group: supports ascend and aggregates are
  // contiguous ranges, so the touched list is the run of distinct values
  W.gtouch_ptr.assign(ng + 1, 0);
  W.gtouch.clear();
  L.M.assign(ng, 0);
  for (int64_t g = 0; g < ng; ++g) {
    int32_t last = -1;
    for (int64_t q = G.sptr[g]; q < G.sptr[g + 1]; ++q) {
      int32_t a = W.agg_of[G.supp[q]];
      if (a != last) {
        W.gtouch.push_back(a);
        last = a;
      }
    }
    W.gtouch_ptr[g + 1] = (int64_t)W.gtouch.size();
    L.M[g] = (int32_t)(W.gtouch_ptr[g + 1] - W.gtouch_ptr[g]);
  }
  W.nz_ptr.assign(na + 1, 0);
  for (int32_t a : W.gtouch) W.nz_ptr[a + 1]++;
  for (int64_t a = 0; a < na; ++a) W.nz_ptr[a + 1] += W.nz_ptr[a];
  W.nz.assign(W.nz_ptr[na], 0);
  {
    std::vector<int64_t> fill(W.nz_ptr.begin(), W.nz_ptr.end() - 1);
    for (int64_t g = 0; g < ng; ++g)
      for (int64_t e = W.gtouch_ptr[g]; e < W.gtouch_ptr[g + 1]; ++e)
        W.nz[fill[W.gtouch[e]]++] = (int32_t)g;
  }
  // Omega_i = omega_i then Gamma_i ascending
  std::vector<std::vector<int32_t>> gam(na);
  int nt = nthreads > 0 ? nthreads : default_threads();
  std::vector<std::vector<int32_t>> mark(nt);
  parallel_for(na, [&](int64_t a, int t) {
    if (mark[t].empty()) mark[t].assign(n, -1);
    auto& mk = mark[t];
    const int64_t w0 = L.astart[a], w1 = L.astart[a + 1];
    auto& out = gam[a];
    for (int64_t e = W.nz_ptr[a]; e < W.nz_ptr[a + 1]; ++e) {
      const int64_t g = W.nz[e];
      for (int64_t q = G.sptr[g]; q < G.sptr[g + 1]; ++q) {
        const int32_t d = G.supp[q];
        if (d >= w0 && d < w1) continue;
        if (mk[d] != (int32_t)a) {
          mk[d] = (int32_t)a;
          out.push_back(d);
        }
      }
    }
    std::sort(out.begin(), out.end());
  }, nthreads);
  L.optr.assign(na + 1, 0);
  for (int64_t a = 0; a < na; ++a)
    L.optr[a + 1] = L.optr[a] + (L.astart[a + 1] - L.astart[a]) + (int64_t)gam[a].size();
  L.oidx.resize(L.optr[na]);
  for (int64_t a = 0; a < na; ++a) {
    int64_t o = L.optr[a];
    for (int64_t d = L.astart[a]; d < L.astart[a + 1]; ++d) L.oidx[o++] = (int32_t)d;
    for (int32_t d : gam[a]) L.oidx[o++] = d;
  }
  // cover lists: unknown -> aggregates whose Omega holds it
  std::vector<int64_t> cptr(n + 1, 0);
  for (int32_t d : L.oidx) cptr[d + 1]++;
  for (int64_t d = 0; d < n; ++d) cptr[d + 1] += cptr[d];
  std::vector<int32_t> cov(cptr[n]);
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t a = 0; a < na; ++a)
      for (int64_t o = L.optr[a]; o < L.optr[a + 1]; ++o) cov[fill[L.oidx[o]]++] = (int32_t)a;
  }
  int64_t nmult = 0;
  for (int64_t d = 0; d < n; ++d) nmult = std::max(nmult, cptr[d + 1] - cptr[d]);
  L.n_mult = (int)nmult;
  // aggregate graph: i ~ j iff A(Omega_i, Omega_j) != 0 (structural)
  std::vector<std::vector<int32_t>> adj(na);
  std::vector<std::vector<int32_t>> mark2(nt);
  parallel_for(na, [&](int64_t a, int t) {
    if (mark2[t].empty()) mark2[t].assign(na, -1);
    auto& mk = mark2[t];
    auto& out = adj[a];
    mk[a] = (int32_t)a;
    for (int64_t o = L.optr[a]; o < L.optr[a + 1]; ++o) {
      const int32_t d = L.oidx[o];
      for (int64_t e = W.A.ptr[d]; e < W.A.ptr[d + 1]; ++e) {
        const int32_t f = W.A.col[e];
        for (int64_t c = cptr[f]; c < cptr[f + 1]; ++c) {
          const int32_t b = cov[c];
          if (mk[b] != (int32_t)a) {
            mk[b] = (int32_t)a;
            out.push_back(b);
          }
        }
      }
    }
  }, nthreads);
  std::vector<int32_t> color(na, -1);
  int ncol = 0;
  std::vector<int32_t> seen;
  for (int64_t a = 0; a < na; ++a) {
    seen.assign(adj[a].size() + 1, 0);
    for (int32_t b : adj[a])
      if (color[b] >= 0 && color[b] < (int32_t)seen.size()) seen[color[b]] = 1;
    int c = 0;
    while (seen[c]) ++c;
    color[a] = c;
    ncol = std::max(ncol, c + 1);
  }
  L.n_color = ncol;
  L.thresh = std::max(0.1, (p.kappa - ncol) / ((double)ncol * (double)std::max(1, L.n_mult)));
}

// Eigenvector count of one aggregate (sec. 3.4 and the cluster reading).
int select_count(const double* mu, int nw, const lsamg_params& p, int level, double thresh,
                 bool& hazard) {
  int k;
  hazard = false;
  if (p.n_eig_fixed > 0) {
    k = std::min(p.n_eig_fixed, nw);
  } else {
    const double cut = (1.0 / thresh) * (1.0 - p.thresh_margin);
    int count = 0;
    for (int j = 0; j < nw; ++j) {
      if (mu[j] < cut) ++count;
      if (std::fabs(mu[j] - 1.0 / thresh) <= 1e-8 / thresh) hazard = true;
    }
    k = std::min(count, nw / cmin_at(p, level));
  }
  k = std::max(k, 1);
  auto tie = [&](int j) {
    return std::fabs(mu[j] - mu[j - 1]) <= p.tie_rtol * std::fabs(mu[j]) + p.tie_atol;
  };
  const int k0 = k;
  while (k > 0 && k < nw && tie(k)) --k;
  if (k == 0) {
    k = k0;
    while (k < nw && tie(k)) ++k;
  }
  return k;
}

// Rows of B = W^{1/2} G_{nz_i} for aggregate a: every row of the groups in nz_i.
int64_t local_rows(const Level& L, const Work& W, int64_t a) {
  int64_t rows = 0;
  for (int64_t e = W.nz_ptr[a]; e < W.nz_ptr[a + 1]; ++e) rows += L.G.nrows[W.nz[e]];
  return rows;
}

// The local blocks of aggregate a (sec. 3.1.1, eq:gevp-S), written into
// zero-initialised column-major buffers: Bw and Bg (leading dimension ldb)
// the omega_i and Gamma_i columns of B = W^{1/2} G_{nz_i} (W = 1/M per
// group; rows of nz_i's groups in order, so A~_i = B^T B), Aww (leading
// dimension ldw) = G_{nz,omega}^T G_{nz,omega}, and, if Ai is not null, Ai
// (leading dimension ldo) = A(Omega_i, Omega_i).  loc holds n entries, all
// -1 on entry and again on return.
void local_blocks(const Level& L, const Work& W, int64_t a, std::vector<int32_t>& loc, double* Bw,
                  double* Bg, int64_t ldb, double* Aww, int ldw, double* Ai, int ldo) {
  const Groups& G = L.G;
  const int nw = (int)(L.astart[a + 1] - L.astart[a]);
  const int64_t o0 = L.optr[a];
  const int nO = (int)(L.optr[a + 1] - o0);
  for (int j = 0; j < nO; ++j) loc[L.oidx[o0 + j]] = j;
  std::vector<int> lp;
  int64_t r0 = 0;
  for (int64_t e = W.nz_ptr[a]; e < W.nz_ptr[a + 1]; ++e) {
    const int64_t g = W.nz[e];
    const int64_t s0 = G.sptr[g];
    const int ns = (int)(G.sptr[g + 1] - s0);
    const double sw = std::sqrt(1.0 / (double)L.M[g]);
    lp.resize(ns);
    for (int q = 0; q < ns; ++q) lp[q] = loc[G.supp[s0 + q]];
    const double* R = G.val.data() + G.vptr[g];
    for (int r = 0; r < G.nrows[g]; ++r) {
      const double* row = R + (size_t)r * ns;
      for (int qc = 0; qc < ns; ++qc) {
        const double vc = row[qc];
        if (vc == 0.0) continue;
        const int c = lp[qc];
        if (c >= nw) {
          Bg[(size_t)(c - nw) * ldb + r0 + r] = sw * vc;
          continue;
        }
        Bw[(size_t)c * ldb + r0 + r] = sw * vc;
        double* colw = Aww + (size_t)c * ldw;
        for (int qr = 0; qr < ns; ++qr)
          if (lp[qr] < nw) colw[lp[qr]] += row[qr] * vc;
      }
    }
    r0 += G.nrows[g];
  }
  if (Ai) {
    for (int r = 0; r < nO; ++r) {
      const int32_t d = L.oidx[o0 + r];
      for (int64_t e = W.A.ptr[d]; e < W.A.ptr[d + 1]; ++e) {
        const int c = loc[W.A.col[e]];
        if (c >= 0) Ai[(size_t)c * ldo + r] = W.A.val[e];
      }
    }
  }
  for (int j = 0; j < nO; ++j) loc[L.oidx[o0 + j]] = -1;
}

// Concatenate the per-aggregate results into the level's arrays.
void store_local(Level& L, std::vector<std::vector<double>>& mus,
                 std::vector<std::vector<double>>& zs, std::vector<std::vector<double>>& zh,
                 std::vector<std::vector<double>>& za, bool additive, int nthreads) {
  const int64_t na = L.nagg;
  L.muptr.assign(na + 1, 0);
  L.zoff.assign(na + 1, 0);
  L.poff.assign(na + 1, 0);
  for (int64_t a = 0; a < na; ++a) {
    L.muptr[a + 1] = L.muptr[a] + (int64_t)mus[a].size();
    L.zoff[a + 1] = L.zoff[a] + (int64_t)zs[a].size();
    L.poff[a + 1] = L.poff[a] + (int64_t)zh[a].size();
  }
  L.mu.resize(L.muptr[na]);
  L.Z.resize(L.zoff[na]);
  L.Zhat.resize(L.poff[na]);
  if (additive) {
    L.aoff.assign(na + 1, 0);
    for (int64_t a = 0; a < na; ++a) L.aoff[a + 1] = L.aoff[a] + (int64_t)za[a].size();
    L.Ainv_loc.resize(L.aoff[na]);
  }
  parallel_for(na, [&](int64_t a, int) {
    std::copy(mus[a].begin(), mus[a].end(), L.mu.begin() + L.muptr[a]);
    std::copy(zs[a].begin(), zs[a].end(), L.Z.begin() + L.zoff[a]);
    std::copy(zh[a].begin(), zh[a].end(), L.Zhat.begin() + L.poff[a]);
    if (additive) std::copy(za[a].begin(), za[a].end(), L.Ainv_loc.begin() + L.aoff[a]);
  }, nthreads);
}

// Local eigenproblems (eq:gevp-S) and smoother rows, one aggregate at a time.
void spectral_and_smoother(Level& L, Work& W, const lsamg_params& p, int level, int nthreads) {
  const int64_t na = L.nagg, n = L.n;
  L.k.assign(na, 0);
  std::vector<std::vector<double>> mus(na), zh(na), zs(na), za(na);
  const bool additive = p.cycle == LSAMG_CYCLE_ADDITIVE;
  std::atomic<int64_t> hazards{0};
  // per-phase thread time (verbose): local factor, Schur complement, local
  // eigenproblem, local inverse rows
  std::atomic<int64_t> ph_ns[4] = {{0}, {0}, {0}, {0}};
  std::atomic<int64_t> max_nO{0}, max_rows{0};
  auto tick = [] { return std::chrono::steady_clock::now(); };
  auto add_ns = [&](int i, std::chrono::steady_clock::time_point t0) {
    ph_ns[i] += std::chrono::duration_cast<std::chrono::nanoseconds>(tick() - t0).count();
  };
  int nt = nthreads > 0 ? nthreads : default_threads();
  std::vector<std::vector<int32_t>> locs(nt);
  // verbose: a line per tenth of the level's aggregates finished
  std::atomic<int64_t> finished{0};
  const int64_t tenth = std::max<int64_t>(1, na / 10);
  const auto t_level = tick();
  parallel_for(na, [&](int64_t a, int t) {
    struct Done {
      std::atomic<int64_t>& f;
      int64_t na, tenth;
      bool verbose;
      int level;
      std::chrono::steady_clock::time_point t0;
      ~Done() {
        const int64_t d = ++f;
        if (verbose && na >= 20 && d % tenth == 0)
          std::fprintf(stderr, "lsamg setup: level %d: %lld of %lld aggregates, %.1f s\n", level,
                       (long long)d, (long long)na,
                       std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      }
    } done{finished, na, tenth, p.verbose != 0, level, t_level};
    if (locs[t].empty()) locs[t].assign(n, -1);
    auto& loc = locs[t];
    const int nw = (int)(L.astart[a + 1] - L.astart[a]);
    const int64_t o0 = L.optr[a];
    const int nO = (int)(L.optr[a + 1] - o0);
    const int ng = nO - nw;
    // B = W^{1/2} G_{nz,Omega} (rows x nO, column-major; A~_i = B^T B),
    // A_ww = G_{nz,w}^T G_{nz,w} and A_i = A(Omega_i, Omega_i)
    auto t_ph = tick();
    const int64_t rows = local_rows(L, W, a);
    for (int64_t cur = max_nO.load(); nO > cur && !max_nO.compare_exchange_weak(cur, nO);) {
    }
    for (int64_t cur = max_rows.load(); rows > cur && !max_rows.compare_exchange_weak(cur, rows);) {
    }
    std::vector<double> B((size_t)rows * nO, 0.0), Aww((size_t)nw * nw, 0.0);
    std::vector<double> Ai((size_t)nO * nO, 0.0);
    local_blocks(L, W, a, loc, B.data(), B.data() + (size_t)nw * rows, rows, Aww.data(), nw,
                 Ai.data(), nO);
    // S~ = min over u_Gamma of the energy: B_w^T (I - Q Q^T) B_w, Q a basis
    // of range(B_Gamma) (the pseudo-inverse reading of eq:gevp-S)
    std::vector<double> S((size_t)nw * nw);
    add_ns(0, t_ph);
    t_ph = tick();
    if (schur_svd((int)rows, nw, ng, B.data(), p.pinv_rtol, S.data()) < 0)
      fail(LSAMG_ENOTSPD, "singular value iteration did not converge");
    add_ns(1, t_ph);
    t_ph = tick();
    // S~ u = mu A_ww u  ->  C = L^{-1} S~ L^{-T}
    if (!chol_lower(nw, Aww.data())) fail(LSAMG_ENOTSPD, "A(omega,omega) is not SPD");
    std::vector<double> X(S);
    trsm_lower(nw, Aww.data(), nw, X.data());
    std::vector<double> C((size_t)nw * nw);
    for (int j = 0; j < nw; ++j)
      for (int i = 0; i < nw; ++i) C[(size_t)j * nw + i] = X[(size_t)i * nw + j];
    trsm_lower(nw, Aww.data(), nw, C.data());
    for (int j = 0; j < nw; ++j)
      for (int i = j + 1; i < nw; ++i) {
        const double s = 0.5 * (C[(size_t)j * nw + i] + C[(size_t)i * nw + j]);
        C[(size_t)j * nw + i] = s;
        C[(size_t)i * nw + j] = s;
      }
    std::vector<double> mu(nw);
    if (!sym_eig(nw, C.data(), mu.data())) fail(LSAMG_ENOTSPD, "eigensolver did not converge");
    bool hz = false;
    const int k = select_count(mu.data(), nw, p, level, L.thresh, hz);
    if (hz) hazards++;
    trsm_lower_t(nw, Aww.data(), k, C.data());          // U = L^{-T} Y
    std::vector<double> Zh((size_t)nw * k);
    for (int t2 = 0; t2 < k; ++t2) {
      const double* u = C.data() + (size_t)t2 * nw;
      int jm = 0;
      for (int j = 1; j < nw; ++j)
        if (std::fabs(u[j]) > std::fabs(u[jm])) jm = j;
      const double sg = u[jm] < 0.0 ? -1.0 : 1.0;
      for (int j = 0; j < nw; ++j) Zh[(size_t)j * k + t2] = sg * u[j];
    }
    L.k[a] = k;
    mus[a] = std::move(mu);
    zh[a] = std::move(Zh);
    add_ns(2, t_ph);
    t_ph = tick();
    // smoother: Z_i = A_i^{-1}(omega_i, Omega_i)
    if (!chol_lower(nO, Ai.data())) fail(LSAMG_ENOTSPD, "local block A(Omega,Omega) is not SPD");
    std::vector<double> Zc((size_t)nO * nw, 0.0);
    for (int j = 0; j < nw; ++j) Zc[(size_t)j * nO + j] = 1.0;
    trsm_lower(nO, Ai.data(), nw, Zc.data());
    trsm_lower_t(nO, Ai.data(), nw, Zc.data());
    zs[a] = std::move(Zc);          // column j = row j of A_i^{-1} restricted to omega
    if (additive) {                 // the whole A_i^{-1} (additive Schwarz smoother)
      std::vector<double> Za((size_t)nO * nO, 0.0);
      for (int j = 0; j < nO; ++j) Za[(size_t)j * nO + j] = 1.0;
      trsm_lower(nO, Ai.data(), nO, Za.data());
      trsm_lower_t(nO, Ai.data(), nO, Za.data());
      za[a] = std::move(Za);
    }
    add_ns(3, t_ph);
  }, nthreads);
  L.hazards = hazards.load();
  if (p.verbose) {
    std::fprintf(stderr,
                 "lsamg setup: level %d: %lld aggregates, largest |Omega| %lld, most rows %lld; "
                 "thread seconds: local factor %.1f, Schur complement %.1f, eigenproblem %.1f, "
                 "local inverse %.1f\n",
                 level, (long long)na, (long long)max_nO.load(), (long long)max_rows.load(),
                 ph_ns[0] * 1e-9, ph_ns[1] * 1e-9, ph_ns[2] * 1e-9, ph_ns[3] * 1e-9);
    std::fflush(stderr);
  }
  store_local(L, mus, zs, zh, za, additive, nthreads);
}

// The same local problems with their dense work on the HIP device
// (device_local_problems): aggregates sorted by |Omega_i| and cut into
// batches of similar size (each block padded to its batch's largest), the
// blocks assembled on the host threads, factorised in one batched pass per
// batch, and the eigenvector counts (sec. 3.4) and signs taken on the host
// as in the host path.
void spectral_and_smoother_device(Level& L, Work& W, const lsamg_params& p, int level,
                                  int nthreads) {
  const int64_t na = L.nagg, n = L.n;
  L.k.assign(na, 0);
  const bool additive = p.cycle == LSAMG_CYCLE_ADDITIVE;
  std::vector<std::vector<double>> mus(na), zh(na), zs(na), za(na);
  std::vector<int32_t> nwv(na), nov(na);
  std::vector<int64_t> rowv(na);
  for (int64_t a = 0; a < na; ++a) {
    nwv[a] = (int32_t)(L.astart[a + 1] - L.astart[a]);
    nov[a] = (int32_t)(L.optr[a + 1] - L.optr[a]);
    rowv[a] = local_rows(L, W, a);
  }
  std::vector<int64_t> order(na);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return nov[x] != nov[y] ? nov[x] < nov[y] : rowv[x] < rowv[y];
  });
  const int nt = nthreads > 0 ? nthreads : default_threads();
  std::vector<std::vector<int32_t>> locs(nt);
  std::atomic<int64_t> hazards{0};
  double t_asm = 0, t_dev = 0, t_post = 0;
  double ph[7] = {0, 0, 0, 0, 0, 0, 0};
  int64_t full_rank = 0, with_gamma = 0;      // B_Gamma blocks, and those of full column rank
  int nbatch = 0;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto secs = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  // a batch grows while its padded blocks stay within 2^31 doubles (16 GiB),
  // and, once it holds 64 aggregates (enough to fill the device), while its
  // largest |Omega| stays within 1.25 x + 16 of its smallest
  const double cap = (double)(1LL << 31);
  for (int64_t i = 0; i < na;) {
    int64_t R = rowv[order[i]], Wd = nwv[order[i]], Od = nov[order[i]];
    int64_t Gd = Od - Wd;
    int64_t j = i + 1;
    auto per = [](int64_t r, int64_t w, int64_t g, int64_t o) {
      return (double)(2 * r * (w + g) + 3 * w * w + 2 * o * o + 2 * o * w);
    };
    for (; j < na; ++j) {
      const int64_t a = order[j];
      if (j - i >= 64 && nov[a] > 1.25 * nov[order[i]] + 16) break;
      const int64_t r2 = std::max(R, rowv[a]), w2 = std::max<int64_t>(Wd, nwv[a]);
      const int64_t g2 = std::max<int64_t>(Gd, nov[a] - nwv[a]), o2 = std::max<int64_t>(Od, nov[a]);
      if ((double)(j - i + 1) * per(r2, w2, g2, o2) > cap) break;
      R = r2, Wd = w2, Gd = g2, Od = o2;
    }
    const int nb = (int)(j - i);
    auto t0 = now();
    std::vector<int32_t> bnw(nb), rank(nb);
    // batch buffers left uninitialised here: each aggregate's thread clears
    // its own blocks, and the device writes every output entry
    auto buf = [](size_t c) { return std::unique_ptr<double[]>(new double[std::max<size_t>(c, 1)]); };
    auto Bb = buf((size_t)nb * R * (Gd + Wd));          // per aggregate [B_Gamma B_w]
    auto Aww = buf((size_t)nb * Wd * Wd), Ai = buf((size_t)nb * Od * Od);
    parallel_for(nb, [&](int64_t b, int t) {
      if (locs[t].empty()) locs[t].assign(n, -1);
      const int64_t a = order[i + b];
      bnw[b] = nwv[a];
      double* bg = Bb.get() + (size_t)b * R * (Gd + Wd);
      double* bw = bg + (size_t)R * Gd;
      double* aww = Aww.get() + (size_t)b * Wd * Wd;
      double* ai = Ai.get() + (size_t)b * Od * Od;
      std::fill_n(bg, (size_t)R * (Gd + Wd), 0.0);
      std::fill_n(aww, (size_t)Wd * Wd, 0.0);
      std::fill_n(ai, (size_t)Od * Od, 0.0);
      local_blocks(L, W, a, locs[t], bw, bg, R, aww, (int)Wd, ai, (int)Od);
      for (int64_t q = nwv[a]; q < Wd; ++q) aww[(size_t)q * Wd + q] = 1.0;
      for (int64_t q = nov[a]; q < Od; ++q) ai[(size_t)q * Od + q] = 1.0;
    }, nthreads);
    t_asm += secs(t0);
    t0 = now();
    auto mu = buf((size_t)nb * Wd), U = buf((size_t)nb * Wd * Wd), Z = buf((size_t)nb * Od * Wd);
    auto Ainv = buf(additive ? (size_t)nb * Od * Od : 0);
    std::string msg;
    const int rc = device_local_problems(p.device, nb, (int)R, (int)Wd, (int)Gd, (int)Od,
                                         p.pinv_rtol, bnw.data(), Bb.get(), Aww.get(), Ai.get(),
                                         mu.get(), U.get(), Z.get(),
                                         additive ? Ainv.get() : nullptr, rank.data(),
                                         p.verbose ? ph : nullptr, msg);
    if (rc != LSAMG_OK) fail(rc, msg);
    for (int b = 0; b < nb; ++b) {
      const int64_t a = order[i + b];
      full_rank += rank[b] == nov[a] - nwv[a];
      with_gamma += nov[a] > nwv[a];
    }
    t_dev += secs(t0);
    t0 = now();
    parallel_for(nb, [&](int64_t b, int) {
      const int64_t a = order[i + b];
      const int nw = nwv[a], nO = nov[a];
      const double* m = mu.get() + (size_t)b * Wd;
      bool hz = false;
      const int k = select_count(m, nw, p, level, L.thresh, hz);
      if (hz) hazards++;
      std::vector<double> Zh((size_t)nw * k);
      const double* ub = U.get() + (size_t)b * Wd * Wd;
      for (int t2 = 0; t2 < k; ++t2) {
        const double* u = ub + (size_t)t2 * Wd;
        int jm = 0;
        for (int q = 1; q < nw; ++q)
          if (std::fabs(u[q]) > std::fabs(u[jm])) jm = q;
        const double sg = u[jm] < 0.0 ? -1.0 : 1.0;
        for (int q = 0; q < nw; ++q) Zh[(size_t)q * k + t2] = sg * u[q];
      }
      L.k[a] = k;
      mus[a].assign(m, m + nw);
      zh[a] = std::move(Zh);
      std::vector<double> Zc((size_t)nO * nw);
      const double* zb = Z.get() + (size_t)b * Od * Wd;
      for (int q = 0; q < nw; ++q)
        std::copy(zb + (size_t)q * Od, zb + (size_t)q * Od + nO, Zc.begin() + (size_t)q * nO);
      zs[a] = std::move(Zc);
      if (additive) {
        std::vector<double> Za((size_t)nO * nO);
        const double* ab = Ainv.get() + (size_t)b * Od * Od;
        for (int q = 0; q < nO; ++q)
          std::copy(ab + (size_t)q * Od, ab + (size_t)q * Od + nO, Za.begin() + (size_t)q * nO);
        za[a] = std::move(Za);
      }
    }, nthreads);
    t_post += secs(t0);
    ++nbatch;
    i = j;
  }
  L.hazards = hazards.load();
  if (p.verbose) {
    std::fprintf(stderr,
                 "lsamg setup: level %d: %lld aggregates in %d device batches; seconds: blocks "
                 "%.2f, device %.2f (uploads %.2f, SVD %.2f, Schur products %.2f, Cholesky "
                 "and solves %.2f, eigensolver %.2f, local inverses %.2f, downloads %.2f), "
                 "counts and copies %.2f; Gamma blocks of full column rank: %lld of %lld\n",
                 level, (long long)na, nbatch, t_asm, t_dev, ph[0], ph[1], ph[2], ph[3], ph[4],
                 ph[5], ph[6], t_post, (long long)full_rank, (long long)with_gamma);
    std::fflush(stderr);
  }
  store_local(L, mus, zs, zh, za, additive, nthreads);
}

// Next level: numbering (aggregated or not), and G_{l+1} = G_l P_l grouped by
// the set of parent aggregates each row touches, every group replaced by the
// R factor of its QR factorisation.
void next_level(Level& L, Work& W, Level& N, bool aggregate_next, const lsamg_params& p,
                int level, int nthreads) {
  const int64_t na = L.nagg;
  const int ndim = L.ndim;
  std::vector<int32_t> pc((size_t)na * ndim);
  for (int64_t a = 0; a < na; ++a) {
    int64_t r = a;
    for (int d = 0; d < ndim; ++d) {
      pc[(size_t)a * ndim + d] = (int32_t)(r % L.aext[d]);
      r /= L.aext[d];
    }
  }
  std::vector<int64_t> wk(na);
  for (int64_t a = 0; a < na; ++a) wk[a] = L.k[a];
  std::vector<int64_t> cagg(na, 0);
  N.ndim = ndim;
  for (int d = 0; d < 3; ++d) N.ext[d] = L.aext[d];
  if (aggregate_next && p.aggregation == LSAMG_AGG_STANDARD) {
    // the graph of A_{l+1} joins every coarse unknown of parent a to every one
    // of parent b when a row of G_l touches both (and those of a to each
    // other), and the unknowns are numbered parent by parent: its standard
    // aggregation keeps each parent's unknowns together and equals the
    // standard aggregation of this parent graph, visited in parent order
    std::vector<std::pair<int64_t, int64_t>> edges;
    for (int64_t g = 0; g < L.G.ng(); ++g)
      for (int64_t x = W.gtouch_ptr[g]; x < W.gtouch_ptr[g + 1]; ++x)
        for (int64_t y = x + 1; y < W.gtouch_ptr[g + 1]; ++y)
          if (W.gtouch[x] != W.gtouch[y])
            edges.emplace_back(std::min(W.gtouch[x], W.gtouch[y]),
                               std::max(W.gtouch[x], W.gtouch[y]));
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    std::vector<int64_t> ptr, adj;
    adjacency(na, edges, ptr, adj);
    int64_t nagg = 0;
    cagg = aggregate_standard(na, std::move(ptr), std::move(adj), agg_passes_at(p, level + 1), nagg);
    N.block = 0;
    N.nagg = nagg;
    for (int d = 0; d < 3; ++d) N.aext[d] = 1;
  } else if (aggregate_next) {
    AggResult r = aggregate_points(pc, wk, ndim, N.ext, p.block, p.omega_max);
    cagg = r.id;
    N.block = r.b;
    N.nagg = r.nagg;
    for (int d = 0; d < 3; ++d) N.aext[d] = r.aext[d];
  }
  std::vector<int64_t> order(na);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t x, int64_t y) { return cagg[x] < cagg[y]; });
  L.cstart.assign(na + 1, 0);
  std::vector<int64_t> canon_off(na + 1, 0);
  for (int64_t a = 0; a < na; ++a) canon_off[a + 1] = canon_off[a] + L.k[a];
  int64_t off = 0;
  N.n = canon_off[na];
  N.coord.resize((size_t)N.n * ndim);
  N.canon.resize(N.n);
  if (aggregate_next) N.astart.assign(N.nagg + 1, 0);
  for (int64_t t = 0; t < na; ++t) {
    const int64_t a = order[t];
    L.cstart[a] = off;
    for (int s = 0; s < L.k[a]; ++s) {
      for (int d = 0; d < ndim; ++d) N.coord[(size_t)(off + s) * ndim + d] = pc[(size_t)a * ndim + d];
      N.canon[off + s] = canon_off[a] + s;
    }
    if (aggregate_next) N.astart[cagg[a] + 1] += L.k[a];
    off += L.k[a];
  }
  L.cstart[na] = off;
  if (aggregate_next)
    for (int64_t c = 0; c < N.nagg; ++c) N.astart[c + 1] += N.astart[c];
  // group the rows of G_l by touched-aggregate set
  const Groups& G = L.G;
  const int64_t ng = G.ng();
  typedef std::array<int32_t, 8> Key;
  std::vector<Key> keys(ng);
  for (int64_t g = 0; g < ng; ++g) {
    Key k;
    k.fill(-1);
    const int64_t t0 = W.gtouch_ptr[g], nt = W.gtouch_ptr[g + 1] - t0;
    if (nt > 8) fail(LSAMG_EINVAL, "a row of G touches more than 8 aggregates");
    for (int64_t e = 0; e < nt; ++e) k[e] = W.gtouch[t0 + e];
    std::sort(k.begin(), k.begin() + nt);
    keys[g] = k;
  }
  std::vector<int64_t> gord(ng);
  std::iota(gord.begin(), gord.end(), 0);
  std::sort(gord.begin(), gord.end(), [&](int64_t x, int64_t y) {
    if (keys[x] != keys[y]) return keys[x] < keys[y];
    return x < y;
  });
  std::vector<int64_t> gstart;
  for (int64_t t = 0; t < ng; ++t)
    if (t == 0 || keys[gord[t]] != keys[gord[t - 1]]) gstart.push_back(t);
  gstart.push_back(ng);
  const int64_t nng = (int64_t)gstart.size() - 1;
  std::vector<std::vector<int32_t>> nsupp(nng);
  std::vector<std::vector<double>> nval(nng);
  std::vector<int32_t> nrows(nng);
  parallel_for(nng, [&](int64_t h, int) {
    const Key& key = keys[gord[gstart[h]]];
    std::vector<int64_t> par;
    for (int32_t a : key)
      if (a >= 0) par.push_back(a);
    std::sort(par.begin(), par.end(), [&](int64_t x, int64_t y) { return L.cstart[x] < L.cstart[y]; });
    std::vector<int32_t> supp;
    std::vector<int64_t> pos(par.size());
    for (size_t e = 0; e < par.size(); ++e) {
      pos[e] = (int64_t)supp.size();
      for (int s = 0; s < L.k[par[e]]; ++s) supp.push_back((int32_t)(L.cstart[par[e]] + s));
    }
    const int c = (int)supp.size();
    int64_t rows = 0;
    for (int64_t t = gstart[h]; t < gstart[h + 1]; ++t) rows += G.nrows[gord[t]];
    std::vector<double> B((size_t)rows * c, 0.0);     // column-major rows x c
    int64_t r0 = 0;
    for (int64_t t = gstart[h]; t < gstart[h + 1]; ++t) {
      const int64_t g = gord[t];
      const int64_t s0 = G.sptr[g];
      const int ns = (int)(G.sptr[g + 1] - s0);
      const double* R = G.val.data() + G.vptr[g];
      for (int q = 0; q < ns; ++q) {
        const int32_t d = G.supp[s0 + q];
        const int32_t a = W.agg_of[d];
        const int64_t e = std::find(par.begin(), par.end(), (int64_t)a) - par.begin();
        const int kk = L.k[a];
        const int pw = (int)(d - L.astart[a]);
        const double* zrow = L.Zhat.data() + L.poff[a] + (size_t)pw * kk;
        for (int r = 0; r < G.nrows[g]; ++r) {
          const double v = R[(size_t)r * ns + q];
          if (v == 0.0) continue;
          for (int s = 0; s < kk; ++s) B[(size_t)(pos[e] + s) * rows + r0 + r] += v * zrow[s];
        }
      }
      r0 += G.nrows[g];
    }
    qr_r((int)rows, c, B.data());
    const int nr = (int)std::min<int64_t>(rows, c);
    std::vector<double> out((size_t)nr * c);
    for (int r = 0; r < nr; ++r)
      for (int j = 0; j < c; ++j) out[(size_t)r * c + j] = B[(size_t)j * rows + r];
    nsupp[h] = std::move(supp);
    nval[h] = std::move(out);
    nrows[h] = nr;
  }, nthreads);
  Groups& NG = N.G;
  NG.sptr.assign(nng + 1, 0);
  NG.vptr.assign(nng + 1, 0);
  NG.nrows = nrows;
  for (int64_t h = 0; h < nng; ++h) {
    NG.sptr[h + 1] = NG.sptr[h] + (int64_t)nsupp[h].size();
    NG.vptr[h + 1] = NG.vptr[h] + (int64_t)nval[h].size();
  }
  NG.supp.resize(NG.sptr[nng]);
  NG.val.resize(NG.vptr[nng]);
  for (int64_t h = 0; h < nng; ++h) {
    std::copy(nsupp[h].begin(), nsupp[h].end(), NG.supp.begin() + NG.sptr[h]);
    std::copy(nval[h].begin(), nval[h].end(), NG.val.begin() + NG.vptr[h]);
  }
}

// Dense inverse of the coarsest A_L (on the HIP device `device` if >= 0).
void coarsest_inverse(Level& L, Work& W, int nthreads, int device) {
  const int64_t n = L.n;
  if (n > 40000) fail(LSAMG_EINVAL, "coarsest level too large for a dense solve");
  std::vector<double> A((size_t)n * n, 0.0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = W.A.ptr[r]; e < W.A.ptr[r + 1]; ++e) A[(size_t)W.A.col[e] * n + r] = W.A.val[e];
  if (device >= 0) {
    L.Ainv.assign((size_t)n * n, 0.0);
    std::string msg;
    const int rc = device_spd_inverse(device, (int)n, A.data(), L.Ainv.data(), msg);
    if (rc != LSAMG_OK) fail(rc, msg);
    return;
  }
  if (!chol_lower((int)n, A.data())) fail(LSAMG_ENOTSPD, "coarsest matrix is not SPD");
  L.Ainv.assign((size_t)n * n, 0.0);
  parallel_for(n, [&](int64_t j, int) {
    double* x = L.Ainv.data() + (size_t)j * n;
    x[j] = 1.0;
    trsm_lower((int)n, A.data(), 1, x);
    trsm_lower_t((int)n, A.data(), 1, x);
  }, nthreads);
}

}  // namespace

bool setup_on_device(const lsamg_params& p, int64_t n) {
  if (p.device < 0 || p.setup_device == LSAMG_SETUP_HOST) return false;
  return p.setup_device == LSAMG_SETUP_DEVICE || n >= kAutoDeviceSetupN;
}

int build_hierarchy(const lsamg_csr& Gin, const lsamg_params& p, Hierarchy& H, std::string& msg) {
  auto t0 = std::chrono::steady_clock::now();
  try {
    H.params = p;
    const bool standard = p.aggregation == LSAMG_AGG_STANDARD;
    if (!standard && p.aggregation != LSAMG_AGG_LATTICE) fail(LSAMG_EINVAL, "bad aggregation");
    // standard aggregation needs no lattice: the columns form a line
    const int ndim = standard && p.ndim == 0 ? 1 : p.ndim;
    if (ndim < 1 || ndim > 3) fail(LSAMG_EINVAL, "ndim must be 1, 2 or 3");
    int grid[3] = {1, 1, 1};
    int64_t np = 1;
    for (int d = 0; d < ndim; ++d) {
      grid[d] = standard && p.ndim == 0 ? (int)std::min<int64_t>(Gin.n, INT32_MAX) : p.grid[d];
      if (grid[d] <= 0) fail(LSAMG_EINVAL, "grid extents must be positive");
      np *= grid[d];
    }
    if (Gin.n != np) fail(LSAMG_EINVAL, "G has n columns != product of grid extents");
    if (standard && (p.nagg_passes < 1 || p.nagg_passes > 8)) fail(LSAMG_EINVAL, "bad agg_passes");
    if (p.cycle != LSAMG_CYCLE_V && p.cycle != LSAMG_CYCLE_ADDITIVE) fail(LSAMG_EINVAL, "bad cycle");
    if (p.setup_device < LSAMG_SETUP_HOST || p.setup_device > LSAMG_SETUP_AUTO)
      fail(LSAMG_EINVAL, "bad setup_device");
    if (p.setup_device == LSAMG_SETUP_DEVICE && p.device < 0)
      fail(LSAMG_EINVAL, "setup on the device needs a HIP device (device >= 0)");
    const bool on_dev = setup_on_device(p, Gin.n);
    if (Gin.m <= 0 || Gin.n <= 0 || !Gin.rowptr || (Gin.nnz > 0 && (!Gin.col || !Gin.val)))
      fail(LSAMG_EINVAL, "bad G");
    if (p.block < 1 || p.omega_max < 1 || p.max_levels < 1) fail(LSAMG_EINVAL, "bad params");
    if (Gin.rowptr[0] != 0 || Gin.rowptr[Gin.m] != Gin.nnz) fail(LSAMG_EINVAL, "bad rowptr");
    if (Gin.n > INT32_MAX) fail(LSAMG_EINVAL, "n too large");
    const int nthreads = p.nthreads;
    H.ndim = ndim;
    const int64_t n = Gin.n;
    // level-0 aggregation on the canonical lattice
    std::vector<int32_t> pc((size_t)n * ndim);
    for (int64_t c = 0; c < n; ++c) {
      int64_t r = c;
      for (int d = 0; d < ndim; ++d) {
        pc[(size_t)c * ndim + d] = (int32_t)(r % grid[d]);
        r /= grid[d];
      }
    }
    H.levels.clear();
    H.levels.emplace_back();
    Level& L0 = H.levels[0];
    L0.n = n;
    L0.ndim = ndim;
    for (int d = 0; d < 3; ++d) L0.ext[d] = d < ndim ? grid[d] : 1;
    const bool agg0 = (p.max_levels > 1) && (n > p.max_coarse);
    std::vector<int64_t> aid(n, 0);
    if (agg0 && standard) {
      // graph of A = G^T G: columns sharing a row of G (exact zeros dropped)
      std::vector<std::pair<int64_t, int64_t>> edges;
      std::vector<int64_t> cols;
      for (int64_t r = 0; r < Gin.m; ++r) {
        cols.clear();
        for (int64_t e = Gin.rowptr[r]; e < Gin.rowptr[r + 1]; ++e) {
          const int32_t c = Gin.col[e];
          if (c < 0 || c >= n) fail(LSAMG_EINVAL, "column index out of range");
          if (Gin.val[e] != 0.0) cols.push_back(c);
        }
        for (size_t x = 0; x < cols.size(); ++x)
          for (size_t y = x + 1; y < cols.size(); ++y)
            if (cols[x] != cols[y])
              edges.emplace_back(std::min(cols[x], cols[y]), std::max(cols[x], cols[y]));
      }
      std::sort(edges.begin(), edges.end());
      edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
      std::vector<int64_t> ptr, adj;
      adjacency(n, edges, ptr, adj);
      int64_t nagg = 0;
      aid = aggregate_standard(n, std::move(ptr), std::move(adj), agg_passes_at(p, 0), nagg);
      L0.block = 0;
      L0.nagg = nagg;
    } else if (agg0) {
      std::vector<int64_t> w(n, 1);
      AggResult r = aggregate_points(pc, w, ndim, L0.ext, p.block, p.omega_max);
      aid = r.id;
      L0.block = r.b;
      L0.nagg = r.nagg;
      for (int d = 0; d < 3; ++d) L0.aext[d] = r.aext[d];
    }
    std::vector<int64_t> perm(n);      // internal -> canonical
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return aid[x] < aid[y]; });
    std::vector<int32_t> inv(n);
    for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
    L0.canon = perm;
    L0.coord.resize((size_t)n * ndim);
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < ndim; ++d) L0.coord[(size_t)i * ndim + d] = pc[(size_t)perm[i] * ndim + d];
    if (agg0) {
      L0.astart.assign(L0.nagg + 1, 0);
      for (int64_t c = 0; c < n; ++c) L0.astart[aid[c] + 1]++;
      for (int64_t a = 0; a < L0.nagg; ++a) L0.astart[a + 1] += L0.astart[a];
    }
    // level-0 groups: every non-empty row of G (exact zeros dropped)
    Groups& G0 = L0.G;
    G0.sptr.assign(1, 0);
    G0.vptr.assign(1, 0);
    H.row_map.clear();
    std::vector<std::pair<int32_t, double>> ent;
    for (int64_t r = 0; r < Gin.m; ++r) {
      ent.clear();
      const int64_t e0 = Gin.rowptr[r], e1 = Gin.rowptr[r + 1];
      if (e1 < e0) fail(LSAMG_EINVAL, "rowptr not monotone");
      for (int64_t e = e0; e < e1; ++e) {
        const int32_t c = Gin.col[e];
        const double v = Gin.val[e];
        if (c < 0 || c >= n) fail(LSAMG_EINVAL, "column index out of range");
        if (!std::isfinite(v)) fail(LSAMG_EBADINPUT, "non-finite entry in G");
        if (v != 0.0) ent.emplace_back(inv[c], v);
      }
      if (ent.empty()) continue;
      std::sort(ent.begin(), ent.end());
      for (size_t q = 1; q < ent.size(); ++q)
        if (ent[q].first == ent[q - 1].first) fail(LSAMG_EINVAL, "duplicate column in a row of G");
      H.row_map.push_back(r);
      for (auto& pr : ent) {
        G0.supp.push_back(pr.first);
        G0.val.push_back(pr.second);
      }
      G0.sptr.push_back((int64_t)G0.supp.size());
      G0.vptr.push_back((int64_t)G0.val.size());
      G0.nrows.push_back(1);
    }
    H.m0 = (int64_t)H.row_map.size();
    // Algorithm 1 main loop
    int l = 0;
    bool aggregated = agg0;
    auto progress = [&](int lev, const char* what) {
      if (!p.verbose) return;
      const double t =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      std::fprintf(stderr, "lsamg setup: level %d (n=%lld) %s, %.1f s\n", lev,
                   (long long)H.levels[lev].n, what, t);
      std::fflush(stderr);
    };
    for (;;) {
      Level& L = H.levels[l];
      Work W;
      build_A(L, W, nthreads);
      L.a_nnz = W.A.ptr[L.n];
      if (!aggregated) {
        L.coarsest = true;
        coarsest_inverse(L, W, nthreads, on_dev ? p.device : -1);
        progress(l, "coarsest inverse done");
        break;
      }
      overlap_and_colour(L, W, p, nthreads);
      progress(l, "overlap and colouring done");
      if (on_dev)
        spectral_and_smoother_device(L, W, p, l, nthreads);
      else
        spectral_and_smoother(L, W, p, l, nthreads);
      progress(l, "local eigenproblems and smoother done");
      int64_t nn = 0;
      for (int32_t kk : L.k) nn += kk;
      const bool stall = (double)nn > p.stall_ratio * (double)L.n;
      const bool agg_next = (l + 1 < p.max_levels - 1) && (nn > p.max_coarse) && !stall;
      Level N;
      next_level(L, W, N, agg_next, p, l, nthreads);
      H.levels.push_back(std::move(N));
      aggregated = agg_next;
      ++l;
    }
  } catch (const SetupError& e) {
    msg = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed during setup";
    return LSAMG_ENOMEM;
  } catch (const std::exception& e) {
    msg = e.what();
    return LSAMG_EINVAL;
  }
  H.setup_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return LSAMG_OK;
}

// C = G^+ F by the symmetric eigen-decomposition G = V diag(w) V^T:
// C = V diag(1/w_k, kept) V^T F
int gram_pinv_apply(int s, const double* G, const double* F, double* C, double rtol) {
  std::vector<double> V((size_t)s * s), w(s);
  for (int i = 0; i < s; ++i)          // column-major symmetric copy, (G + G^T) / 2
    for (int j = 0; j < s; ++j) V[(size_t)j * s + i] = 0.5 * (G[(size_t)i * s + j] + G[(size_t)j * s + i]);
  if (!sym_eig(s, V.data(), w.data())) return -1;
  const double wmax = s > 0 ? std::max(w[s - 1], 0.0) : 0.0;
  std::vector<double> VtF((size_t)s * s, 0.0);   // (V^T F) scaled by 1/w, row k
  int rank = 0;
  for (int k = 0; k < s; ++k) {
    if (!(w[k] > rtol * wmax) || w[k] <= 0.0) continue;
    ++rank;
    const double* vk = V.data() + (size_t)k * s;  // eigenvector k (column k)
    double* row = VtF.data() + (size_t)k * s;
    for (int i = 0; i < s; ++i) {
      const double vi = vk[i];
      if (vi == 0.0) continue;
      const double* fi = F + (size_t)i * s;
      for (int j = 0; j < s; ++j) row[j] += vi * fi[j];
    }
    for (int j = 0; j < s; ++j) row[j] /= w[k];
  }
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double v = 0.0;
      for (int k = 0; k < s; ++k) v += V[(size_t)k * s + i] * VtF[(size_t)k * s + j];
      C[(size_t)i * s + j] = v;
    }
  return rank;
}

}  // namespace lsamg

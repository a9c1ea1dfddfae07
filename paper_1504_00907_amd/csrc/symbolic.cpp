// Host symbolic setup: validation of the pattern, non-overlapping and expanded
// subdomain sets (Section 6: graph distance Delta in the stored pattern of A),
// conflict colouring of the multiplicative sweep, subdomain adjacency (block
// pattern of A0, Section 4), and the block-tridiagonal level structure used by
// the local factors.  Integer work only.
#include <algorithm>
#include <cstdlib>
#include <numeric>
#include <thread>

#include "common.hpp"
#include "symv_tile.hpp"

namespace ddg {

namespace {

void check_pattern(int64_t n, const int64_t* rp, const int32_t* ci) {
  DDG_REQUIRE(n > 0, DDG_ERR_INVALID_ARG, "n must be positive");
  DDG_REQUIRE(rp[0] == 0, DDG_ERR_INVALID_ARG, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i) {
    DDG_REQUIRE(rp[i + 1] >= rp[i], DDG_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
    bool diag = false;
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      int32_t c = ci[t];
      DDG_REQUIRE(c >= 0 && c < n, DDG_ERR_INVALID_ARG, "column index out of range in row " + std::to_string(i));
      if (t > rp[i]) DDG_REQUIRE(ci[t - 1] < c, DDG_ERR_INVALID_ARG, "columns must be strictly increasing in row " + std::to_string(i));
      if (c == i) diag = true;
    }
    DDG_REQUIRE(diag, DDG_ERR_INVALID_ARG, "missing diagonal entry in row " + std::to_string(i));
  }
  // structural symmetry
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      int32_t c = ci[t];
      const int32_t* b = ci + rp[c];
      const int32_t* e = ci + rp[c + 1];
      DDG_REQUIRE(std::binary_search(b, e, (int32_t)i), DDG_ERR_INVALID_ARG,
                  "pattern not symmetric at (" + std::to_string(i) + "," + std::to_string(c) + ")");
    }
  }
}

// Run f(i) for i in [0, count) over a few host threads.
template <class Fn>
void parallel_for(int32_t count, Fn&& f) {
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  int32_t nt = (int32_t)std::min<unsigned>(hw, (unsigned)std::max(1, count / 8));
  if (nt <= 1) {
    for (int32_t i = 0; i < count; ++i) f(i, 0);
    return;
  }
  std::vector<std::thread> th;
  std::vector<Error> errs(nt);
  std::vector<int> failed(nt, 0);
  for (int32_t t = 0; t < nt; ++t) {
    th.emplace_back([&, t]() {
      try {
        for (int32_t i = t; i < count; i += nt) f(i, t);
      } catch (const Error& e) {
        errs[t] = e;
        failed[t] = 1;
      }
    });
  }
  for (auto& x : th) x.join();
  for (int32_t t = 0; t < nt; ++t)
    if (failed[t]) throw errs[t];
}

}  // namespace

void build_symbolic(Symbolic& S, int64_t n, const int64_t* rp, const int32_t* ci,
                    const int32_t* part, int32_t n_parts, int32_t overlap, int32_t tile,
                    int32_t block_target) {
  check_pattern(n, rp, ci);
  DDG_REQUIRE(n_parts >= 1, DDG_ERR_INVALID_ARG, "n_parts must be >= 1");
  DDG_REQUIRE(overlap >= 0, DDG_ERR_INVALID_ARG, "overlap must be >= 0");
  DDG_REQUIRE(n < (int64_t)1 << 31, DDG_ERR_UNSUPPORTED, "n must fit int32 indices");
  S.n = n;
  S.nnz = rp[n];
  S.n_parts = n_parts;
  S.overlap = overlap;

  // --- non-overlapping sets (counting sort keeps ascending order)
  S.own_ptr.assign(n_parts + 1, 0);
  for (int64_t g = 0; g < n; ++g) {
    DDG_REQUIRE(part[g] >= 0 && part[g] < n_parts, DDG_ERR_INVALID_ARG, "partition id out of range at " + std::to_string(g));
    S.own_ptr[part[g] + 1]++;
  }
  for (int32_t i = 0; i < n_parts; ++i) {
    DDG_REQUIRE(S.own_ptr[i + 1] > 0, DDG_ERR_INVALID_ARG, "subdomain " + std::to_string(i) + " is empty");
    S.own_ptr[i + 1] += S.own_ptr[i];
  }
  S.own_idx.resize(n);
  {
    std::vector<int64_t> fill(S.own_ptr.begin(), S.own_ptr.end() - 1);
    for (int64_t g = 0; g < n; ++g) S.own_idx[fill[part[g]]++] = (int32_t)g;
  }
  S.max_own = 0;
  for (int32_t i = 0; i < n_parts; ++i)
    S.max_own = std::max<int32_t>(S.max_own, (int32_t)(S.own_ptr[i + 1] - S.own_ptr[i]));

  // --- expanded sets: breadth-first Delta levels over stored entries
  std::vector<std::vector<int32_t>> sets(n_parts);
  parallel_for(n_parts, [&](int32_t i, int) {
    std::vector<int32_t> cur(S.own_idx.begin() + S.own_ptr[i], S.own_idx.begin() + S.own_ptr[i + 1]);
    std::vector<int32_t> front = cur, next;
    std::vector<int32_t> all = cur;
    for (int32_t lev = 0; lev < overlap; ++lev) {
      next.clear();
      for (int32_t v : front)
        for (int64_t t = rp[v]; t < rp[v + 1]; ++t) next.push_back(ci[t]);
      std::sort(next.begin(), next.end());
      next.erase(std::unique(next.begin(), next.end()), next.end());
      std::vector<int32_t> fresh;
      std::set_difference(next.begin(), next.end(), all.begin(), all.end(), std::back_inserter(fresh));
      std::vector<int32_t> merged;
      merged.reserve(all.size() + fresh.size());
      std::merge(all.begin(), all.end(), fresh.begin(), fresh.end(), std::back_inserter(merged));
      all.swap(merged);
      front.swap(fresh);
      if (front.empty()) break;
    }
    sets[i].swap(all);
  });
  S.set_ptr.assign(n_parts + 1, 0);
  for (int32_t i = 0; i < n_parts; ++i) S.set_ptr[i + 1] = S.set_ptr[i] + (int64_t)sets[i].size();
  DDG_REQUIRE(S.set_ptr[n_parts] < ((int64_t)1 << 31), DDG_ERR_UNSUPPORTED, "sum of expanded sets too large");
  S.set_idx.resize(S.set_ptr[n_parts]);
  S.max_set = 0;
  for (int32_t i = 0; i < n_parts; ++i) {
    std::copy(sets[i].begin(), sets[i].end(), S.set_idx.begin() + S.set_ptr[i]);
    S.max_set = std::max<int32_t>(S.max_set, (int32_t)sets[i].size());
  }

  // --- membership (node -> subdomains whose expanded set contains it)
  std::vector<int64_t> mem_ptr(n + 1, 0);
  for (int64_t t = 0; t < (int64_t)S.set_idx.size(); ++t) mem_ptr[S.set_idx[t] + 1]++;
  for (int64_t g = 0; g < n; ++g) mem_ptr[g + 1] += mem_ptr[g];
  std::vector<int32_t> mem(S.set_idx.size());
  {
    std::vector<int64_t> fill(mem_ptr.begin(), mem_ptr.end() - 1);
    for (int32_t i = 0; i < n_parts; ++i)
      for (int64_t t = S.set_ptr[i]; t < S.set_ptr[i + 1]; ++t) mem[fill[S.set_idx[t]]++] = i;
  }

  // --- conflicts: j conflicts with i when set_j meets N[set_i]
  std::vector<std::vector<int32_t>> conf(n_parts);
  parallel_for(n_parts, [&](int32_t i, int) {
    std::vector<int32_t> js;
    for (int64_t t = S.set_ptr[i]; t < S.set_ptr[i + 1]; ++t) {
      int32_t v = S.set_idx[t];
      for (int64_t u = rp[v]; u < rp[v + 1]; ++u) {
        int32_t w = ci[u];  // w in N[set_i] (includes v itself through the diagonal)
        for (int64_t m = mem_ptr[w]; m < mem_ptr[w + 1]; ++m)
          if (mem[m] != i) js.push_back(mem[m]);
      }
    }
    std::sort(js.begin(), js.end());
    js.erase(std::unique(js.begin(), js.end()), js.end());
    conf[i].swap(js);
  });
  // --- greedy colouring in increasing subdomain id
  S.colour.assign(n_parts, -1);
  S.n_colours = 0;
  {
    std::vector<int32_t> stamp(n_parts + 1, -1);
    for (int32_t i = 0; i < n_parts; ++i) {
      for (int32_t j : conf[i])
        if (j < i) stamp[S.colour[j]] = i;
      int32_t c = 0;
      while (stamp[c] == i) ++c;
      S.colour[i] = c;
      S.n_colours = std::max(S.n_colours, c + 1);
    }
  }
  S.conf_ptr.assign(n_parts + 1, 0);
  for (int32_t i = 0; i < n_parts; ++i) S.conf_ptr[i + 1] = S.conf_ptr[i] + (int32_t)conf[i].size();
  S.conf_idx.resize(S.conf_ptr[n_parts]);
  for (int32_t i = 0; i < n_parts; ++i) std::copy(conf[i].begin(), conf[i].end(), S.conf_idx.begin() + S.conf_ptr[i]);
  S.colour_ptr.assign(S.n_colours + 1, 0);
  for (int32_t i = 0; i < n_parts; ++i) S.colour_ptr[S.colour[i] + 1]++;
  for (int32_t c = 0; c < S.n_colours; ++c) S.colour_ptr[c + 1] += S.colour_ptr[c];
  S.colour_subs.resize(n_parts);
  {
    std::vector<int32_t> fill(S.colour_ptr.begin(), S.colour_ptr.end() - 1);
    for (int32_t i = 0; i < n_parts; ++i) S.colour_subs[fill[S.colour[i]]++] = i;
  }

  // --- subdomain adjacency through stored entries (block pattern of A0)
  S.nbr_ptr.assign(n_parts + 1, 0);
  std::vector<std::vector<int32_t>> nb(n_parts);
  parallel_for(n_parts, [&](int32_t i, int) {
    std::vector<int32_t> js;
    for (int64_t t = S.own_ptr[i]; t < S.own_ptr[i + 1]; ++t) {
      int32_t g = S.own_idx[t];
      for (int64_t u = rp[g]; u < rp[g + 1]; ++u) js.push_back(part[ci[u]]);
    }
    std::sort(js.begin(), js.end());
    js.erase(std::unique(js.begin(), js.end()), js.end());
    nb[i].swap(js);
  });
  for (int32_t i = 0; i < n_parts; ++i) S.nbr_ptr[i + 1] = S.nbr_ptr[i] + (int32_t)nb[i].size();
  S.nbr_idx.resize(S.nbr_ptr[n_parts]);
  for (int32_t i = 0; i < n_parts; ++i) std::copy(nb[i].begin(), nb[i].end(), S.nbr_idx.begin() + S.nbr_ptr[i]);

  // --- local structure: block-tridiagonal levels in the ascending local order
  struct Local {
    std::vector<int32_t> bstart, bsize;
    std::vector<int64_t> lo_cnt, up_cnt, in_cnt;  // per local row
    std::vector<int32_t> lo_col, up_col, in_col;
    std::vector<int64_t> lo_pos, up_pos, in_pos;
  };
  std::vector<Local> loc(n_parts);
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::vector<int32_t>> lmap(hw, std::vector<int32_t>());
  // choose tile from the typical level width when not given
  S.tile = tile;
  parallel_for(n_parts, [&](int32_t i, int tid) {
    auto& map = lmap[tid];
    if ((int64_t)map.size() != n) map.assign(n, -1);
    int32_t* set = S.set_idx.data() + S.set_ptr[i];
    int32_t ni = (int32_t)(S.set_ptr[i + 1] - S.set_ptr[i]);
    // Level structure of the local rows taken in the order `ord` (global ids):
    // greedy boundaries (rows of level m+1 and later may only reach back to
    // level m, so s_{m+1} = max(s_m + 1, min{j : min_{j' >= j} first(j') >= s_m})),
    // then consecutive levels merged (tiny ones absorbed, grown up to the target).
    const int32_t target = block_target > 0 ? block_target : 0;
    const int32_t min_rows = 16;
    auto levels_of = [&](const int32_t* ord, std::vector<int32_t>& bstart, std::vector<int32_t>& bsize) {
      for (int32_t j = 0; j < ni; ++j) map[ord[j]] = j;
      std::vector<int32_t> first(ni);
      for (int32_t j = 0; j < ni; ++j) {
        int32_t g = ord[j];
        int32_t f = j;
        for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
          int32_t lc = map[ci[t]];
          if (lc >= 0) f = std::min(f, lc);
        }
        first[j] = f;
      }
      std::vector<int32_t> suf(ni + 1, INT32_MAX);
      for (int32_t j = ni - 1; j >= 0; --j) suf[j] = std::min(suf[j + 1], first[j]);
      std::vector<int32_t> bnd{0};
      int32_t j = 0;
      while (bnd.back() < ni) {
        int32_t cur = bnd.back();
        while (j < ni && suf[j] < cur) ++j;  // suf is non-decreasing
        bnd.push_back(std::min(std::max(cur + 1, j), ni));
      }
      bstart.clear();
      bsize.clear();
      int32_t s0 = 0;
      for (size_t m = 1; m < bnd.size(); ++m) {
        int32_t e = bnd[m];
        bool last = (m + 1 == bnd.size());
        int32_t size = e - s0;
        int32_t next_size = last ? 0 : bnd[m + 1] - e;
        bool absorb = !last && (size < min_rows || (target > 0 && size + next_size <= target));
        if (!absorb) {
          bstart.push_back(s0);
          bsize.push_back(size);
          s0 = e;
        }
      }
      for (int32_t jj = 0; jj < ni; ++jj) map[ord[jj]] = -1;
      double cost = 0.0;  // factor entries ~ sum of squared level sizes
      for (int32_t b : bsize) cost += (double)b * b;
      return cost;
    };
    Local& L = loc[i];
    // candidate 1: ascending global order
    levels_of(set, L.bstart, L.bsize);
    // candidate 2, only for subdomains whose natural levels are very wide (irregular
    // shapes): breadth-first levels of the local graph from a pseudo-peripheral row
    // (rows sorted by distance, then global id), kept when it narrows the widest level.
    // Narrow natural levels are kept even when the breadth-first ones store fewer
    // entries: the sweep's cost per level is mostly latency, so more levels cost more.
    const int32_t wide_level = 1024;
    int32_t max_nat = 0;
    for (int32_t b : L.bsize) max_nat = std::max(max_nat, b);
    if (max_nat > wide_level && ni > 2 * min_rows) {
      for (int32_t j = 0; j < ni; ++j) map[set[j]] = j;
      std::vector<int32_t> dist(ni), queue(ni);
      auto bfs = [&](int32_t src) {
        std::fill(dist.begin(), dist.end(), -1);
        int32_t head = 0, tail = 0;
        dist[src] = 0;
        queue[tail++] = src;
        while (head < tail) {
          int32_t v = queue[head++];
          int32_t g = set[v];
          for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
            int32_t w = map[ci[t]];
            if (w >= 0 && dist[w] < 0) {
              dist[w] = dist[v] + 1;
              queue[tail++] = w;
            }
          }
        }
        return tail;  // rows reached
      };
      auto degree = [&](int32_t v) {
        int32_t g = set[v], d = 0;
        for (int64_t t = rp[g]; t < rp[g + 1]; ++t) d += map[ci[t]] >= 0;
        return d;
      };
      int32_t src = 0;
      for (int32_t v = 1; v < ni; ++v)
        if (degree(v) < degree(src)) src = v;
      int32_t ecc = -1;
      bool connected = true;
      for (int it = 0; it < 6; ++it) {
        if (bfs(src) != ni) {
          connected = false;
          break;
        }
        int32_t e = *std::max_element(dist.begin(), dist.end());
        if (e <= ecc) break;
        ecc = e;
        int32_t best = -1;
        for (int32_t v = 0; v < ni; ++v)
          if (dist[v] == e && (best < 0 || degree(v) < degree(best))) best = v;
        if (best == src) break;
        src = best;
      }
      if (connected && bfs(src) == ni) {
        std::vector<int32_t> ord(set, set + ni);
        std::vector<int32_t> key(ni);
        for (int32_t v = 0; v < ni; ++v) key[v] = dist[v];
        std::vector<int32_t> idx(ni);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        for (int32_t v = 0; v < ni; ++v) ord[v] = set[idx[v]];
        for (int32_t jj = 0; jj < ni; ++jj) map[set[jj]] = -1;
        std::vector<int32_t> bs2, sz2;
        levels_of(ord.data(), bs2, sz2);
        int32_t max_bfs = 0;
        for (int32_t b : sz2) max_bfs = std::max(max_bfs, b);
        if (max_bfs < max_nat) {
          std::copy(ord.begin(), ord.end(), set);
          L.bstart.swap(bs2);
          L.bsize.swap(sz2);
        }
      } else {
        for (int32_t jj = 0; jj < ni; ++jj) map[set[jj]] = -1;
      }
    }
    for (int32_t j = 0; j < ni; ++j) map[set[j]] = j;
    // block id of each local row
    std::vector<int32_t> blk(ni);
    for (size_t b = 0; b < L.bstart.size(); ++b)
      for (int32_t r = L.bstart[b]; r < L.bstart[b] + L.bsize[b]; ++r) blk[r] = (int32_t)b;
    L.lo_cnt.assign(ni, 0);
    L.up_cnt.assign(ni, 0);
    L.in_cnt.assign(ni, 0);
    for (int32_t jj = 0; jj < ni; ++jj) {
      int32_t g = set[jj];
      for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
        int32_t lc = map[ci[t]];
        if (lc < 0) continue;
        int32_t d = blk[lc] - blk[jj];
        DDG_REQUIRE(d >= -1 && d <= 1, DDG_ERR_HIP, "internal: level structure not block tridiagonal");
        if (d < 0) { L.lo_col.push_back(lc); L.lo_pos.push_back(t); L.lo_cnt[jj]++; }
        else if (d > 0) { L.up_col.push_back(lc); L.up_pos.push_back(t); L.up_cnt[jj]++; }
        else { L.in_col.push_back(lc); L.in_pos.push_back(t); L.in_cnt[jj]++; }
      }
    }
    for (int32_t jj = 0; jj < ni; ++jj) map[set[jj]] = -1;
  });

  // --- concatenate
  S.sub_blk_ptr.assign(n_parts + 1, 0);
  for (int32_t i = 0; i < n_parts; ++i) S.sub_blk_ptr[i + 1] = S.sub_blk_ptr[i] + (int32_t)loc[i].bstart.size();
  int32_t nb_tot = S.sub_blk_ptr[n_parts];
  S.blk_start.resize(nb_tot);
  S.blk_size.resize(nb_tot);
  S.blk_foff.resize(nb_tot + 1);
  S.max_blk = 0;
  S.max_blocks = 0;
  for (int32_t i = 0; i < n_parts; ++i) {
    std::copy(loc[i].bstart.begin(), loc[i].bstart.end(), S.blk_start.begin() + S.sub_blk_ptr[i]);
    std::copy(loc[i].bsize.begin(), loc[i].bsize.end(), S.blk_size.begin() + S.sub_blk_ptr[i]);
    S.max_blocks = std::max<int32_t>(S.max_blocks, (int32_t)loc[i].bstart.size());
    for (int32_t b : loc[i].bsize) S.max_blk = std::max(S.max_blk, b);
  }
  if (S.tile <= 0) {
    // automatic: the typical level width decides the tile edge.  Edge 64 streams about
    // a quarter faster per byte than 32 (measured, compact diagonal tiles), so it wins
    // once its padding costs less than that: from about 168 rows
    std::vector<int32_t> w(S.blk_size);
    std::nth_element(w.begin(), w.begin() + w.size() / 2, w.end());
    int32_t med = w[w.size() / 2];
    S.tile = med >= 168 ? 64 : (med >= 48 ? 32 : 16);
  }
  DDG_REQUIRE(S.tile == 16 || S.tile == 32 || S.tile == 64, DDG_ERR_INVALID_ARG, "tile must be 16, 32 or 64");
  int64_t off = 0;
  for (int32_t b = 0; b < nb_tot; ++b) {
    S.blk_foff[b] = off;
    off += level_elems(S.blk_size[b], S.tile);  // lower tiles, diagonal tiles compact
  }
  S.blk_foff[nb_tot] = off;
  S.fac_elems = off;
  // Middle level of the twisted factorisation: the top chain eliminates levels
  // 0..m-1, the bottom chain K-1..m+1, and a solve runs both chains down, the middle
  // level, then both back.  A level costs its tiles plus a fixed latency (in tile
  // units); m minimises 2 max(top, bottom) + middle, nearest (K-1)/2 on ties.  Any m
  // gives the same exact local solve.
  S.sub_mid.assign(n_parts, 0);
  {
    const int64_t lat = 16;
    for (int32_t i = 0; i < n_parts; ++i) {
      const int32_t kb0 = S.sub_blk_ptr[i], K = S.sub_blk_ptr[i + 1] - kb0;
      std::vector<int64_t> pre(K + 1, 0);
      for (int32_t k = 0; k < K; ++k) pre[k + 1] = pre[k] + lat + tiles_for(S.blk_size[kb0 + k], S.tile);
      int32_t best = (K - 1) / 2;
      int64_t best_cost = -1;
      for (int32_t m = 0; m < K; ++m) {
        const int64_t top = pre[m], bot = pre[K] - pre[m + 1];
        const int64_t cost = 2 * std::max(top, bot) + (pre[m + 1] - pre[m]);
        const int32_t d = std::abs(m - (K - 1) / 2), db = std::abs(best - (K - 1) / 2);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && d < db)) {
          best = m;
          best_cost = cost;
        }
      }
      S.sub_mid[i] = best;
    }
  }

  int64_t rows = S.set_ptr[n_parts];
  // ELL couplings
  S.cl = 0;
  S.cu = 0;
  for (int32_t i = 0; i < n_parts; ++i)
    for (size_t j = 0; j < loc[i].lo_cnt.size(); ++j) {
      S.cl = std::max<int32_t>(S.cl, (int32_t)loc[i].lo_cnt[j]);
      S.cu = std::max<int32_t>(S.cu, (int32_t)loc[i].up_cnt[j]);
    }
  const int32_t cl = std::max(1, S.cl), cu = std::max(1, S.cu);
  S.cl = cl;
  S.cu = cu;
  S.lo_col.assign(rows * cl, -1);
  S.lo_pos.assign(rows * cl, -1);
  S.up_col.assign(rows * cu, -1);
  S.up_pos.assign(rows * cu, -1);
  parallel_for(n_parts, [&](int32_t i, int) {
    const Local& L = loc[i];
    int64_t lo_o = 0, up_o = 0;
    for (size_t j = 0; j < L.lo_cnt.size(); ++j) {
      const int64_t row = S.set_ptr[i] + (int64_t)j;
      for (int64_t c = 0; c < L.lo_cnt[j]; ++c) {
        S.lo_col[row * cl + c] = L.lo_col[lo_o];
        S.lo_pos[row * cl + c] = L.lo_pos[lo_o];
        ++lo_o;
      }
      for (int64_t c = 0; c < L.up_cnt[j]; ++c) {
        S.up_col[row * cu + c] = L.up_col[up_o];
        S.up_pos[row * cu + c] = L.up_pos[up_o];
        ++up_o;
      }
    }
  });
  // sliced copy of the couplings for the sweep (rows with more than kCplRegs couplings)
  S.sliced = S.cl > kCplRegs || S.cu > kCplRegs;
  if (S.sliced) {
    S.blk_slice.assign(nb_tot + 1, 0);
    for (int32_t b = 0; b < nb_tot; ++b) S.blk_slice[b + 1] = S.blk_slice[b] + (S.blk_size[b] + 63) / 64;
    const int32_t nsl = S.blk_slice[nb_tot];
    for (int32_t i = 0; i < n_parts; ++i)
      S.max_sub_slices = std::max(S.max_sub_slices, S.blk_slice[S.sub_blk_ptr[i + 1]] - S.blk_slice[S.sub_blk_ptr[i]]);
    S.sl_row.assign(nsl, 0);
    S.sl_rows.assign(nsl, 0);
    std::vector<int32_t> wlo(nsl, 0), wup(nsl, 0), lrow(nsl, 0);
    parallel_for(n_parts, [&](int32_t i, int) {
      for (int32_t b = S.sub_blk_ptr[i]; b < S.sub_blk_ptr[i + 1]; ++b)
        for (int32_t sl = S.blk_slice[b]; sl < S.blk_slice[b + 1]; ++sl) {
          const int32_t r0 = S.blk_start[b] + 64 * (sl - S.blk_slice[b]);
          const int32_t nr = std::min(64, S.blk_start[b] + S.blk_size[b] - r0);
          S.sl_row[sl] = S.set_ptr[i] + r0;
          S.sl_rows[sl] = nr;
          lrow[sl] = r0;
          for (int32_t l = 0; l < nr; ++l) {
            wlo[sl] = std::max<int32_t>(wlo[sl], (int32_t)loc[i].lo_cnt[r0 + l]);
            wup[sl] = std::max<int32_t>(wup[sl], (int32_t)loc[i].up_cnt[r0 + l]);
          }
        }
    });
    S.sl_lo_off.assign(nsl + 1, 0);
    S.sl_up_off.assign(nsl + 1, 0);
    for (int32_t sl = 0; sl < nsl; ++sl) {
      S.sl_lo_off[sl + 1] = S.sl_lo_off[sl] + 64 * (int64_t)wlo[sl];
      S.sl_up_off[sl + 1] = S.sl_up_off[sl] + 64 * (int64_t)wup[sl];
    }
    S.sl_lo_col.assign(S.sl_lo_off[nsl], 0);
    S.sl_up_col.assign(S.sl_up_off[nsl], 0);
    // a padding entry points at its own row: the workgroup that solves a level
    // always holds that level's rows, so the zero product never reads a stale value
    auto fill = [&](int32_t sl, const std::vector<int32_t>& ell, int32_t c, const std::vector<int64_t>& off,
                    std::vector<int32_t>& out) {
      const int32_t w = (int32_t)((off[sl + 1] - off[sl]) / 64);
      for (int32_t l = 0; l < S.sl_rows[sl]; ++l)
        for (int32_t q = 0; q < w; ++q) {
          const int32_t col = ell[(S.sl_row[sl] + l) * c + q];
          out[off[sl] + 64 * q + l] = col >= 0 ? col : lrow[sl] + l;
        }
    };
    parallel_for(nsl, [&](int32_t sl, int) {
      fill(sl, S.lo_col, cl, S.sl_lo_off, S.sl_lo_col);
      fill(sl, S.up_col, cu, S.sl_up_off, S.sl_up_col);
    });
  }
  // same-level entries (setup only) in CSR form
  S.in_ptr.assign(rows + 1, 0);
  for (int32_t i = 0; i < n_parts; ++i)
    for (size_t j = 0; j < loc[i].in_cnt.size(); ++j) S.in_ptr[S.set_ptr[i] + j + 1] = loc[i].in_cnt[j];
  for (int64_t r = 0; r < rows; ++r) S.in_ptr[r + 1] += S.in_ptr[r];
  S.in_col.resize(S.in_ptr[rows]);
  S.in_pos.resize(S.in_ptr[rows]);
  for (int32_t i = 0; i < n_parts; ++i) {
    const int64_t o = S.in_ptr[S.set_ptr[i]];
    std::copy(loc[i].in_col.begin(), loc[i].in_col.end(), S.in_col.begin() + o);
    std::copy(loc[i].in_pos.begin(), loc[i].in_pos.end(), S.in_pos.begin() + o);
  }
}

}  // namespace ddg

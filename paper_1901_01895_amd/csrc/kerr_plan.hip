// Host-side plan of the packed matrix-core Kerr contraction (no device
// code): the order of the pairs, the zero blocks of the packed tensor, and
// the passes of row tiles with the k-steps each of them multiplies.
// setup_mfma builds the device tables from it; mmnlse_kerr_plan returns it
// without a device.
//
// Packed form (symmetric S): rows r = (p <= n), columns q = (l <= m),
// Sp[r][q] = w_q S[p, l, m, n] with w_q = 2 for l < m.  Rows are sorted by
// their zero pattern over q (equal patterns adjacent), the groups of equal
// rows chained greedily by Hamming distance, and the same order is used for
// the columns.  A block of 32 rows x one k-step (8 columns FP32, 16 split)
// is multiplied only when it holds a nonzero entry.  On the FP32 path the
// row tiles are then cut from that row order by a dynamic program: a tile
// takes 1 to 32 consecutive rows (the rest of its 32 slots are zero padding
// rows), so a tile need not straddle two row groups with different zero
// blocks.

#include <algorithm>
#include <random>
#include <cstdlib>
#include <utility>
#include <vector>

#include "common.h"

namespace mmnlse {

int mfma_tile_width(int M, int T) { return M <= 64 && T % 128 == 0 ? 128 : 32; }

float packed_entry(const float *S, int M, int ar, int br, int aq, int bq) {
  const float w = aq < bq ? 2.f : 1.f;
  return w * S[(((size_t)ar * M + aq) * M + bq) * M + br];
}

// Place the rows of every tile so that both lane halves can scatter at once.
// In the 32 x 32 MFMA accumulator lane half h holds rows 8g + 4h + j
// (g, j < 4) of its 32 samples, so at each of its 16 steps the scatter
// updates the modes of slot 8g + j (half 0) and slot 8g + 4 + j (half 1)
// in the same instructions.  Rows are matched into 16 such pairs with
// different p and different n (padding rows match anything), greedily over
// up to 64 seeded orders; which slot of a tile holds which of its rows does
// not change the tile's blocks or k-lists.  A tile without such a matching
// keeps its order and the scatter where the halves take turns.
static void arrange_tile_rows(KerrPlan &kp) {
  kp.both.assign(kp.nrt, 0);
  std::mt19937 rng(20190105u);
  for (int t = 0; t < kp.nrt; ++t) {
    const size_t s0 = (size_t)t * 32;
    std::vector<int> real;
    for (int i = 0; i < 32; ++i)
      if (kp.rows[s0 + i] >= 0) real.push_back(i);
    const int r = (int)real.size();
    const int need = std::max(0, r - 16);  // real-real pairs needed so the rest fit the padding
    auto fits = [&](int x, int y) { return kp.ra[s0 + x] != kp.ra[s0 + y] && kp.rb[s0 + x] != kp.rb[s0 + y]; };
    std::vector<std::pair<int, int>> best;
    bool ok = false;
    std::vector<int> order = real;
    for (int attempt = 0; attempt < 64 && !ok; ++attempt) {
      if (attempt) std::shuffle(order.begin(), order.end(), rng);
      std::vector<char> used(32, 0);
      std::vector<std::pair<int, int>> pr;
      for (int x : order) {
        if (used[x]) continue;
        for (int y : order)
          if (y != x && !used[y] && fits(x, y)) {
            used[x] = used[y] = 1;
            pr.push_back({x, y});
            break;
          }
      }
      if ((int)pr.size() >= need) {
        ok = true;
        best.swap(pr);
      }
    }
    if (!ok) continue;
    // slot pairs (8g + j, 8g + 4 + j): matched pairs first, then single rows
    // with padding partners, then padding
    std::vector<char> placed(32, 0);
    std::vector<std::pair<int, int>> all = best;
    for (auto &q : best) placed[q.first] = placed[q.second] = 1;
    for (int x : real)
      if (!placed[x]) all.push_back({x, -1});
    std::vector<int> nrow(32, -1), na(32, 0), nb(32, 0);
    for (size_t k = 0; k < all.size(); ++k) {
      const int g = (int)k / 4, j = (int)k % 4;
      const int sl[2] = {8 * g + j, 8 * g + 4 + j};
      const int src[2] = {all[k].first, all[k].second};
      for (int h = 0; h < 2; ++h)
        if (src[h] >= 0) {
          nrow[sl[h]] = kp.rows[s0 + src[h]];
          na[sl[h]] = kp.ra[s0 + src[h]];
          nb[sl[h]] = kp.rb[s0 + src[h]];
        }
    }
    for (int i = 0; i < 32; ++i) {
      kp.rows[s0 + i] = nrow[i];
      kp.ra[s0 + i] = na[i];
      kp.rb[s0 + i] = nb[i];
    }
    kp.both[t] = 1;
  }
}

void plan_kerr(const float *S, int M, bool split, KerrPlan &kp) {
  const int P = M * (M + 1) / 2;
  const int Ppad = (P + 31) / 32 * 32;  // columns: a multiple of the 8 and 16 column k-steps
  kp.P = P;
  kp.Ppad = Ppad;
  kp.kw = split ? 16 : 8;
  kp.nk = Ppad / kp.kw;
  std::vector<int> na(P), nb(P);
  {
    int r = 0;
    for (int i = 0; i < M; ++i)
      for (int j = i; j < M; ++j, ++r) {
        na[r] = i;
        nb[r] = j;
      }
  }
  // zero pattern of every row over the natural column order
  const int words = (P + 63) / 64;
  std::vector<uint64_t> mask((size_t)P * words, 0);
  double nonzero = 0;
  for (int r = 0; r < P; ++r)
    for (int q = 0; q < P; ++q)
      if (packed_entry(S, M, na[r], nb[r], na[q], nb[q]) != 0.f) {
        mask[(size_t)r * words + q / 64] |= 1ull << (q % 64);
        nonzero += 1;
      }
  auto row = [&](int r) { return mask.data() + (size_t)r * words; };
  std::vector<int> perm(P);
  for (int i = 0; i < P; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
    return std::lexicographical_compare(row(x), row(x) + words, row(y), row(y) + words);
  });
  // A row tile that straddles two groups of equal rows multiplies the union
  // of their patterns, so neighbouring groups should be similar: chain the
  // groups greedily, each next group the one nearest (Hamming distance) to
  // the last (skipped when that search would be too long).
  {
    std::vector<int> gs;
    for (int i = 0; i < P; ++i)
      if (i == 0 || !std::equal(row(perm[i]), row(perm[i]) + words, row(perm[i - 1]))) gs.push_back(i);
    gs.push_back(P);
    const int G = (int)gs.size() - 1;
    if (G > 2 && (double)G * G * words <= 2e8) {
      std::vector<char> used(G, 0);
      std::vector<int> order{0};
      used[0] = 1;
      for (int n = 1; n < G; ++n) {
        const uint64_t *cur = row(perm[gs[order.back()]]);
        int best = -1;
        long bestd = -1;
        for (int g = 0; g < G; ++g) {
          if (used[g]) continue;
          const uint64_t *o = row(perm[gs[g]]);
          long d = 0;
          for (int w = 0; w < words; ++w) d += __builtin_popcountll(cur[w] ^ o[w]);
          if (best < 0 || d < bestd) {
            best = g;
            bestd = d;
          }
        }
        used[best] = 1;
        order.push_back(best);
      }
      std::vector<int> p2;
      p2.reserve(P);
      for (int g : order)
        for (int i = gs[g]; i < gs[g + 1]; ++i) p2.push_back(perm[i]);
      perm.swap(p2);
    }
  }
  kp.perm = perm;
  kp.a.assign(Ppad, 0);
  kp.b.assign(Ppad, 0);
  std::vector<int> inv(P);
  for (int i = 0; i < P; ++i) {
    kp.a[i] = na[perm[i]];
    kp.b[i] = nb[perm[i]];
    inv[perm[i]] = i;
  }
  // k-steps (of the permuted columns) in which each row, in row order, holds a nonzero
  const int nk = kp.nk, kw = kp.kw;
  const int kwords = (nk + 63) / 64;
  std::vector<uint64_t> rk((size_t)P * kwords, 0);
  for (int rp = 0; rp < P; ++rp) {
    const uint64_t *m = row(perm[rp]);
    uint64_t *o = rk.data() + (size_t)rp * kwords;
    for (int w = 0; w < words; ++w)
      for (uint64_t bits = m[w]; bits; bits &= bits - 1) {
        const int k = inv[64 * w + __builtin_ctzll(bits)] / kw;
        o[k / 64] |= 1ull << (k % 64);
      }
  }
  // Row tiles: fixed runs of 32 rows, or, when that costs more, the cut of
  // the row order into tiles of 1..32 rows minimising the listed k-steps
  // plus kTilePenalty per tile (a tile's scatter and B formation cost about
  // that many k-steps of matrix-core work).
  constexpr int kTilePenalty = 2;
  const bool cut_fp32 = !split && (double)nonzero < (double)P * P;
  std::vector<int> cut;  // tile boundaries in the row order
  {
    std::vector<uint64_t> u(kwords);
    auto cost_of = [&](int i, int j) {  // rows i .. j-1 as one tile
      std::fill(u.begin(), u.end(), 0ull);
      for (int r = i; r < j; ++r)
        for (int w = 0; w < kwords; ++w) u[w] |= rk[(size_t)r * kwords + w];
      long c = kTilePenalty;
      for (int w = 0; w < kwords; ++w) c += __builtin_popcountll(u[w]);
      return c;
    };
    long fixed = 0;
    for (int i = 0; i < P; i += 32) fixed += cost_of(i, std::min(P, i + 32));
    std::vector<long> best(P + 1, -1);
    std::vector<int> from(P + 1, 0);
    best[0] = 0;
    // a dense tensor keeps the fixed tiles; so does the split path, whose
    // passes pair tiles to share the costlier bf16 B formation (measured on
    // the 36-mode tensor: FP32 3.22 -> 3.00 ms per step with the cut tiles,
    // split 1.62 -> 1.70)
    if (cut_fp32) {
      for (int i = 0; i < P; ++i) {
        std::fill(u.begin(), u.end(), 0ull);
        for (int j = i + 1; j <= std::min(P, i + 32); ++j) {
          for (int w = 0; w < kwords; ++w) u[w] |= rk[(size_t)(j - 1) * kwords + w];
          long c = best[i] + kTilePenalty;
          for (int w = 0; w < kwords; ++w) c += __builtin_popcountll(u[w]);
          if (best[j] < 0 || c < best[j]) {
            best[j] = c;
            from[j] = i;
          }
        }
      }
    }
    if (best[P] >= 0 && best[P] < fixed) {
      for (int j = P; j > 0; j = from[j]) cut.push_back(j);
      cut.push_back(0);
      std::reverse(cut.begin(), cut.end());
    } else {
      for (int i = 0; i < P; i += 32) cut.push_back(i);
      cut.push_back(P);
    }
  }
  const int nrt = (int)cut.size() - 1;
  kp.nrt = nrt;
  kp.rows.assign((size_t)nrt * 32, -1);
  kp.ra.assign((size_t)nrt * 32, 0);
  kp.rb.assign((size_t)nrt * 32, 0);
  // tiles holding a nonzero in each column (natural column index)
  const int twords = (nrt + 63) / 64;
  std::vector<uint64_t> ct((size_t)P * twords, 0);
  for (int t = 0; t < nrt; ++t)
    for (int i = cut[t]; i < cut[t + 1]; ++i) {
      const size_t slot = (size_t)t * 32 + (i - cut[t]);
      kp.rows[slot] = perm[i];
      kp.ra[slot] = na[perm[i]];
      kp.rb[slot] = nb[perm[i]];
      const uint64_t *m = row(perm[i]);
      for (int w = 0; w < words; ++w)
        for (uint64_t bits = m[w]; bits; bits &= bits - 1)
          ct[(size_t)(64 * w + __builtin_ctzll(bits)) * twords + t / 64] |= 1ull << (t % 64);
    }
  std::vector<uint64_t>().swap(mask);
  // Column positions: the sorted order in k-steps of kw columns or, with
  // the cut row tiles, the cut of that order into k-steps of 1..kw columns
  // (the other positions are zero padding columns) that minimises the listed
  // (tile, k-step) blocks plus half a block per k-step.  Padded to a
  // multiple of 32 positions.
  std::vector<int> cols;
  if (cut_fp32) {
    std::vector<uint64_t> u(twords);
    auto blocks = [&](int i, int j) {  // tiles listing the k-step of columns i .. j-1
      std::fill(u.begin(), u.end(), 0ull);
      for (int c = i; c < j; ++c)
        for (int w = 0; w < twords; ++w) u[w] |= ct[(size_t)perm[c] * twords + w];
      long n = 0;
      for (int w = 0; w < twords; ++w) n += __builtin_popcountll(u[w]);
      return n;
    };
    long fixed = 0;
    for (int i = 0; i < P; i += kw) fixed += 2 * blocks(i, std::min(P, i + kw)) + 1;
    std::vector<long> best(P + 1, -1);
    std::vector<int> from(P + 1, 0);
    best[0] = 0;
    for (int i = 0; i < P; ++i)
      for (int j = i + 1; j <= std::min(P, i + kw); ++j) {
        const long c = best[i] + 2 * blocks(i, j) + 1;
        if (best[j] < 0 || c < best[j]) {
          best[j] = c;
          from[j] = i;
        }
      }
    if (best[P] < fixed) {
      std::vector<int> cc;
      for (int j = P; j > 0; j = from[j]) cc.push_back(j);
      cc.push_back(0);
      std::reverse(cc.begin(), cc.end());
      for (size_t k = 0; k + 1 < cc.size(); ++k) {
        for (int c = cc[k]; c < cc[k + 1]; ++c) cols.push_back(perm[c]);
        while (cols.size() % kw) cols.push_back(-1);
      }
    }
  }
  if (cols.empty()) cols = perm;
  while (cols.size() % 32) cols.push_back(-1);
  kp.Ppad = (int)cols.size();
  kp.nk = kp.Ppad / kw;
  kp.cols = cols;
  kp.a.assign(kp.Ppad, 0);
  kp.b.assign(kp.Ppad, 0);
  for (int j = 0; j < kp.Ppad; ++j)
    if (cols[j] >= 0) {
      kp.a[j] = na[cols[j]];
      kp.b[j] = nb[cols[j]];
    }
  const int nkc = kp.nk;
  std::vector<uint8_t> occ((size_t)nrt * nkc, 0);
  for (int j = 0; j < kp.Ppad; ++j)
    if (cols[j] >= 0)
      for (int w = 0; w < twords; ++w)
        for (uint64_t bits = ct[(size_t)cols[j] * twords + w]; bits; bits &= bits - 1)
          occ[(size_t)(64 * w + __builtin_ctzll(bits)) * nkc + j / kw] = 1;
  // Row tiles per pass.  RTM = 4 halves the B formations per output row but
  // needs 128 accumulator registers, which costs the second wave per SIMD;
  // that wave exists only for M <= 64 (two 128-sample workgroups fit one
  // CU's LDS), so RTM = 2 there and 4 above (measured: 36 modes 4.5 vs 5.8 ms
  // per step, 120 modes 1441 vs 1167).  MMNLSE_MFMA_RT=2 or 4 overrides.
  const char *rt_env = std::getenv("MMNLSE_MFMA_RT");
  const int rt_req = rt_env ? std::atoi(rt_env) : 0;
  const int rtm = rt_req == 2 || rt_req == 4 ? rt_req : (M > 64 ? 4 : 2);
  kp.rtm = rtm;
  // listed k-steps of tiles rt0 .. rt0+nt-1 (union of their nonzero blocks)
  auto listed = [&](int rt0, int nt, std::vector<int32_t> *out) {
    int len = 0;
    for (int k = 0; k < nkc; ++k) {
      bool any = false;
      for (int t = 0; t < nt; ++t) any = any || occ[(size_t)(rt0 + t) * nkc + k];
      if (any) {
        ++len;
        if (out) out->push_back(k);
      }
    }
    return len;
  };
  // Passes of 1, 2 or RTM tiles, chosen by a cost model in cycles per listed
  // k-step of one wave: matrix-core time per tile (FP32: 8 32x32x2 products of
  // 64 cycles; split: 6 32x32x16 products of 32) plus forming the B fragment
  // once per pass (about 40 resp. 110 vector instructions of 4 cycles).  A
  // pass shares B between its tiles but multiplies the union of their lists,
  // so tiles with different zero patterns are better run alone.  Minimum
  // total cost over the row tiles by dynamic programming.
  const double mc = split ? 192.0 : 512.0, bc = split ? 440.0 : 160.0;
  std::vector<double> best(nrt + 1, 0.0);
  std::vector<int> take(nrt + 1, 1);
  for (int i = 1; i <= nrt; ++i) {
    best[i] = best[i - 1] + listed(i - 1, 1, nullptr) * (mc + bc);
    for (int nt = 2; nt <= rtm; nt *= 2) {
      if (i < nt) break;
      const double c = best[i - nt] + listed(i - nt, nt, nullptr) * (nt * mc + bc);
      if (c < best[i]) {
        best[i] = c;
        take[i] = nt;
      }
    }
  }
  std::vector<std::pair<int, int>> runs;
  for (int i = nrt; i > 0; i -= take[i]) runs.push_back({i - take[i], take[i]});
  kp.passes.clear();
  kp.klist.clear();
  double executed = 0;
  for (auto it = runs.rbegin(); it != runs.rend(); ++it) {
    const int off = (int)kp.klist.size();
    const int len = listed(it->first, it->second, &kp.klist);
    kp.passes.push_back(make_int4(it->first, it->second, off, len));
    executed += (double)it->second * 32 * kw * len;
  }
  kp.entries[0] = (double)P * P;
  kp.entries[1] = executed;
  kp.entries[2] = nonzero;
  kp.occ.swap(occ);
  arrange_tile_rows(kp);
}

void plan_groups(const KerrPlan &kp, int nw, int rw, int kc, KerrGroups &g) {
  const int nrt = kp.nrt, nk = kp.nk;
  g = KerrGroups();
  g.nw = nw;
  g.rw = rw;
  g.kc = kc;
  if (nrt == 0) return;
  const int cap = nw * rw;
  const int ng = (nrt + cap - 1) / cap;
  g.ngroups = ng;
  g.tiles.assign((size_t)ng * nw * rw, -1);
  auto occ = [&](int t, int k) { return (int)kp.occ[(size_t)t * nk + k]; };
  for (int gi = 0; gi < ng; ++gi) {
    const int t0 = (int)((long)gi * nrt / ng), t1 = (int)((long)(gi + 1) * nrt / ng), n = t1 - t0;
    std::vector<int> ks;  // listed k-steps: some tile of the group holds a nonzero block
    bool full = true;
    for (int k = 0; k < nk; ++k) {
      int c = 0;
      for (int t = t0; t < t1; ++t) c += occ(t, k);
      if (c) ks.push_back(k);
      full = full && c == n;
    }
    // wave of each tile: dealt in turn, then pairwise swaps while they lower
    // the sum over chunks of the busiest wave's block count
    std::vector<int> wv(n);
    for (int i = 0; i < n; ++i) wv[i] = i % nw;
    auto cost = [&]() {
      long tot = 0;
      std::vector<int> per(nw);
      for (size_t c0 = 0; c0 < ks.size(); c0 += kc) {
        std::fill(per.begin(), per.end(), 0);
        for (size_t c = c0; c < std::min(ks.size(), c0 + kc); ++c)
          for (int i = 0; i < n; ++i) per[wv[i]] += occ(t0 + i, ks[c]);
        tot += *std::max_element(per.begin(), per.end());
      }
      return tot;
    };
    long best = cost();
    if (!full) {
      // bounded local search (a few sweeps over the pairs of the group's tiles)
      for (int sweep = 0; sweep < 8; ++sweep) {
        bool better = false;
        for (int i = 0; i < n; ++i)
          for (int j = i + 1; j < n; ++j) {
            if (wv[i] == wv[j]) continue;
            std::swap(wv[i], wv[j]);
            const long c = cost();
            if (c < best) {
              best = c;
              better = true;
            } else {
              std::swap(wv[i], wv[j]);
            }
          }
        if (!better) break;
      }
    }
    g.chunk_max += (double)best;
    std::vector<int> fill(nw, 0);
    std::vector<int> slot_tile((size_t)nw * rw, -1);
    for (int i = 0; i < n; ++i) {
      const int w = wv[i], j = fill[w]++;
      slot_tile[(size_t)w * rw + j] = t0 + i;
      g.tiles[((size_t)gi * nw + w) * rw + j] = t0 + i;
    }
    g.range.push_back(make_int2((int)g.list.size(), (int)ks.size()));
    for (int k : ks) {
      uint32_t masks = 0;
      for (int w = 0; w < nw; ++w)
        for (int j = 0; j < rw; ++j) {
          const int t = slot_tile[(size_t)w * rw + j];
          if (t >= 0 && occ(t, k)) {
            masks |= 1u << (8 * w + j);
            g.blocks += 1;
          }
        }
      g.list.push_back(make_int2(k, (int)masks));
    }
  }
}

}  // namespace mmnlse

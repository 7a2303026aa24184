// Host-side ligand preprocessing for libmdock: validation, centring, torsion tree,
// moving-set masks and the intramolecular pair list with per-pair coefficients.
//
// The ligand is a set of point atoms whose degrees of freedom are translation,
// orientation and the rotatable bonds (paper, Background, "Design and Structure of
// MiniMDock").  The energy kernel turns atoms about those bonds in a fixed order
// (Section "Approach 1", listing of decomposed target functions); here the order is
// encoded per atom as a bit mask over torsions sorted by depth, so a kernel lane can
// apply its own atom's chain deepest-first about reference-frame axes.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <sstream>

#include "internal.h"

namespace mdock {

namespace {

bool finite3(const float* p) {
  return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]);
}

// graph distances from `src` over the bond graph
std::vector<int> bfs(const std::vector<std::vector<int>>& adj, int src, std::vector<int>* parent) {
  std::vector<int> d(adj.size(), -1);
  if (parent) parent->assign(adj.size(), -1);
  std::queue<int> q;
  d[src] = 0;
  q.push(src);
  while (!q.empty()) {
    int a = q.front();
    q.pop();
    for (int b : adj[a]) {
      if (d[b] < 0) {
        d[b] = d[a] + 1;
        if (parent) (*parent)[b] = a;
        q.push(b);
      }
    }
  }
  return d;
}

}  // namespace

std::string prepare_ligand(int n, const float* xyz, const int* type, const float* charge,
                           int n_bonds, const int* bonds, int n_torsions, const int* torsions,
                           int root, int n_types, const float* tp, LigHost& out,
                           bool& range_error) {
  range_error = false;
  if (n < 1 || n > kMaxAtoms) {
    range_error = true;
    return "n_atoms must be in [1, 128]";
  }
  if (n_torsions < 0 || n_torsions > kMaxTorsions) {
    range_error = true;
    return "n_torsions must be in [0, 32]";
  }
  if (n_types != kTypes) return "n_types must be 7";
  if (!xyz || !type || !charge || !tp) return "null ligand array";
  if (n_bonds < n - 1 || n_bonds > 4 * n) return "n_bonds must be in [n_atoms - 1, 4 n_atoms] (a connected bond graph)";
  if (n_bonds > 0 && !bonds) return "null bond array";
  if (n_torsions > 0 && !torsions) return "null torsion array";
  if (root < 0 || root >= n) return "root atom out of range";
  for (int i = 0; i < n; ++i) {
    if (!finite3(xyz + 3 * i) || !std::isfinite(charge[i])) return "non-finite coordinate or charge";
    if (type[i] < 0 || type[i] >= n_types) return "atom type out of range";
  }
  for (int t = 0; t < n_types * 7; ++t)
    if (!std::isfinite(tp[t])) return "non-finite type parameter";
  for (int t = 0; t < n_types; ++t) {
    int role = (int)tp[t * 7 + 4];
    if (role < 0 || role > 2 || tp[t * 7 + 0] <= 0.f || tp[t * 7 + 1] < 0.f)
      return "invalid type parameters";
  }
  std::vector<std::vector<int>> adj(n);
  for (int b = 0; b < n_bonds; ++b) {
    int a0 = bonds[2 * b], a1 = bonds[2 * b + 1];
    if (a0 < 0 || a0 >= n || a1 < 0 || a1 >= n || a0 == a1) return "bond atom index out of range";
    if (std::find(adj[a0].begin(), adj[a0].end(), a1) != adj[a0].end()) return "bond listed twice";
    adj[a0].push_back(a1);
    adj[a1].push_back(a0);
  }
  std::vector<int> parent;
  std::vector<int> depth = bfs(adj, root, &parent);
  for (int i = 0; i < n; ++i)
    if (depth[i] < 0) return "bonds do not connect every atom";

  // torsions: orient from the root side, collect moving sets
  struct Tor { int a, b, gene, depth_a; std::vector<char> moving; };
  std::vector<Tor> tors;
  std::vector<char> used(n_bonds > 0 ? n_bonds : 1, 0);
  for (int k = 0; k < n_torsions; ++k) {
    int bi = torsions[k];
    if (bi < 0 || bi >= n_bonds) return "torsion bond index out of range";
    if (used[bi]) return "torsion bond listed twice";
    used[bi] = 1;
    int a = bonds[2 * bi], b = bonds[2 * bi + 1];
    if (depth[a] > depth[b]) std::swap(a, b);
    if (adj[a].size() < 2 || adj[b].size() < 2) return "a terminal bond cannot be a torsion";
    Tor t{a, b, 7 + k, depth[a], std::vector<char>(n, 0)};
    // far side of the bond: everything reachable from b without crossing (a, b); a bond in a
    // ring has no far side (a is reached too)
    std::vector<int> stack{b};
    t.moving[b] = 1;
    while (!stack.empty()) {
      const int x = stack.back();
      stack.pop_back();
      for (int y : adj[x])
        if (!t.moving[y] && !(x == b && y == a)) {
          t.moving[y] = 1;
          stack.push_back(y);
        }
    }
    if (t.moving[a]) return "a rotatable bond cannot lie in a ring";
    tors.push_back(std::move(t));
  }
  std::stable_sort(tors.begin(), tors.end(),
                   [](const Tor& x, const Tor& y) { return x.depth_a < y.depth_a; });

  // centre the reference coordinates on their centroid
  double c[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) c[d] += xyz[3 * i + d];
  for (int d = 0; d < 3; ++d) c[d] /= n;
  std::vector<double> p0(3 * n);
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) p0[3 * i + d] = (double)xyz[3 * i + d] - c[d];

  out = LigHost();
  out.n_atoms = n;
  out.n_tors = n_torsions;
  out.n_genes = 7 + n_torsions;
  out.atom_p0q.resize(n);
  out.atom_type.assign(type, type + n);
  out.atom_mask.assign(n, 0u);
  for (int i = 0; i < n; ++i)
    out.atom_p0q[i] = make_float4((float)p0[3 * i], (float)p0[3 * i + 1], (float)p0[3 * i + 2], charge[i]);
  for (int k = 0; k < n_torsions; ++k) {
    const Tor& t = tors[k];
    double u[3], len = 0;
    for (int d = 0; d < 3; ++d) {
      u[d] = p0[3 * t.b + d] - p0[3 * t.a + d];
      len += u[d] * u[d];
    }
    len = std::sqrt(len);
    if (!(len > 1e-6)) return "zero-length rotatable bond";
    out.tor_axis.push_back(make_float4((float)(u[0] / len), (float)(u[1] / len), (float)(u[2] / len), 0.f));
    out.tor_pivot.push_back(make_float4((float)p0[3 * t.a], (float)p0[3 * t.a + 1], (float)p0[3 * t.a + 2], 0.f));
    out.tor_ab.push_back(make_int2(t.a, t.b));
    out.tor_gene.push_back(t.gene);
    for (int i = 0; i < n; ++i)
      if (t.moving[i]) out.atom_mask[i] |= (1u << k);
  }

  // pair list: at least 3 bonds apart and separated by a rotatable bond (different masks)
  const double wel = (double)kWel * kCoulomb;
  for (int i = 0; i < n; ++i) {
    std::vector<int> di = bfs(adj, i, nullptr);
    for (int j = i + 1; j < n; ++j) {
      if (di[j] < 3 || out.atom_mask[i] == out.atom_mask[j]) continue;
      const float* ti = tp + 7 * type[i];
      const float* tj = tp + 7 * type[j];
      int ri = (int)ti[4], rj = (int)tj[4];
      const float* acc = nullptr;
      if (ri == 1 && rj == 2) acc = tj;
      if (ri == 2 && rj == 1) acc = ti;
      double c12, cn;
      bool hb = acc != nullptr;
      if (hb) {
        double r = acc[5], e = acc[6];
        c12 = kWhb * 5.0 * e * std::pow(r, 12);
        cn = kWhb * 6.0 * e * std::pow(r, 10);
      } else {
        double r = 0.5 * ((double)ti[0] + tj[0]);
        double e = std::sqrt((double)ti[1] * tj[1]);
        c12 = kWvdw * e * std::pow(r, 12);
        cn = kWvdw * 2.0 * e * std::pow(r, 6);
      }
      double si = ti[3] + kQasp * std::fabs((double)charge[i]);
      double sj = tj[3] + kQasp * std::fabs((double)charge[j]);
      double ds = kWds * (si * tj[2] + sj * ti[2]);
      double qq = wel * (double)charge[i] * (double)charge[j];
      out.pair_ij.push_back((uint32_t)i | ((uint32_t)j << 8) | ((hb ? 1u : 0u) << 16));
      out.pair_coef.push_back(make_float4((float)c12, (float)cn, (float)qq, (float)ds));
    }
  }
  out.gene_tor.assign(out.n_tors, 0);
  for (int k = 0; k < out.n_tors; ++k) out.gene_tor[out.tor_gene[k] - 7] = k;
  out.raw_ij = out.pair_ij;
  out.raw_coef = out.pair_coef;
  plan_ligand(out, PlanParams());
  return std::string();
}


// Pair schedule: rows of 64 slots, lanes split into groups of about N/div lanes in which no atom
// occurs twice per row (so the kernel's per-group force updates never collide).  Greedy row by
// row: the remaining pairs whose atoms have the most pairs left go first, each into a group where
// both of its atoms are still free, either way round, chosen to keep the row's LDS accesses
// spread over the banks (a slot's atoms are symmetric in the kernel).  The H-bond pairs go into the first rows (their
// free slots then take other pairs), so the rows after them need no per-slot choice between the
// 12-6 and 12-10 forms; when that layout takes more rows than one sequence of all pairs, the
// latter is used and every row up to the last H-bond pair is mixed (mix_rows).  Empty slots name
// the spare atom N.  Then the LDS plan: per-wave buffers first, then as many pair rows as fit the
// block budget (plus the one row behind them that the pair loop prefetches).
void plan_ligand(LigHost& out, const PlanParams& pp) {
  const int n = out.n_atoms;
  const int P = (int)out.raw_ij.size();
  const int A = n > kWave ? 2 : 1;
  const int div = std::max(2, std::min(8, pp.group_div));
  const int wpp = (pp.wpp == 2 || pp.wpp == 4) ? pp.wpp : 1;
  const int wpb = wpp > 1 ? wpp : std::max(1, std::min(max_waves_per_block(A), pp.wpb));
  // groups of about n / group_div lanes, larger where the block's waves could not hold one force
  // copy per group in LDS
  int want = std::max(1, std::min(kWave, n / div));
  auto fits = [&](int w) {
    const int k = (kWave + w - 1) / w;
    return (size_t)wpb * lds_wave_bytes(n, k, A, out.n_tors) + lds_pose_share_bytes(n, wpp) <=
           (size_t)kMaxLdsPerBlock;
  };
  while (want < kWave && !fits(want)) ++want;
  const int K = (kWave + want - 1) / want;
  const int m = (kWave + K - 1) / K;
  std::vector<int> left(n, 0);
  for (uint32_t v : out.raw_ij) {
    ++left[v & 0xff];
    ++left[(v >> 8) & 0xff];
  }
  // LDS banks (32 four-byte banks, 32 lanes served at a time): the pair loop reads a slot's two
  // atoms' x and y with one two-word load and z with another, from the coordinates and from its
  // group's force copy (read, then written back).  Word w of an access lies in bank w mod 32.
  const int pitch = lds_pitch(A);
  const int copy_words = (int)(lds_coord_bytes(A) / 4);
  // One row under construction: its slots (and which were turned round), the atoms each lane
  // group already holds, how far each group is filled, and per half-row the number of words each
  // of the row's eight accesses (i or j atom; coordinates or force copy; x-y pair or z) places in
  // each bank, with the largest of those counts.
  struct Row {
    std::vector<int> slot;
    std::vector<uint8_t> flip;
    std::vector<uint64_t> used;
    std::vector<int> fill;
    std::vector<uint8_t> bank;   // [2 halves][8 accesses][32 banks]
    std::vector<uint8_t> top;    // [2 halves][8 accesses]
  };
  auto new_row = [&]() {
    Row r;
    r.slot.assign(kWave, -1);
    r.flip.assign(kWave, 0);
    r.used.assign(2 * K, 0);
    r.fill.resize(K);
    for (int g = 0; g < K; ++g) r.fill[g] = g * m;
    r.bank.assign(2 * 8 * 32, 0);
    r.top.assign(2 * 8, 0);
    return r;
  };
  // the words atom a touches through access group (coordinates x-y, z; force copy x-y, z) in lane
  // group g
  auto words = [&](int a, int g, int k, int* w) {
    const int base = (k >= 2 ? g * copy_words : 0) + a;
    if ((k & 1) == 0) {
      w[0] = base;
      w[1] = base + pitch;
      return 2;
    }
    w[0] = base + 2 * pitch;
    return 1;
  };
  // growth of the row's bank-conflict cycles (force copies count twice: read and write) if atom a
  // (side 0) and atom b (side 1) took a slot of group g in half h
  auto growth = [&](const Row& row, int h, int g, int a, int b) {
    int inc = 0;
    for (int side = 0; side < 2; ++side)
      for (int k = 0; k < 4; ++k) {
        int w[2];
        const int nw = words(side == 0 ? a : b, g, k, w);
        const int acc = h * 8 + side * 4 + k;
        int top = row.top[acc];
        for (int q = 0; q < nw; ++q) top = std::max(top, (int)row.bank[acc * 32 + (w[q] & 31)] + 1);
        inc += (top - row.top[acc]) * (k >= 2 ? 2 : 1);
      }
    return inc;
  };
  auto take = [&](Row& row, int h, int g, int a, int b) {
    for (int side = 0; side < 2; ++side)
      for (int k = 0; k < 4; ++k) {
        int w[2];
        const int nw = words(side == 0 ? a : b, g, k, w);
        const int acc = h * 8 + side * 4 + k;
        for (int q = 0; q < nw; ++q) {
          uint8_t& c = row.bank[acc * 32 + (w[q] & 31)];
          ++c;
          row.top[acc] = std::max(row.top[acc], c);
        }
      }
  };
  // places what fits of `rem` into the row (the pairs whose atoms have the most pairs left
  // first) and keeps the rest in `rem`.  A pair may go into any group where both its atoms are
  // still free, either way round: of the groups already in use and the first free one, the group
  // and orientation that add the fewest bank-conflict cycles to the row (ties: the earlier group,
  // the pair as listed).
  auto fill_row = [&](Row& row, std::vector<int>& rem, std::vector<int>& left, int& groups_used) {
    std::stable_sort(rem.begin(), rem.end(), [&](int x, int y) {
      const uint32_t a = out.raw_ij[x], b = out.raw_ij[y];
      return left[a & 0xff] + left[(a >> 8) & 0xff] > left[b & 0xff] + left[(b >> 8) & 0xff];
    });
    std::vector<int> next;
    for (int p : rem) {
      const int i = out.raw_ij[p] & 0xff, j = (out.raw_ij[p] >> 8) & 0xff;
      int best_g = -1, best_flip = 0, best_inc = 0;
      for (int g = 0; g < K; ++g) {
        const int end = std::min(kWave, (g + 1) * m);
        const bool bi = (row.used[2 * g + (i >> 6)] >> (i & 63)) & 1u;
        const bool bj = (row.used[2 * g + (j >> 6)] >> (j & 63)) & 1u;
        if (row.fill[g] >= end || bi || bj) continue;
        // beyond the groups in use only the first free one, so no more force copies are needed
        // than a first-fit placement would use
        if (best_g >= 0 && g >= groups_used) break;
        const int h = row.fill[g] < 32 ? 0 : 1;
        for (int f = 0; f < 2; ++f) {
          const int inc = f == 0 ? growth(row, h, g, i, j) : growth(row, h, g, j, i);
          if (best_g < 0 || inc < best_inc) {
            best_g = g;
            best_flip = f;
            best_inc = inc;
          }
        }
      }
      if (best_g < 0) {
        next.push_back(p);
        continue;
      }
      const int g = best_g, h = row.fill[g] < 32 ? 0 : 1;
      take(row, h, g, best_flip ? j : i, best_flip ? i : j);
      row.flip[row.fill[g]] = (uint8_t)best_flip;
      row.slot[row.fill[g]++] = p;
      row.used[2 * g + (i >> 6)] |= 1ull << (i & 63);
      row.used[2 * g + (j >> 6)] |= 1ull << (j & 63);
      --left[i];
      --left[j];
      groups_used = std::max(groups_used, g + 1);
    }
    rem.swap(next);
  };
  std::vector<int> all(P), plain, hbond;
  std::iota(all.begin(), all.end(), 0);
  for (int p = 0; p < P; ++p) ((out.raw_ij[p] >> 16) & 1u ? hbond : plain).push_back(p);
  // (a) every pair in one sequence of rows
  std::vector<Row> rows_a;
  int groups_a = 0;
  {
    std::vector<int> l = left;
    while (!all.empty()) {
      rows_a.push_back(new_row());
      fill_row(rows_a.back(), all, l, groups_a);
    }
  }
  // (b) the H-bond pairs' rows first, their free slots filled with other pairs, then rows of
  // other pairs only
  std::vector<Row> rows_b;
  int groups_b = 0;
  {
    std::vector<int> l = left;
    while (!hbond.empty()) {
      rows_b.push_back(new_row());
      fill_row(rows_b.back(), hbond, l, groups_b);
    }
    for (Row& r : rows_b) fill_row(r, plain, l, groups_b);
    while (!plain.empty()) {
      rows_b.push_back(new_row());
      fill_row(rows_b.back(), plain, l, groups_b);
    }
  }
  // (b) spares the kernel the per-slot H-bond select on the rows after the H-bond rows; it is
  // used unless it takes more rows (H-bond pairs concentrate on the few donor and acceptor atoms,
  // which limits how many fit a conflict-free row)
  const bool use_b = rows_b.size() <= rows_a.size();
  const std::vector<Row>& rows = use_b ? rows_b : rows_a;
  int mix = 0;
  for (size_t r = 0; r < rows.size(); ++r)
    for (int s2 : rows[r].slot)
      if (s2 >= 0 && ((out.raw_ij[s2] >> 16) & 1u)) mix = (int)r + 1;
  out.mix_rows = mix;
  const int groups_used = use_b ? groups_b : groups_a;
  std::vector<uint32_t> ij;
  std::vector<float4> coef;
  const uint32_t pad = kPairPad | (uint32_t)n | ((uint32_t)n << 8);
  for (const Row& r : rows)
    for (int l = 0; l < kWave; ++l) {
      uint32_t v = r.slot[l] < 0 ? pad : out.raw_ij[r.slot[l]];
      if (r.slot[l] >= 0 && r.flip[l]) v = (v & ~0xffffu) | ((v & 0xffu) << 8) | ((v >> 8) & 0xffu);
      ij.push_back(v);
      coef.push_back(r.slot[l] < 0 ? make_float4(0.f, 0.f, 0.f, 0.f) : out.raw_coef[r.slot[l]]);
    }
  out.n_pairs = P;
  out.n_rows = (int)(ij.size() / kWave);
  out.pair_ij.swap(ij);
  out.pair_coef.swap(coef);
  out.group_lanes = m;
  out.n_copies = groups_used;
  out.plan = pp;
  out.wpp = wpp;
  out.wpb = wpb;
  const size_t budget = (size_t)std::max(0, std::min(pp.lds_budget, kMaxLdsPerBlock));
  const size_t waves = (size_t)out.wpb * lds_wave_bytes(n, out.n_copies, A, out.n_tors) +
                       lds_pose_share_bytes(n, out.wpp);
  int pr = out.n_rows;
  while (pr > 0 && waves + lds_pairs_bytes(pr) > budget) --pr;
  out.pl_rows = pr;
  out.lds_bytes = (int)(waves + lds_pairs_bytes(pr));
}

}  // namespace mdock

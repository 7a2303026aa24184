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

// graph distances from `src` over the tree adjacency
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
  if (n_bonds != n - 1) return "bonds must form a tree: n_bonds must equal n_atoms - 1";
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
    // far side of the bond: atoms whose path to the root passes through b
    for (int i = 0; i < n; ++i) {
      int x = i;
      while (x != root && x != b) x = parent[x];
      t.moving[i] = (x == b) ? 1 : 0;
    }
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
  // Interleave the pairs round-robin over their first atom, so that the 64 pairs a wavefront
  // handles at once touch mostly distinct atoms (their force updates then rarely hit the same
  // LDS address at the same time).
  {
    std::vector<std::vector<size_t>> by_i(n);
    for (size_t p = 0; p < out.pair_ij.size(); ++p) by_i[out.pair_ij[p] & 0xff].push_back(p);
    std::vector<uint32_t> ij;
    std::vector<float4> coef;
    ij.reserve(out.pair_ij.size());
    coef.reserve(out.pair_ij.size());
    for (size_t round = 0; ij.size() < out.pair_ij.size(); ++round)
      for (int i = 0; i < n; ++i)
        if (round < by_i[i].size()) {
          ij.push_back(out.pair_ij[by_i[i][round]]);
          coef.push_back(out.pair_coef[by_i[i][round]]);
        }
    out.pair_ij.swap(ij);
    out.pair_coef.swap(coef);
  }
  // LDS plan and incidence tables.  Chunk size: all pairs when they fit, else halved until the
  // per-wave force buffers of a block fit the budget.  Each chunk's table lists, for every
  // atom, the chunk's pairs it belongs to with the sign of its end, one column per atom so that
  // a wavefront reads a row in one access.
  {
    const int P = (int)out.pair_ij.size();
    const int A = n > kWave ? 2 : 1;
    out.inc_stride = kWave * A;
    int C = std::max(1, std::min(P, kChunkMax));
    while (C > 64 && (size_t)kWavesPerBlock * lds_wave_bytes(C, A) > kLdsBudget * 5 / 8) C = (C + 1) / 2;
    // several chunks: a multiple of the wavefront width, so every pair stays on the lane it has
    // in a single pass over the list (the energy-only path) and the sums agree bitwise
    if (C < P) C = std::max(kWave, C / kWave * kWave);
    out.chunk = C;
    out.n_chunks = P == 0 ? 0 : (P + C - 1) / C;
    out.inc_rows.clear();
    out.inc.clear();
    int total = 0;
    for (int c = 0; c < out.n_chunks; ++c) {
      const int c0 = c * C, c1 = std::min(P, c0 + C);
      std::vector<std::vector<uint16_t>> per(n);
      for (int p = c0; p < c1; ++p) {
        const uint32_t i = out.pair_ij[p] & 0xff, j = (out.pair_ij[p] >> 8) & 0xff;
        per[i].push_back((uint16_t)(p - c0));              // first atom: +force
        per[j].push_back((uint16_t)((p - c0) | 0x8000));   // second atom: -force
      }
      size_t w = 0;
      for (auto& v : per) w = std::max(w, v.size());
      out.inc_rows.push_back(make_int2(total, (int)w));
      out.inc.resize((size_t)(total + (int)w) * out.inc_stride, (uint16_t)kIncNone);
      for (int a = 0; a < n; ++a)
        for (size_t t = 0; t < per[a].size(); ++t) out.inc[(total + t) * out.inc_stride + a] = per[a][t];
      total += (int)w;
    }
    const size_t waves = (size_t)kWavesPerBlock * lds_wave_bytes(C, A);
    const size_t ib = lds_inc_bytes(total, out.inc_stride);
    out.inc_lds = (ib <= kIncLdsMax && waves + ib <= kLdsBudget) ? 1 : 0;
    const size_t fixed = waves + (out.inc_lds ? ib : 0);
    int pl = P;
    while (pl > 0 && fixed + lds_pairs_bytes(pl) > kLdsBudget) pl = std::max(0, pl - 64);
    out.pl = pl;
    out.lds_bytes = (int)(fixed + lds_pairs_bytes(pl));
  }
  return std::string();
}

}  // namespace mdock

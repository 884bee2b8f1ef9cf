// Host construction of hp spaces with the minimum rule on structured 3D
// meshes (Sec. 3): entity degrees and numbering, the cell-local -> global
// maps, owners, Dirichlet flags and a colouring for matrix-free diagonals.
#include <algorithm>
#include <cmath>

#include "hp.h"

namespace mfs {

namespace {

// merge duplicate columns, drop exact zeros
void compress(std::vector<std::pair<int64_t, double>> &w) {
  std::sort(w.begin(), w.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
  size_t o = 0;
  for (size_t i = 0; i < w.size();) {
    int64_t c = w[i].first;
    double s = 0;
    while (i < w.size() && w[i].first == c) s += w[i++].second;
    if (s != 0.0) w[o++] = {c, s};
  }
  w.resize(o);
}

// GLL nodes of degree m (cached) and the Lagrange basis on them at t
const std::vector<double> &gll(int m) {
  static const std::vector<std::vector<double>> cache = [] {
    std::vector<std::vector<double>> c(MAXQ);
    for (int k = 1; k < MAXQ; ++k) c[k] = gll_nodes(k);
    return c;
  }();
  return cache[m];
}
struct Lag {
  double v[MAXQ];
  double operator[](int j) const { return v[j]; }
};
Lag lag1(int m, double t) {
  const auto &x = gll(m);
  Lag L;
  for (int j = 0; j <= m; ++j) {
    double p = 1.0;
    for (int l = 0; l <= m; ++l)
      if (l != j) p *= (t - x[l]) / (x[j] - x[l]);
    L.v[j] = p;
  }
  return L;
}

}  // namespace

void HpSpaceHost::build(const int n_[3], const std::vector<int> &degrees) {
  for (int a = 0; a < 3; ++a) n[a] = n_[a];
  deg = degrees;
  const int64_t ncells = (int64_t)n[0] * n[1] * n[2];
  MFS_REQUIRE((int64_t)deg.size() == ncells, MFS_EINVAL, "degree array has %zu entries for %lld cells", deg.size(),
              (long long)ncells);
  auto D = [&](int x, int y, int z) { return deg[x + (int64_t)n[0] * (y + (int64_t)n[1] * z)]; };
  nvert = (int64_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  int64_t off = nvert;
  // entity degree = lowest degree of the cells around it
  auto entity_min = [&](const int idx[3], const bool fixed[3]) {
    int lo[3], hi[3];
    for (int b = 0; b < 3; ++b) {
      if (fixed[b]) {
        lo[b] = std::max(idx[b] - 1, 0);
        hi[b] = std::min(idx[b], n[b] - 1);
      } else {
        lo[b] = hi[b] = idx[b];
      }
    }
    int m = 1 << 20;
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) m = std::min(m, D(x, y, z));
    return m;
  };
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) ebox[a][b] = n[b] + (b == a ? 0 : 1);
    const int64_t cnt = (int64_t)ebox[a][0] * ebox[a][1] * ebox[a][2];
    edeg[a].resize(cnt);
    eoff[a].resize(cnt);
    const bool fixed[3] = {a != 0, a != 1, a != 2};
    int idx[3];
    for (idx[2] = 0; idx[2] < ebox[a][2]; ++idx[2])
      for (idx[1] = 0; idx[1] < ebox[a][1]; ++idx[1])
        for (idx[0] = 0; idx[0] < ebox[a][0]; ++idx[0]) {
          const int64_t e = eidx(a, idx);
          edeg[a][e] = entity_min(idx, fixed);
          eoff[a][e] = off;
          off += edeg[a][e] - 1;
        }
  }
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) fbox[a][b] = n[b] + (b == a ? 1 : 0);
    const int64_t cnt = (int64_t)fbox[a][0] * fbox[a][1] * fbox[a][2];
    fdeg[a].resize(cnt);
    foff[a].resize(cnt);
    const bool fixed[3] = {a == 0, a == 1, a == 2};
    int idx[3];
    for (idx[2] = 0; idx[2] < fbox[a][2]; ++idx[2])
      for (idx[1] = 0; idx[1] < fbox[a][1]; ++idx[1])
        for (idx[0] = 0; idx[0] < fbox[a][0]; ++idx[0]) {
          const int64_t f = fidx(a, idx);
          fdeg[a][f] = entity_min(idx, fixed);
          foff[a][f] = off;
          off += (int64_t)(fdeg[a][f] - 1) * (fdeg[a][f] - 1);
        }
  }
  coff.resize(ncells);
  for (int64_t c = 0; c < ncells; ++c) {
    coff[c] = off;
    off += (int64_t)(deg[c] - 1) * (deg[c] - 1) * (deg[c] - 1);
  }
  N = off;
  MFS_REQUIRE(N < (1LL << 31), MFS_EINVAL, "hp space too large for 32-bit indices");

  // Dirichlet: every unknown on the boundary
  dirichlet.assign(N, 0);
  for (int z = 0; z <= n[2]; ++z)
    for (int y = 0; y <= n[1]; ++y)
      for (int x = 0; x <= n[0]; ++x)
        if (x == 0 || x == n[0] || y == 0 || y == n[1] || z == 0 || z == n[2]) dirichlet[vertex(x, y, z)] = 1;
  for (int a = 0; a < 3; ++a) {
    int idx[3];
    for (idx[2] = 0; idx[2] < ebox[a][2]; ++idx[2])
      for (idx[1] = 0; idx[1] < ebox[a][1]; ++idx[1])
        for (idx[0] = 0; idx[0] < ebox[a][0]; ++idx[0]) {
          bool bnd = false;
          for (int b = 0; b < 3; ++b)
            if (b != a) bnd = bnd || idx[b] == 0 || idx[b] == n[b];
          if (!bnd) continue;
          const int64_t e = eidx(a, idx);
          for (int j = 0; j < edeg[a][e] - 1; ++j) dirichlet[eoff[a][e] + j] = 1;
        }
    for (idx[2] = 0; idx[2] < fbox[a][2]; ++idx[2])
      for (idx[1] = 0; idx[1] < fbox[a][1]; ++idx[1])
        for (idx[0] = 0; idx[0] < fbox[a][0]; ++idx[0]) {
          if (idx[a] != 0 && idx[a] != n[a]) continue;
          const int64_t f = fidx(a, idx);
          const int64_t m1 = fdeg[a][f] - 1;
          for (int64_t j = 0; j < m1 * m1; ++j) dirichlet[foff[a][f] + j] = 1;
        }
  }

  // cell-local rows; the owner of an unknown is the first cell with a local
  // node exactly at its point (an identity row)
  owner_cell.assign(N, -1);
  owner_local.assign(N, -1);
  row_base.resize(ncells + 1);
  row_ptr.assign(1, 0);
  col.clear();
  val.clear();
  std::vector<std::pair<int64_t, double>> w;
  for (int64_t c = 0; c < ncells; ++c) {
    row_base[c] = (int64_t)row_ptr.size() - 1;
    const int cc[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((int64_t)n[0] * n[1]))};
    const int k = deg[c];
    const auto &x = gll(k);
    for (int l = 0; l <= k; ++l)
      for (int j = 0; j <= k; ++j)
        for (int i = 0; i <= k; ++i) {
          const int li[3] = {i, j, l};
          int pos[3], nfixed = 0, fixed_axis = -1, free_axis = -1;
          for (int b = 0; b < 3; ++b) {
            const bool f = li[b] == 0 || li[b] == k;
            pos[b] = cc[b] + (li[b] == k ? 1 : 0);
            if (f) {
              ++nfixed;
              fixed_axis = b;
            } else {
              free_axis = b;
              pos[b] = cc[b];
            }
          }
          w.clear();
          if (nfixed == 3) {
            w.push_back({vertex(pos[0], pos[1], pos[2]), 1.0});
          } else if (nfixed == 2) {
            edge_weights(free_axis, pos, x[li[free_axis]], 1.0, w);
          } else if (nfixed == 1) {
            const int a = fixed_axis, a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
            face_weights(a, pos, x[li[a1]], x[li[a2]], w);
          } else {
            w.push_back({coff[c] + (i - 1) + (int64_t)(k - 1) * ((j - 1) + (int64_t)(k - 1) * (l - 1)), 1.0});
          }
          compress(w);
          if (w.size() == 1 && w[0].second == 1.0 && owner_cell[w[0].first] < 0) {
            owner_cell[w[0].first] = (int)c;
            owner_local[w[0].first] = i + (k + 1) * (j + (k + 1) * l);
          }
          for (const auto &p : w) {
            col.push_back((int)p.first);
            val.push_back(p.second);
          }
          row_ptr.push_back((int64_t)col.size());
        }
  }
  row_base[ncells] = (int64_t)row_ptr.size() - 1;
  for (int64_t g = 0; g < N; ++g)
    MFS_REQUIRE(owner_cell[g] >= 0, MFS_EINVAL, "hp unknown %lld has no owning cell", (long long)g);
}

void HpSpaceHost::edge_weights(int a, const int e[3], double t, double scale,
                               std::vector<std::pair<int64_t, double>> &out) const {
  const int64_t ei = eidx(a, e);
  const int m = edeg[a][ei];
  const Lag L = lag1(m, t);
  int end[3] = {e[0], e[1], e[2]};
  end[a] += 1;
  for (int j = 0; j <= m; ++j) {
    if (L[j] == 0.0) continue;
    int64_t g;
    if (j == 0)
      g = vertex(e[0], e[1], e[2]);
    else if (j == m)
      g = vertex(end[0], end[1], end[2]);
    else
      g = eoff[a][ei] + j - 1;
    out.push_back({g, scale * L[j]});
  }
}

void HpSpaceHost::face_weights(int a, const int f[3], double s, double t,
                               std::vector<std::pair<int64_t, double>> &out) const {
  const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
  const int64_t fi = fidx(a, f);
  const int m = fdeg[a][fi];
  const auto &x = gll(m);
  const Lag Ls = lag1(m, s), Lt = lag1(m, t);
  for (int q = 0; q <= m; ++q)
    for (int p = 0; p <= m; ++p) {
      const double w = Ls[p] * Lt[q];
      if (w == 0.0) continue;
      const bool pe = p == 0 || p == m, qe = q == 0 || q == m;
      int e[3] = {f[0], f[1], f[2]};
      if (pe && qe) {
        if (p == m) e[a1] += 1;
        if (q == m) e[a2] += 1;
        out.push_back({vertex(e[0], e[1], e[2]), w});
      } else if (pe) {  // edge along a2 on the side a1 = p / m
        if (p == m) e[a1] += 1;
        edge_weights(a2, e, x[q], w, out);
      } else if (qe) {
        if (q == m) e[a2] += 1;
        edge_weights(a1, e, x[p], w, out);
      } else {
        out.push_back({foff[a][fi] + (p - 1) + (int64_t)(m - 1) * (q - 1), w});
      }
    }
}

void HpSpaceHost::reference_point(int64_t g, double p[3]) const {
  if (g < nvert) {
    p[0] = (double)(g % (n[0] + 1));
    p[1] = (double)((g / (n[0] + 1)) % (n[1] + 1));
    p[2] = (double)(g / ((int64_t)(n[0] + 1) * (n[1] + 1)));
    return;
  }
  for (int a = 0; a < 3; ++a) {
    const auto &o = eoff[a];
    if (o.empty()) continue;
    const int64_t last = o.back() + edeg[a].back() - 1;
    if (g >= o.front() && g < last) {
      const int64_t e = (int64_t)(std::upper_bound(o.begin(), o.end(), g) - o.begin()) - 1;
      const int64_t j = g - o[e];
      const int m = edeg[a][e];
      const int idx[3] = {(int)(e % ebox[a][0]), (int)((e / ebox[a][0]) % ebox[a][1]),
                          (int)(e / ((int64_t)ebox[a][0] * ebox[a][1]))};
      for (int b = 0; b < 3; ++b) p[b] = idx[b];
      p[a] += gll(m)[j + 1];
      return;
    }
  }
  for (int a = 0; a < 3; ++a) {
    const auto &o = foff[a];
    if (o.empty()) continue;
    const int64_t last = o.back() + (int64_t)(fdeg[a].back() - 1) * (fdeg[a].back() - 1);
    if (g >= o.front() && g < last) {
      const int64_t f = (int64_t)(std::upper_bound(o.begin(), o.end(), g) - o.begin()) - 1;
      const int64_t j = g - o[f];
      const int m = fdeg[a][f];
      const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
      const int idx[3] = {(int)(f % fbox[a][0]), (int)((f / fbox[a][0]) % fbox[a][1]),
                          (int)(f / ((int64_t)fbox[a][0] * fbox[a][1]))};
      const auto &x = gll(m);
      for (int b = 0; b < 3; ++b) p[b] = idx[b];
      p[a1] += x[1 + j % (m - 1)];
      p[a2] += x[1 + j / (m - 1)];
      return;
    }
  }
  const int64_t c = (int64_t)(std::upper_bound(coff.begin(), coff.end(), g) - coff.begin()) - 1;
  const int k = deg[c];
  const int64_t j = g - coff[c];
  const auto &x = gll(k);
  const int cc[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((int64_t)n[0] * n[1]))};
  p[0] = cc[0] + x[1 + j % (k - 1)];
  p[1] = cc[1] + x[1 + (j / (k - 1)) % (k - 1)];
  p[2] = cc[2] + x[1 + j / ((int64_t)(k - 1) * (k - 1))];
}

std::vector<int> HpSpaceHost::colours(int *ncolours) const {
  int Me = 0, Mf = 0, Mc = 0;
  for (int a = 0; a < 3; ++a) {
    for (int m : edeg[a]) Me = std::max(Me, m - 1);
    for (int m : fdeg[a]) Mf = std::max(Mf, (m - 1) * (m - 1));
  }
  for (int k : deg) Mc = std::max(Mc, (k - 1) * (k - 1) * (k - 1));
  std::vector<int> col(N, 0);
  for (int z = 0; z <= n[2]; ++z)
    for (int y = 0; y <= n[1]; ++y)
      for (int x = 0; x <= n[0]; ++x) col[vertex(x, y, z)] = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
  const int be = 8, bf = be + 12 * Me, bc = bf + 6 * Mf;
  for (int a = 0; a < 3; ++a) {
    const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;  // the two fixed axes of an edge along a
    int idx[3];
    for (idx[2] = 0; idx[2] < ebox[a][2]; ++idx[2])
      for (idx[1] = 0; idx[1] < ebox[a][1]; ++idx[1])
        for (idx[0] = 0; idx[0] < ebox[a][0]; ++idx[0]) {
          const int64_t e = eidx(a, idx);
          const int cls = (idx[o1] & 1) | ((idx[o2] & 1) << 1);
          for (int j = 0; j < edeg[a][e] - 1; ++j) col[eoff[a][e] + j] = be + (a * 4 + cls) * Me + j;
        }
    for (idx[2] = 0; idx[2] < fbox[a][2]; ++idx[2])
      for (idx[1] = 0; idx[1] < fbox[a][1]; ++idx[1])
        for (idx[0] = 0; idx[0] < fbox[a][0]; ++idx[0]) {
          const int64_t f = fidx(a, idx);
          const int cls = idx[a] & 1;
          const int m1 = fdeg[a][f] - 1;
          for (int j = 0; j < m1 * m1; ++j) col[foff[a][f] + j] = bf + (a * 2 + cls) * Mf + j;
        }
  }
  for (size_t c = 0; c < deg.size(); ++c) {
    const int k1 = deg[c] - 1;
    for (int j = 0; j < k1 * k1 * k1; ++j) col[coff[c] + j] = bc + j;
  }
  *ncolours = bc + Mc;
  return col;
}

}  // namespace mfs

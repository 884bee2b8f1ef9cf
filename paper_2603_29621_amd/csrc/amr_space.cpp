// Host construction of the conforming Q_k space on a locally refined mesh:
// unknown numbering, hanging-node constraints and the cell-local row maps.
#include <algorithm>
#include <cmath>
#include <utility>

#include "amr.h"

namespace mfs {

namespace {

// stable LSD radix sort of 64-bit words by their upper 32 bits
void radix_sort_hi32(std::vector<uint64_t> &a) {
  std::vector<uint64_t> tmp(a.size());
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = 32 + 8 * pass;
    size_t cnt[257] = {};
    for (uint64_t v : a) cnt[((v >> sh) & 255) + 1] += 1;
    for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
    for (uint64_t v : a) tmp[cnt[(v >> sh) & 255]++] = v;
    a.swap(tmp);
  }
}

// value of the 1D Lagrange polynomial i of the k + 1 equispaced nodes at t
double lagrange1(int k, int i, double t) {
  double v = 1.0;
  for (int j = 0; j <= k; ++j)
    if (j != i) v *= (t - (double)j / k) / ((double)(i - j) / k);
  return v;
}

}  // namespace

void AmrSpaceHost::build(int n_, int L_, int64_t ncells_, const int *level_, const int *idx_, int k_) {
  MFS_REQUIRE(n_ >= 1 && n_ <= 4096, MFS_EINVAL, "base cells per direction %d out of range", n_);
  MFS_REQUIRE(L_ >= 0 && L_ <= 4, MFS_EINVAL, "refinement levels %d out of range [0, 4]", L_);
  MFS_REQUIRE(k_ == 1 || k_ == 2, MFS_EUNSUPPORTED, "refined meshes support degrees 1 and 2 (got %d)", k_);
  MFS_REQUIRE(ncells_ >= 1 && level_ && idx_, MFS_EINVAL, "empty cell list");
  n = n_;
  L = L_;
  k = k_;
  ncells = ncells_;
  R = (int64_t)k * n << L;
  const int64_t R1 = R + 1;
  MFS_REQUIRE(R1 * R1 * R1 < (int64_t(1) << 31), MFS_EINVAL, "refined mesh too fine for 32-bit positions");
  const int nb1 = k + 1, nb = nb1 * nb1 * nb1;
  MFS_REQUIRE(ncells * nb < (int64_t(1) << 31), MFS_EINVAL, "too many cells");
  level.assign(level_, level_ + ncells);
  idx.assign(idx_, idx_ + 3 * ncells);
  // the leaves must partition the cube: volume and disjointness at the finest level
  const int64_t F = (int64_t)n << L;
  {
    std::vector<uint8_t> cover((size_t)(F * F * F), 0);
    int64_t vol = 0;
    for (int64_t c = 0; c < ncells; ++c) {
      const int l = level[c];
      MFS_REQUIRE(l >= 0 && l <= L, MFS_EINVAL, "cell %lld: level %d out of range", (long long)c, l);
      const int64_t m = (int64_t)n << l, s = int64_t(1) << (L - l);
      for (int a = 0; a < 3; ++a)
        MFS_REQUIRE(idx[3 * c + a] >= 0 && idx[3 * c + a] < m, MFS_EINVAL, "cell %lld: index out of range",
                    (long long)c);
      vol += s * s * s;
      MFS_REQUIRE(vol <= F * F * F, MFS_EINVAL, "cells overlap");
      for (int64_t z = 0; z < s; ++z)
        for (int64_t y = 0; y < s; ++y)
          for (int64_t x = 0; x < s; ++x) {
            const int64_t f = (idx[3 * c] * s + x) + F * ((idx[3 * c + 1] * s + y) + F * (idx[3 * c + 2] * s + z));
            MFS_REQUIRE(!cover[f], MFS_EINVAL, "cells overlap at cell %lld", (long long)c);
            cover[f] = 1;
          }
    }
    MFS_REQUIRE(vol == F * F * F, MFS_EINVAL, "cells do not cover the cube");
  }
  // positions of every cell-local node, sorted by position (stable in the slot)
  auto origin = [&](int64_t c, int a) { return (int64_t)idx[3 * c + a] * k << (L - level[c]); };
  std::vector<uint64_t> ks((size_t)(ncells * nb));
  for (int64_t c = 0; c < ncells; ++c) {
    const int64_t u = int64_t(1) << (L - level[c]);
    const int64_t o0 = origin(c, 0), o1 = origin(c, 1), o2 = origin(c, 2);
    for (int t = 0; t < nb; ++t) {
      const int64_t p0 = o0 + (t % nb1) * u, p1 = o1 + ((t / nb1) % nb1) * u, p2 = o2 + (t / (nb1 * nb1)) * u;
      const uint64_t key = (uint64_t)(p0 + R1 * (p1 + R1 * p2));
      ks[c * nb + t] = (key << 32) | (uint64_t)(c * nb + t);
    }
  }
  radix_sort_hi32(ks);
  std::vector<int> raw_of_slot((size_t)(ncells * nb));
  std::vector<int64_t> raw_key, raw_first;  // per raw position: key and first slot
  for (size_t i = 0; i < ks.size(); ++i) {
    const uint64_t key = ks[i] >> 32;
    if (raw_key.empty() || (uint64_t)raw_key.back() != key) {
      raw_key.push_back((int64_t)key);
      raw_first.push_back((int64_t)(ks[i] & 0xffffffffu));
    }
    raw_of_slot[ks[i] & 0xffffffffu] = (int)(raw_key.size() - 1);
  }
  std::vector<uint64_t>().swap(ks);
  const int64_t Nraw = (int64_t)raw_key.size();
  // leaf ids of the levels that can hold masters (all but the finest)
  std::vector<std::vector<int>> cell_at(L);
  for (int l = 0; l < L; ++l) cell_at[l].assign((size_t)(((int64_t)n << l) * ((int64_t)n << l) * ((int64_t)n << l)), -1);
  for (int64_t c = 0; c < ncells; ++c)
    if (level[c] < L) {
      const int64_t m = (int64_t)n << level[c];
      cell_at[level[c]][idx[3 * c] + m * (idx[3 * c + 1] + m * idx[3 * c + 2])] = (int)c;
    }
  // hanging positions: the coarsest leaf whose closed box holds the position
  // without it being one of the leaf's nodes
  std::vector<int> master((size_t)Nraw, -1);
  for (int64_t r = 0; r < Nraw; ++r) {
    const int64_t p[3] = {raw_key[r] % R1, (raw_key[r] / R1) % R1, raw_key[r] / (R1 * R1)};
    for (int l = 0; l < L && master[r] < 0; ++l) {
      const int64_t u = int64_t(1) << (L - l), s = k * u, m = (int64_t)n << l;
      if (p[0] % u == 0 && p[1] % u == 0 && p[2] % u == 0) continue;  // a node of every level-l cell here
      int64_t lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        hi[a] = std::min(p[a] / s, m - 1);
        lo[a] = (p[a] % s == 0) ? std::max<int64_t>(p[a] / s - 1, 0) : hi[a];
      }
      for (int64_t z = lo[2]; z <= hi[2] && master[r] < 0; ++z)
        for (int64_t y = lo[1]; y <= hi[1] && master[r] < 0; ++y)
          for (int64_t x = lo[0]; x <= hi[0] && master[r] < 0; ++x) {
            const int id = cell_at[l][x + m * (y + m * z)];
            if (id >= 0) master[r] = id;
          }
    }
  }
  std::vector<std::vector<int>>().swap(cell_at);
  // unknowns
  std::vector<int> true_of((size_t)Nraw, -1);
  N = 0;
  for (int64_t r = 0; r < Nraw; ++r)
    if (master[r] < 0) true_of[r] = (int)N++;
  nhanging = Nraw - N;
  tpos.resize((size_t)(3 * N));
  V.dirichlet.assign((size_t)N, 0);
  V.owner_cell.resize((size_t)N);
  V.owner_local.resize((size_t)N);
  for (int64_t r = 0; r < Nraw; ++r) {
    const int g = true_of[r];
    if (g < 0) continue;
    const int64_t p[3] = {raw_key[r] % R1, (raw_key[r] / R1) % R1, raw_key[r] / (R1 * R1)};
    bool bnd = false;
    for (int a = 0; a < 3; ++a) {
      tpos[3 * g + a] = p[a];
      bnd = bnd || p[a] == 0 || p[a] == R;
    }
    V.dirichlet[g] = bnd ? 1 : 0;
    V.owner_cell[g] = (int)(raw_first[r] / nb);
    V.owner_local[g] = (int)(raw_first[r] % nb);
  }
  // expansions of the hanging positions, masters' levels ascending (a hanging
  // master of a level-l leaf hangs on a coarser leaf, so it comes first)
  std::vector<int64_t> hang;
  for (int64_t r = 0; r < Nraw; ++r)
    if (master[r] >= 0) hang.push_back(r);
  std::stable_sort(hang.begin(), hang.end(), [&](int64_t a, int64_t b) { return level[master[a]] < level[master[b]]; });
  std::vector<int64_t> hslot((size_t)Nraw, -1), hptr(1, 0);
  std::vector<int> hcol;
  std::vector<double> hval;
  std::vector<std::pair<int, double>> terms;
  for (size_t h = 0; h < hang.size(); ++h) {
    const int64_t r = hang[h];
    const int c = master[r];
    const int64_t s = (int64_t)k << (L - level[c]);
    const int64_t p[3] = {raw_key[r] % R1, (raw_key[r] / R1) % R1, raw_key[r] / (R1 * R1)};
    double w1[3][3];
    for (int a = 0; a < 3; ++a) {
      const double t = (double)(p[a] - origin(c, a)) / (double)s;
      for (int i = 0; i <= k; ++i) w1[a][i] = lagrange1(k, i, t);
    }
    terms.clear();
    for (int t = 0; t < nb; ++t) {
      const double w = w1[0][t % nb1] * w1[1][(t / nb1) % nb1] * w1[2][t / (nb1 * nb1)];
      if (std::fabs(w) < 1e-14) continue;
      const int rs = raw_of_slot[c * nb + t];
      if (true_of[rs] >= 0) {
        terms.emplace_back(true_of[rs], w);
      } else {
        const int64_t q = hslot[rs];
        MFS_REQUIRE(q >= 0, MFS_EINVAL, "hanging-node chain out of order");
        for (int64_t e = hptr[q]; e < hptr[q + 1]; ++e) terms.emplace_back(hcol[e], w * hval[e]);
      }
    }
    std::sort(terms.begin(), terms.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    for (size_t i = 0; i < terms.size();) {
      size_t j = i;
      double v = 0.0;
      for (; j < terms.size() && terms[j].first == terms[i].first; ++j) v += terms[j].second;
      if (std::fabs(v) > 1e-14) {
        hcol.push_back(terms[i].first);
        hval.push_back(v);
      }
      i = j;
    }
    hslot[r] = (int64_t)h;
    hptr.push_back((int64_t)hcol.size());
  }
  // cell-local rows
  V.n[0] = V.n[1] = V.n[2] = n;
  V.deg.assign((size_t)ncells, k);
  V.N = N;
  V.row_base.resize((size_t)ncells + 1);
  V.row_ptr.assign(1, 0);
  V.row_ptr.reserve((size_t)(ncells * nb + 1));
  V.col.clear();
  V.val.clear();
  V.col.reserve((size_t)(ncells * nb));
  V.val.reserve((size_t)(ncells * nb));
  for (int64_t c = 0; c < ncells; ++c) {
    V.row_base[c] = c * nb;
    for (int t = 0; t < nb; ++t) {
      const int rs = raw_of_slot[c * nb + t];
      if (true_of[rs] >= 0) {
        V.col.push_back(true_of[rs]);
        V.val.push_back(1.0);
      } else {
        const int64_t q = hslot[rs];
        for (int64_t e = hptr[q]; e < hptr[q + 1]; ++e) {
          V.col.push_back(hcol[e]);
          V.val.push_back(hval[e]);
        }
      }
      V.row_ptr.push_back((int64_t)V.col.size());
    }
  }
  V.row_base[ncells] = ncells * nb;
  // corner coordinates
  Xcell.resize((size_t)(ncells * 24));
  for (int64_t c = 0; c < ncells; ++c) {
    const double h = 1.0 / (double)((int64_t)n << level[c]);
    for (int v = 0; v < 8; ++v)
      for (int a = 0; a < 3; ++a) Xcell[c * 24 + v * 3 + a] = (idx[3 * c + a] + ((v >> a) & 1)) * h;
  }
}

}  // namespace mfs

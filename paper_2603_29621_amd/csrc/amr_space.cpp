// Host construction of the conforming Q_k space on a locally refined mesh:
// unknown numbering, hanging-node constraints and the cell-local row maps.
#include <algorithm>
#include <array>
#include <cmath>
#include <thread>
#include <unordered_map>
#include <utility>

#include "amr.h"

namespace mfs {

namespace {

// host threads for a loop of n iterations (at least 64k iterations each)
int threads_for(int64_t n) {
  const int64_t hw = std::max<int64_t>(1, std::min<int64_t>(std::thread::hardware_concurrency(), 16));
  return (int)std::max<int64_t>(1, std::min<int64_t>(hw, n / 65536));
}

// f(t, lo, hi) on nt threads over the contiguous chunks of [0, n); f must not throw
template <typename F>
void chunks(int nt, int64_t n, F &&f) {
  if (nt <= 1) {
    f(0, int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back([&, t] { f(t, n * t / nt, n * (t + 1) / nt); });
  for (auto &x : th) x.join();
}

// stable LSD radix sort of 64-bit words by their upper 32 bits: per pass,
// per-chunk digit counts, then every chunk scatters its words in order to its
// own offsets, so the result is the sequential one
void radix_sort_hi32(std::vector<uint64_t> &a) {
  const int64_t n = (int64_t)a.size();
  const int nt = threads_for(n);
  std::vector<uint64_t> tmp(a.size());
  std::vector<std::array<int64_t, 256>> cnt((size_t)nt);
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = 32 + 8 * pass;
    chunks(nt, n, [&](int t, int64_t lo, int64_t hi) {
      cnt[t].fill(0);
      for (int64_t i = lo; i < hi; ++i) cnt[t][(a[i] >> sh) & 255] += 1;
    });
    int64_t run = 0;
    for (int b = 0; b < 256; ++b)
      for (int t = 0; t < nt; ++t) {
        const int64_t c = cnt[t][b];
        cnt[t][b] = run;
        run += c;
      }
    chunks(nt, n, [&](int t, int64_t lo, int64_t hi) {
      std::array<int64_t, 256> &off = cnt[t];
      for (int64_t i = lo; i < hi; ++i) tmp[off[(a[i] >> sh) & 255]++] = a[i];
    });
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
  const int ntc = threads_for(ncells);
  chunks(ntc, ncells, [&](int, int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t u = int64_t(1) << (L - level[c]);
      const int64_t o0 = origin(c, 0), o1 = origin(c, 1), o2 = origin(c, 2);
      for (int t = 0; t < nb; ++t) {
        const int64_t p0 = o0 + (t % nb1) * u, p1 = o1 + ((t / nb1) % nb1) * u, p2 = o2 + (t / (nb1 * nb1)) * u;
        const uint64_t key = (uint64_t)(p0 + R1 * (p1 + R1 * p2));
        ks[c * nb + t] = (key << 32) | (uint64_t)(c * nb + t);
      }
    }
  });
  radix_sort_hi32(ks);
  // distinct positions in sorted order: a new one starts where the key changes
  const int64_t nks = (int64_t)ks.size();
  const int ntk = threads_for(nks);
  std::vector<int64_t> starts((size_t)ntk + 1, 0);
  auto is_new = [&](int64_t i) { return i == 0 || (ks[i] >> 32) != (ks[i - 1] >> 32); };
  chunks(ntk, nks, [&](int t, int64_t lo, int64_t hi) {
    int64_t m = 0;
    for (int64_t i = lo; i < hi; ++i) m += is_new(i);
    starts[t + 1] = m;
  });
  for (int t = 0; t < ntk; ++t) starts[t + 1] += starts[t];
  const int64_t Nraw = starts[ntk];
  std::vector<int> raw_of_slot((size_t)(ncells * nb));
  std::vector<int64_t> raw_key((size_t)Nraw), raw_first((size_t)Nraw);  // per position: key, first slot
  chunks(ntk, nks, [&](int t, int64_t lo, int64_t hi) {
    int64_t r = starts[t] - 1;
    for (int64_t i = lo; i < hi; ++i) {
      const int64_t slot = (int64_t)(ks[i] & 0xffffffffu);
      if (is_new(i)) {
        ++r;
        raw_key[r] = (int64_t)(ks[i] >> 32);
        raw_first[r] = slot;
      }
      raw_of_slot[slot] = (int)r;
    }
  });
  std::vector<uint64_t>().swap(ks);
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
  const int ntr = threads_for(Nraw);
  chunks(ntr, Nraw, [&](int, int64_t r0, int64_t r1) {
  for (int64_t r = r0; r < r1; ++r) {
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
  });
  std::vector<std::vector<int>>().swap(cell_at);
  // unknowns
  std::vector<int> true_of((size_t)Nraw, -1);
  {
    std::vector<int64_t> base((size_t)ntr + 1, 0);
    chunks(ntr, Nraw, [&](int t, int64_t r0, int64_t r1) {
      int64_t m = 0;
      for (int64_t r = r0; r < r1; ++r) m += master[r] < 0;
      base[t + 1] = m;
    });
    for (int t = 0; t < ntr; ++t) base[t + 1] += base[t];
    N = base[ntr];
    chunks(ntr, Nraw, [&](int t, int64_t r0, int64_t r1) {
      int64_t g = base[t];
      for (int64_t r = r0; r < r1; ++r)
        if (master[r] < 0) true_of[r] = (int)g++;
    });
  }
  nhanging = Nraw - N;
  tpos.resize((size_t)(3 * N));
  V.dirichlet.assign((size_t)N, 0);
  V.owner_cell.resize((size_t)N);
  V.owner_local.resize((size_t)N);
  chunks(ntr, Nraw, [&](int, int64_t r0, int64_t r1) {
    for (int64_t r = r0; r < r1; ++r) {
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
  });
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
  V.row_ptr.assign((size_t)(ncells * nb + 1), 0);
  auto row_len = [&](int64_t slot) -> int64_t {
    const int rs = raw_of_slot[slot];
    if (true_of[rs] >= 0) return 1;
    const int64_t q = hslot[rs];
    return hptr[q + 1] - hptr[q];
  };
  // entries per chunk of cells, then each chunk fills its own range in order
  std::vector<int64_t> cbase((size_t)ntc + 1, 0);
  chunks(ntc, ncells, [&](int t, int64_t c0, int64_t c1) {
    int64_t m = 0;
    for (int64_t sl = c0 * nb; sl < c1 * nb; ++sl) m += row_len(sl);
    cbase[t + 1] = m;
  });
  for (int t = 0; t < ntc; ++t) cbase[t + 1] += cbase[t];
  V.col.assign((size_t)cbase[ntc], 0);
  V.val.assign((size_t)cbase[ntc], 0.0);
  chunks(ntc, ncells, [&](int t, int64_t c0, int64_t c1) {
    int64_t o = cbase[t];
    for (int64_t c = c0; c < c1; ++c) {
      V.row_base[c] = c * nb;
      for (int tt = 0; tt < nb; ++tt) {
        const int rs = raw_of_slot[c * nb + tt];
        if (true_of[rs] >= 0) {
          V.col[o] = true_of[rs];
          V.val[o] = 1.0;
          ++o;
        } else {
          const int64_t q = hslot[rs];
          for (int64_t e = hptr[q]; e < hptr[q + 1]; ++e, ++o) {
            V.col[o] = hcol[e];
            V.val[o] = hval[e];
          }
        }
        V.row_ptr[c * nb + tt + 1] = o;
      }
    }
  });
  V.row_base[ncells] = ncells * nb;
  // corner coordinates
  Xcell.resize((size_t)(ncells * 24));
  for (int64_t c = 0; c < ncells; ++c) {
    const double h = 1.0 / (double)((int64_t)n << level[c]);
    for (int v = 0; v < 8; ++v)
      for (int a = 0; a < 3; ++a) Xcell[c * 24 + v * 3 + a] = (idx[3 * c + a] + ((v >> a) & 1)) * h;
  }
}

std::vector<int> AmrSpaceHost::colours(int *ncolours) const {
  // cells of every unknown (CSR)
  std::vector<int64_t> cptr((size_t)N + 1, 0);
  for (int64_t c = 0; c < ncells; ++c)
    for (int64_t r = V.row_base[c]; r < V.row_base[c + 1]; ++r)
      for (int64_t q = V.row_ptr[r]; q < V.row_ptr[r + 1]; ++q) cptr[V.col[q] + 1] += 1;
  for (int64_t g = 0; g < N; ++g) cptr[g + 1] += cptr[g];
  std::vector<int> cells((size_t)cptr[N]);
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t c = 0; c < ncells; ++c)
      for (int64_t r = V.row_base[c]; r < V.row_base[c + 1]; ++r)
        for (int64_t q = V.row_ptr[r]; q < V.row_ptr[r + 1]; ++q) cells[fill[V.col[q]]++] = (int)c;
  }
  std::vector<int> col((size_t)N, -1);
  std::vector<int64_t> seen;  // colour -> the last unknown that met it
  std::vector<int> last_cell((size_t)ncells, -1);
  int nc = 0;
  for (int64_t g = 0; g < N; ++g) {
    for (int64_t e = cptr[g]; e < cptr[g + 1]; ++e) {
      const int c = cells[e];
      if (last_cell[c] == (int)g) continue;  // a cell listed twice for g
      last_cell[c] = (int)g;
      for (int64_t q = V.row_ptr[V.row_base[c]]; q < V.row_ptr[V.row_base[c + 1]]; ++q) {
        const int o = col[V.col[q]];
        if (o >= 0) seen[o] = g;
      }
    }
    int pick = 0;
    while (pick < nc && seen[pick] == g) ++pick;
    if (pick == nc) {
      seen.push_back(-1);
      ++nc;
    }
    col[g] = pick;
  }
  *ncolours = nc;
  return col;
}

void amr_coarsen(int n, const std::vector<int> &level, const std::vector<int> &idx, std::vector<int> &level_c,
                 std::vector<int> &idx_c) {
  const int64_t nc = (int64_t)level.size();
  int L = 0;
  for (int l : level) L = std::max(L, l);
  // children count of every parent, by (level of the parent, index)
  std::unordered_map<int64_t, int> count;
  auto pkey = [&](int l, int64_t x, int64_t y, int64_t z) {
    const int64_t m = (int64_t)n << l;
    return ((int64_t)l << 56) | (x + m * (y + m * z));
  };
  for (int64_t c = 0; c < nc; ++c)
    if (level[c] > 0) count[pkey(level[c] - 1, idx[3 * c] / 2, idx[3 * c + 1] / 2, idx[3 * c + 2] / 2)] += 1;
  struct Cell {
    int l, x, y, z;
  };
  std::vector<Cell> out;
  out.reserve((size_t)nc);
  std::unordered_map<int64_t, int> emitted;
  for (int64_t c = 0; c < nc; ++c) {
    const int l = level[c];
    if (l > 0) {
      const int px = idx[3 * c] / 2, py = idx[3 * c + 1] / 2, pz = idx[3 * c + 2] / 2;
      const int64_t key = pkey(l - 1, px, py, pz);
      if (count[key] == 8) {
        if (emitted.emplace(key, 1).second) out.push_back({l - 1, px, py, pz});
        continue;
      }
    }
    out.push_back({l, idx[3 * c], idx[3 * c + 1], idx[3 * c + 2]});
  }
  std::sort(out.begin(), out.end(), [](const Cell &a, const Cell &b) {
    if (a.l != b.l) return a.l < b.l;
    if (a.z != b.z) return a.z < b.z;
    if (a.y != b.y) return a.y < b.y;
    return a.x < b.x;
  });
  level_c.resize(out.size());
  idx_c.resize(3 * out.size());
  for (size_t i = 0; i < out.size(); ++i) {
    level_c[i] = out[i].l;
    idx_c[3 * i] = out[i].x;
    idx_c[3 * i + 1] = out[i].y;
    idx_c[3 * i + 2] = out[i].z;
  }
  (void)L;
}

AmrTransferHost amr_transfer(int n, const std::vector<int> &lf, const std::vector<int> &xf,
                             const std::vector<int> &lc, const std::vector<int> &xc) {
  const int64_t ncf = (int64_t)lf.size(), ncc = (int64_t)lc.size();
  auto key = [&](int l, int64_t x, int64_t y, int64_t z) {
    const int64_t m = (int64_t)n << l;
    return ((int64_t)l << 56) | (x + m * (y + m * z));
  };
  std::unordered_map<int64_t, int> coarse;
  coarse.reserve((size_t)ncc * 2);
  for (int64_t c = 0; c < ncc; ++c) coarse[key(lc[c], xc[3 * c], xc[3 * c + 1], xc[3 * c + 2])] = (int)c;
  AmrTransferHost T;
  T.parent.resize((size_t)ncf);
  T.octant.resize((size_t)ncf);
  for (int64_t f = 0; f < ncf; ++f) {
    const int l = lf[f];
    auto same = coarse.find(key(l, xf[3 * f], xf[3 * f + 1], xf[3 * f + 2]));
    if (same != coarse.end()) {
      T.parent[f] = same->second;
      T.octant[f] = 8;
      continue;
    }
    MFS_REQUIRE(l > 0, MFS_EINVAL, "coarsening lost a base cell");
    auto par = coarse.find(key(l - 1, xf[3 * f] / 2, xf[3 * f + 1] / 2, xf[3 * f + 2] / 2));
    MFS_REQUIRE(par != coarse.end(), MFS_EINVAL, "fine cell without a coarse parent");
    T.parent[f] = par->second;
    T.octant[f] = (uint8_t)((xf[3 * f] & 1) | ((xf[3 * f + 1] & 1) << 1) | ((xf[3 * f + 2] & 1) << 2));
  }
  T.cptr.assign((size_t)ncc + 1, 0);
  for (int64_t f = 0; f < ncf; ++f) T.cptr[T.parent[f] + 1] += 1;
  for (int64_t c = 0; c < ncc; ++c) T.cptr[c + 1] += T.cptr[c];
  T.child.resize((size_t)ncf);
  std::vector<int64_t> fill(T.cptr.begin(), T.cptr.end() - 1);
  for (int64_t f = 0; f < ncf; ++f) T.child[fill[T.parent[f]]++] = (int)f;
  return T;
}

std::vector<int64_t> amr_injection(const AmrSpaceHost &fine, const AmrSpaceHost &coarse) {
  MFS_REQUIRE(fine.R == 2 * coarse.R, MFS_EINVAL, "levels are not one coarsening apart");
  std::vector<int64_t> inj((size_t)coarse.N);
  const int64_t R1 = fine.R + 1;
  auto kf = [&](int64_t g) { return fine.tpos[3 * g] + R1 * (fine.tpos[3 * g + 1] + R1 * fine.tpos[3 * g + 2]); };
  int64_t f = 0;
  for (int64_t g = 0; g < coarse.N; ++g) {
    const int64_t key = 2 * coarse.tpos[3 * g] + R1 * (2 * coarse.tpos[3 * g + 1] + R1 * 2 * coarse.tpos[3 * g + 2]);
    while (f < fine.N && kf(f) < key) ++f;
    MFS_REQUIRE(f < fine.N && kf(f) == key, MFS_EINVAL, "a coarse unknown is not a fine unknown");
    inj[g] = f;
  }
  return inj;
}

}  // namespace mfs

// ---------------------------------------------------------------- partition metrics
namespace mfs {
namespace {

struct MCell {
  int l, x, y, z;
};

// Morton key of a cell's lowest corner on the finest grid, the level in the
// low bits so that a parent precedes its first child
uint64_t morton_key(const MCell &c, int L) {
  const int s = L - c.l;
  const uint64_t x = (uint64_t)c.x << s, y = (uint64_t)c.y << s, z = (uint64_t)c.z << s;
  uint64_t k = 0;
  for (int b = 0; b < 19; ++b)
    k |= (((x >> b) & 1) << (3 * b)) | (((y >> b) & 1) << (3 * b + 1)) | (((z >> b) & 1) << (3 * b + 2));
  return (k << 5) | (uint64_t)c.l;
}

uint64_t cell_id(const MCell &c, int n) {
  const uint64_t m = (uint64_t)n << c.l;
  return ((uint64_t)c.l << 56) | ((uint64_t)c.x + m * ((uint64_t)c.y + m * (uint64_t)c.z));
}

MCell parent_of(const MCell &c) { return {c.l - 1, c.x / 2, c.y / 2, c.z / 2}; }

// owners of P contiguous Morton chunks (sizes differ by at most one, the
// first count mod P one larger), by cell id
std::unordered_map<uint64_t, int> morton_partition(const std::vector<MCell> &cells, int P, int L, int n) {
  std::vector<std::pair<uint64_t, uint64_t>> order(cells.size());  // (Morton key, cell id)
  for (size_t c = 0; c < cells.size(); ++c) order[c] = {morton_key(cells[c], L), cell_id(cells[c], n)};
  std::sort(order.begin(), order.end());
  std::unordered_map<uint64_t, int> own;
  own.reserve(cells.size() * 2);
  const int64_t N = (int64_t)cells.size(), base = N / P, extra = N % P;
  int64_t k = 0;
  for (int p = 0; p < P; ++p) {
    const int64_t size = base + (p < extra ? 1 : 0);
    for (int64_t i = 0; i < size; ++i) own[order[k + i].second] = p;
    k += size;
  }
  return own;
}

double eta_w(const std::vector<std::vector<MCell>> &levels, const std::vector<std::unordered_map<uint64_t, int>> &own,
             int P, int n) {
  double total = 0, crit = 0;
  for (size_t j = 0; j < levels.size(); ++j) {
    std::vector<int64_t> cnt(P, 0);
    for (const MCell &c : levels[j]) cnt[own[j].at(cell_id(c, n))] += 1;
    total += (double)levels[j].size();
    crit += (double)*std::max_element(cnt.begin(), cnt.end());
  }
  return total / ((double)P * crit);
}

}  // namespace

void amr_mg_metrics(int n, const std::vector<int> &level, const std::vector<int> &idx, int P, double out[4]) {
  int L = 0;
  for (int l : level) L = std::max(L, l);
  std::vector<MCell> leafs(level.size());
  for (size_t c = 0; c < level.size(); ++c) leafs[c] = {level[c], idx[3 * c], idx[3 * c + 1], idx[3 * c + 2]};
  // global coarsening: the library's coarsening, each level partitioned on its own
  std::vector<std::vector<MCell>> G{leafs};
  std::vector<int> lv = level, ix = idx;
  while (*std::max_element(lv.begin(), lv.end()) > 0) {
    std::vector<int> lc, xc;
    amr_coarsen(n, lv, ix, lc, xc);
    MFS_REQUIRE(lc.size() < lv.size(), MFS_EINVAL, "global coarsening made no progress");
    lv.swap(lc);
    ix.swap(xc);
    std::vector<MCell> cs(lv.size());
    for (size_t c = 0; c < lv.size(); ++c) cs[c] = {lv[c], ix[3 * c], ix[3 * c + 1], ix[3 * c + 2]};
    G.push_back(std::move(cs));
  }
  std::vector<std::unordered_map<uint64_t, int>> gown;
  for (const auto &cs : G) gown.push_back(morton_partition(cs, P, L, n));
  int64_t local = 0, tot = 0;
  for (size_t j = 0; j + 1 < G.size(); ++j)
    for (const MCell &c : G[j]) {
      auto it = gown[j + 1].find(cell_id(c, n));
      const int to = it != gown[j + 1].end() ? it->second : gown[j + 1].at(cell_id(parent_of(c), n));
      local += gown[j].at(cell_id(c, n)) == to;
      ++tot;
    }
  out[0] = eta_w(G, gown, P, n);
  out[1] = tot ? (double)local / (double)tot : 1.0;
  // local smoothing: every cell of each refinement level; a leaf keeps its
  // owner, a parent takes the owner of its first child in Morton order
  std::vector<std::vector<MCell>> S(L + 1);
  std::unordered_map<uint64_t, int> seen;
  seen.reserve(leafs.size() * 3);
  for (const MCell &c0 : leafs) {
    MCell c = c0;
    while (true) {
      if (!seen.emplace(cell_id(c, n), 1).second) break;
      S[c.l].push_back(c);
      if (c.l == 0) break;
      c = parent_of(c);
    }
  }
  std::vector<std::unordered_map<uint64_t, int>> lown(L + 1);
  const auto &leaf_own = gown[0];
  for (int l = L; l >= 0; --l) {
    std::unordered_map<uint64_t, std::pair<uint64_t, int>> first;  // parent -> (key, owner) of its first child
    first.reserve(S[l].size() * 2);
    lown[l].reserve(S[l].size() * 2);
    if (l < L)
      for (const MCell &c : S[l + 1]) {
        const uint64_t pid = cell_id(parent_of(c), n), key = morton_key(c, L);
        const int o = lown[l + 1].at(cell_id(c, n));
        auto it = first.find(pid);
        if (it == first.end() || key < it->second.first) first[pid] = {key, o};
      }
    for (const MCell &c : S[l]) {
      const uint64_t id = cell_id(c, n);
      auto it = leaf_own.find(id);
      lown[l][id] = it != leaf_own.end() ? it->second : first.at(id).second;
    }
  }
  local = tot = 0;
  for (int l = L; l > 0; --l)
    for (const MCell &c : S[l]) {
      local += lown[l].at(cell_id(c, n)) == lown[l - 1].at(cell_id(parent_of(c), n));
      ++tot;
    }
  out[2] = eta_w(S, lown, P, n);
  out[3] = tot ? (double)local / (double)tot : 1.0;
}

}  // namespace mfs

// 1D nodes, quadrature and Lagrange tables computed on the host in FP64.
//
// Gauss-Lobatto-Legendre nodes are the end points plus the roots of P_k',
// Gauss-Legendre points the roots of P_q; both by Newton's method on the
// three-term Legendre recurrence, mapped from [-1, 1] to [0, 1].
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "internal.h"

namespace mfs {

namespace {
thread_local char g_err[1024] = "";

// P_n(x) and P_n'(x) by the three-term recurrence
void legendre(int n, double x, double &p, double &dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n)
  dp = n * (p0 - x * p1) / (1.0 - x * x);
}
}  // namespace

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char *get_error() { return g_err; }

std::vector<double> gll_nodes(int k) {
  std::vector<double> t(k + 1);
  t[0] = -1.0;
  t[k] = 1.0;
  for (int j = 1; j < k; ++j) {
    double x = -std::cos(M_PI * j / k);
    for (int it = 0; it < 100; ++it) {
      // f = P_k', f' = P_k'' from the Legendre equation
      double p, dp;
      legendre(k, x, p, dp);
      double d2p = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    t[j] = x;
  }
  std::vector<double> out(k + 1);
  for (int j = 0; j <= k; ++j) out[j] = 0.5 * (t[j] + 1.0);
  // exact symmetry about 1/2
  for (int j = 0; j <= k / 2; ++j) {
    double a = 0.5 * (out[j] + 1.0 - out[k - j]);
    out[j] = a;
    out[k - j] = 1.0 - a;
  }
  if (k % 2 == 0) out[k / 2] = 0.5;
  return out;
}

void gauss_rule(int q, std::vector<double> &x, std::vector<double> &w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double p = 0, dp = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(q, t, p, dp);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    legendre(q, t, p, dp);
    x[i] = 0.5 * (t + 1.0);
    w[i] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/((1-t^2)P'^2) halved for [0,1]
  }
  for (int i = 0; i < q / 2; ++i) {
    double a = 0.5 * (x[i] + 1.0 - x[q - 1 - i]);
    x[i] = a;
    x[q - 1 - i] = 1.0 - a;
    double b = 0.5 * (w[i] + w[q - 1 - i]);
    w[i] = w[q - 1 - i] = b;
  }
  if (q % 2 == 1) x[q / 2] = 0.5;
}

std::vector<double> lagrange_values(const std::vector<double> &nodes, const std::vector<double> &x) {
  const int n = (int)nodes.size(), m = (int)x.size();
  std::vector<double> V((size_t)m * n, 1.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 1.0;
      for (int r = 0; r < n; ++r)
        if (r != j) v *= (x[i] - nodes[r]) / (nodes[j] - nodes[r]);
      V[(size_t)i * n + j] = v;
    }
  return V;
}

std::vector<double> lagrange_derivs(const std::vector<double> &nodes, const std::vector<double> &x) {
  const int n = (int)nodes.size(), m = (int)x.size();
  std::vector<double> D((size_t)m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) {
        if (l == j) continue;
        double t = 1.0 / (nodes[j] - nodes[l]);
        for (int r = 0; r < n; ++r)
          if (r != j && r != l) t *= (x[i] - nodes[r]) / (nodes[j] - nodes[r]);
        s += t;
      }
      D[(size_t)i * n + j] = s;
    }
  return D;
}

std::vector<double> make_tables(int k, int kp) {
  std::vector<double> tab(TAB_SIZE, 0.0);
  const int q = k + 1;
  std::vector<double> gx, gw;
  gauss_rule(q, gx, gw);
  auto put = [&](int off, const std::vector<double> &M, int rows, int cols) {
    for (int i = 0; i < rows; ++i)
      for (int j = 0; j < cols; ++j) tab[off + i * MAXQ + j] = M[(size_t)i * cols + j];
  };
  auto nodes = gll_nodes(k);
  put(TAB_S, lagrange_values(nodes, gx), q, k + 1);
  put(TAB_D, lagrange_derivs(gx, gx), q, q);
  put(TAB_DS, lagrange_derivs(nodes, gx), q, k + 1);
  if (kp > 0) {
    auto pn = gll_nodes(kp);
    put(TAB_SP, lagrange_values(pn, gx), q, kp + 1);
    put(TAB_DSP, lagrange_derivs(pn, gx), q, kp + 1);
  }
  for (int i = 0; i < q; ++i) {
    tab[TAB_W + i] = gw[i];
    tab[TAB_X + i] = gx[i];
  }
  return tab;
}

std::vector<double> h_embedding(int k) {
  auto nodes = gll_nodes(k);
  std::vector<double> fine(2 * k + 1);
  for (int i = 0; i <= k; ++i) fine[i] = 0.5 * nodes[i];
  for (int i = 1; i <= k; ++i) fine[k + i] = 0.5 + 0.5 * nodes[i];
  return lagrange_values(nodes, fine);
}

std::vector<double> p_embedding(int kf, int kc) { return lagrange_values(gll_nodes(kc), gll_nodes(kf)); }

}  // namespace mfs

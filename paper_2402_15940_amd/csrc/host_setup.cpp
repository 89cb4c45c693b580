// Host-side setup: 1D nodes/quadrature/basis tables and the integer maps of a
// structured hexahedral lattice.  Runs once per space/operator; no GPU needed.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace pafem {

namespace {

// P_n(t) and P_{n-1}(t) by the three-term recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}.
void legendre_pair(int n, double t, double& pn, double& pnm1) {
  double p0 = 1.0, p1 = t;
  if (n == 0) {
    pn = 1.0;
    pnm1 = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pnm1 = p0;
}

}  // namespace

void gll_nodes(int p, double* x) {
  // Interior nodes are the roots of P_p' on (-1,1).  With
  //   g(t)  = P_p'(t)  = p (P_{p-1} - t P_p) / (1 - t^2)
  //   g'(t) = (2 t g - p (p+1) P_p) / (1 - t^2)   (Legendre's equation)
  // Newton's method started from the Chebyshev-Gauss-Lobatto points converges
  // quadratically.  The result is symmetrised about 0 and mapped to [0,1].
  std::vector<double> t(p + 1);
  t[0] = -1.0;
  t[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double ti = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, pnm1;
      legendre_pair(p, ti, pn, pnm1);
      double om = 1.0 - ti * ti;
      double g = p * (pnm1 - ti * pn) / om;
      double dg = (2.0 * ti * g - p * (p + 1.0) * pn) / om;
      double step = g / dg;
      ti -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    t[i] = ti;
  }
  for (int i = 0; i <= p / 2; ++i) {
    double s = 0.5 * (t[p - i] - t[i]);
    t[i] = -s;
    t[p - i] = s;
  }
  if (p % 2 == 0) t[p / 2] = 0.0;
  for (int i = 0; i <= p; ++i) x[i] = 0.5 * (t[i] + 1.0);
  x[0] = 0.0;
  x[p] = 1.0;
}

void gauss_legendre(int q, double* x, double* w) {
  // Roots of P_q by Newton from cos(pi (i + 3/4) / (q + 1/2)); weights
  // 2 / ((1 - t^2) P_q'(t)^2) on [-1,1], halved for [0,1].
  std::vector<double> t(q), wt(q);
  for (int i = 0; i < q; ++i) {
    double ti = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pn, pnm1;
      legendre_pair(q, ti, pn, pnm1);
      dp = q * (ti * pn - pnm1) / (ti * ti - 1.0);
      double step = pn / dp;
      ti -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    double pn, pnm1;
    legendre_pair(q, ti, pn, pnm1);
    dp = q * (ti * pn - pnm1) / (ti * ti - 1.0);
    t[i] = ti;
    wt[i] = 2.0 / ((1.0 - ti * ti) * dp * dp);
  }
  // ascending order, symmetrised
  std::reverse(t.begin(), t.end());
  std::reverse(wt.begin(), wt.end());
  for (int i = 0; i < q / 2; ++i) {
    double s = 0.5 * (t[q - 1 - i] - t[i]);
    double ws = 0.5 * (wt[i] + wt[q - 1 - i]);
    t[i] = -s;
    t[q - 1 - i] = s;
    wt[i] = wt[q - 1 - i] = ws;
  }
  if (q % 2 == 1) t[q / 2] = 0.0;
  for (int i = 0; i < q; ++i) {
    x[i] = 0.5 * (t[i] + 1.0);
    w[i] = 0.5 * wt[i];
  }
}

void lagrange_tables(int n, const double* nodes, int m, const double* x, double* B, double* G) {
  // Barycentric weights lambda_a = 1 / prod_{b != a} (x_a - x_b).  For a point
  // away from the nodes: l_a(x) = (lambda_a / (x - x_a)) / sum_b lambda_b / (x - x_b)
  // and l_a'(x) = l_a(x) * sum_{b != a} 1 / (x - x_b).  At a node, l_a = delta and
  // l_a' comes from the differentiation-matrix formula.
  std::vector<double> lam(n);
  for (int a = 0; a < n; ++a) {
    double prod = 1.0;
    for (int b = 0; b < n; ++b)
      if (b != a) prod *= (nodes[a] - nodes[b]);
    lam[a] = 1.0 / prod;
  }
  for (int i = 0; i < m; ++i) {
    int hit = -1;
    for (int a = 0; a < n; ++a)
      if (x[i] == nodes[a]) hit = a;
    if (hit >= 0) {
      for (int a = 0; a < n; ++a) {
        B[i * n + a] = (a == hit) ? 1.0 : 0.0;
        double d;
        if (a != hit) {
          d = (lam[a] / lam[hit]) / (nodes[hit] - nodes[a]);
        } else {
          d = 0.0;
          for (int b = 0; b < n; ++b)
            if (b != hit) d += 1.0 / (nodes[hit] - nodes[b]);
        }
        G[i * n + a] = d;
      }
      continue;
    }
    double den = 0.0;
    for (int a = 0; a < n; ++a) den += lam[a] / (x[i] - nodes[a]);
    for (int a = 0; a < n; ++a) {
      double la = (lam[a] / (x[i] - nodes[a])) / den;
      double s = 0.0;
      for (int b = 0; b < n; ++b)
        if (b != a) s += 1.0 / (x[i] - nodes[b]);
      B[i * n + a] = la;
      G[i * n + a] = la * s;
    }
  }
}

void build_restriction(int nx, int ny, int nz, int p, std::vector<int32_t>& E) {
  const int n = p + 1;
  const int64_t lx = (int64_t)nx * p + 1, ly = (int64_t)ny * p + 1;
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t nl = (int64_t)n * n * n;
  E.resize(ne * nl);
  int64_t pos = 0;
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex)
        for (int c = 0; c < n; ++c)
          for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
              int64_t I = (int64_t)ex * p + a, J = (int64_t)ey * p + b, K = (int64_t)ez * p + c;
              E[pos++] = (int32_t)(I + lx * (J + ly * K));
            }
}

void build_restriction_transpose(const std::vector<int32_t>& E, int64_t ndofs,
                                 std::vector<int32_t>& off, std::vector<int32_t>& idx) {
  // Counting sort by dof; positions within a row stay ascending.
  off.assign(ndofs + 1, 0);
  for (int32_t g : E) off[g + 1]++;
  for (int64_t i = 0; i < ndofs; ++i) off[i + 1] += off[i];
  idx.resize(E.size());
  std::vector<int32_t> cur(off.begin(), off.end() - 1);
  for (size_t k = 0; k < E.size(); ++k) idx[cur[E[k]]++] = (int32_t)k;
}

void build_essential(int nx, int ny, int nz, int p, std::vector<int32_t>& ess,
                     std::vector<uint8_t>& mask) {
  const int64_t lx = (int64_t)nx * p + 1, ly = (int64_t)ny * p + 1, lz = (int64_t)nz * p + 1;
  mask.assign(lx * ly * lz, 0);
  ess.clear();
  for (int64_t K = 0; K < lz; ++K)
    for (int64_t J = 0; J < ly; ++J)
      for (int64_t I = 0; I < lx; ++I) {
        bool b = I == 0 || I == lx - 1 || J == 0 || J == ly - 1 || K == 0 || K == lz - 1;
        if (b) {
          int64_t g = I + lx * (J + ly * K);
          mask[g] = 1;
          ess.push_back((int32_t)g);
        }
      }
}

}  // namespace pafem

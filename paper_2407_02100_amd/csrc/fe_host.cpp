// Host-side FP64 set-up mathematics of libvps.  See fe_host.h.
#include "fe_host.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace vps {

void legendre(int n, double x, double* p, double* dp, double* d2p) {
  // Three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1};
  // derivatives from P_k' recurrence differentiated term by term.
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0, s0 = 0.0, s1 = 0.0;
  if (n == 0) {
    *p = 1.0; *dp = 0.0; *d2p = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    const double d2 = ((2.0 * k + 1.0) * (p1 + x * d1) - k * d0) / (k + 1.0);
    const double s2 = ((2.0 * k + 1.0) * (2.0 * d1 + x * s1) - k * s0) / (k + 1.0);
    p0 = p1; p1 = p2; d0 = d1; d1 = d2; s0 = s1; s1 = s2;
  }
  *p = p1; *dp = d1; *d2p = s1;
}

std::vector<double> gll_points(int k) {
  std::vector<double> x(k + 1);
  x[0] = -1.0;
  x[k] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i < k; ++i) {
    // start at the Chebyshev-Gauss-Lobatto point, Newton on P_k'(x) = 0
    double t = -std::cos(pi * i / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp, d2p;
      legendre(k, t, &p, &dp, &d2p);
      const double step = dp / d2p;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[i] = t;
  }
  for (double& v : x) v = 0.5 * (v + 1.0);
  return x;
}

void gauss_rule(int n, std::vector<double>* x, std::vector<double>* w) {
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double t = -std::cos(pi * (i + 0.75) / (n + 0.5));
    double p = 0, dp = 0, d2p = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, &p, &dp, &d2p);
      const double step = p / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre(n, t, &p, &dp, &d2p);
    (*x)[i] = 0.5 * (t + 1.0);
    (*w)[i] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/((1-t^2)P'^2) on [-1,1], halved
  }
}

double lagrange(const std::vector<double>& nodes, int a, double x) {
  double v = 1.0;
  for (int b = 0; b < (int)nodes.size(); ++b)
    if (b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
  return v;
}

double lagrange_deriv(const std::vector<double>& nodes, int a, double x) {
  double s = 0.0;
  const int n = (int)nodes.size();
  for (int c = 0; c < n; ++c) {
    if (c == a) continue;
    double t = 1.0 / (nodes[a] - nodes[c]);
    for (int b = 0; b < n; ++b)
      if (b != a && b != c) t *= (x - nodes[b]) / (nodes[a] - nodes[b]);
    s += t;
  }
  return s;
}

void reference_matrices(int k, Mat* M, Mat* K) {
  const std::vector<double> nodes = gll_points(k);
  std::vector<double> xq, wq;
  gauss_rule(k + 2, &xq, &wq);
  const int n = k + 1;
  M->assign(n * n, 0.0);
  K->assign(n * n, 0.0);
  for (int q = 0; q < (int)xq.size(); ++q) {
    std::vector<double> v(n), d(n);
    for (int a = 0; a < n; ++a) {
      v[a] = lagrange(nodes, a, xq[q]);
      d[a] = lagrange_deriv(nodes, a, xq[q]);
    }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        (*M)[a * n + b] += wq[q] * v[a] * v[b];
        (*K)[a * n + b] += wq[q] * d[a] * d[b];
      }
  }
}

void assemble_1d(int k, int ncell, double h, Mat* M, Mat* K, const double* cell_weight) {
  Mat Mr, Kr;
  reference_matrices(k, &Mr, &Kr);
  const int n = k * ncell + 1;
  M->assign(n * n, 0.0);
  K->assign(n * n, 0.0);
  for (int c = 0; c < ncell; ++c) {
    const double wgt = cell_weight ? cell_weight[c] : 1.0;
    for (int a = 0; a <= k; ++a)
      for (int b = 0; b <= k; ++b) {
        (*M)[(c * k + a) * n + c * k + b] += wgt * h * Mr[a * (k + 1) + b];
        (*K)[(c * k + a) * n + c * k + b] += wgt * Kr[a * (k + 1) + b] / h;
      }
  }
}

static bool cholesky_lower(int n, Mat* A) {
  // A = L L^T, L overwrites the lower triangle; upper triangle zeroed.
  Mat& a = *A;
  for (int j = 0; j < n; ++j) {
    double d = a[j * n + j];
    for (int p = 0; p < j; ++p) d -= a[j * n + p] * a[j * n + p];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    a[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = a[i * n + j];
      const double* ri = &a[i * n];
      const double* rj = &a[j * n];
      for (int p = 0; p < j; ++p) s -= ri[p] * rj[p];
      a[i * n + j] = s / d;
    }
    for (int i = 0; i < j; ++i) a[i * n + j] = 0.0;
  }
  return true;
}

void gen_eig(int n, const Mat& M, const Mat& K, Mat* T, std::vector<double>* lambda) {
  Mat L = M;
  cholesky_lower(n, &L);
  // Linv = L^{-1} (lower triangular) by forward substitution on unit vectors
  Mat Li(n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int p = 0; p < i; ++p) s -= L[i * n + p] * Li[p * n + c];
      Li[i * n + c] = s / L[i * n + i];
    }
  }
  // C = Linv K Linv^T (symmetric)
  Mat tmp(n * n, 0.0), C(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += Li[i * n + p] * K[p * n + j];
      tmp[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += tmp[i * n + p] * Li[j * n + p];
      C[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) C[i * n + j] = C[j * n + i] = 0.5 * (C[i * n + j] + C[j * n + i]);
  // cyclic Jacobi: C = Q diag Q^T
  Mat Q(n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += C[i * n + j] * C[i * n + j];
        if (i != j) off += C[i * n + j] * C[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          const double crp = C[r * n + p], crq = C[r * n + q];
          C[r * n + p] = c * crp - s * crq;
          C[r * n + q] = s * crp + c * crq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          const double cpr = C[p * n + r], cqr = C[q * n + r];
          C[p * n + r] = c * cpr - s * cqr;
          C[q * n + r] = s * cpr + c * cqr;
        }
        for (int r = 0; r < n; ++r) {
          const double qrp = Q[r * n + p], qrq = Q[r * n + q];
          Q[r * n + p] = c * qrp - s * qrq;
          Q[r * n + q] = s * qrp + c * qrq;
        }
      }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return C[a * n + a] < C[b * n + b]; });
  // T = L^{-T} Q: T[i][m] = sum_p Linv[p][i] Q[p][m]
  T->assign(n * n, 0.0);
  lambda->assign(n, 0.0);
  for (int mi = 0; mi < n; ++mi) {
    const int m = order[mi];
    (*lambda)[mi] = C[m * n + m];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += Li[p * n + i] * Q[p * n + m];
      (*T)[i * n + mi] = s;
    }
  }
}

bool fdm_even_odd(int q, const Mat& T, Mat* Te, Mat* To, std::vector<int>* order) {
  const int ne = (q + 1) / 2, no = (q - 1) / 2;
  std::vector<int> ev, od;
  for (int m = 0; m < q; ++m) {
    double scale = 0.0, es = 0.0, os = 0.0;
    for (int i = 0; i < q; ++i) scale = std::max(scale, std::fabs(T[i * q + m]));
    for (int i = 0; i < q; ++i) {
      es = std::max(es, std::fabs(T[(q - 1 - i) * q + m] - T[i * q + m]));
      os = std::max(os, std::fabs(T[(q - 1 - i) * q + m] + T[i * q + m]));
    }
    if (es <= 1e-10 * scale) ev.push_back(m);
    else if (os <= 1e-10 * scale) od.push_back(m);
    else return false;
  }
  if ((int)ev.size() != ne || (int)od.size() != no) return false;
  Te->assign(ne * ne, 0.0);
  To->assign(std::max(no * no, 1), 0.0);
  for (int j = 0; j < ne; ++j)
    for (int i = 0; i < ne; ++i) (*Te)[i * ne + j] = T[i * q + ev[j]];
  for (int j = 0; j < no; ++j)
    for (int i = 0; i < no; ++i) (*To)[i * no + j] = T[i * q + od[j]];
  order->clear();
  for (int m : ev) order->push_back(m);
  for (int m : od) order->push_back(m);
  return true;
}

bool spd_inverse(int n, Mat* A) {
  Mat L = *A;
  if (!cholesky_lower(n, &L)) return false;
  // W = L^{-1}
  Mat W(static_cast<size_t>(n) * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = c; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      const double* li = &L[static_cast<size_t>(i) * n];
      for (int p = c; p < i; ++p) s -= li[p] * W[static_cast<size_t>(p) * n + c];
      W[static_cast<size_t>(i) * n + c] = s / li[i];
    }
  }
  // A^{-1} = W^T W
  Mat& a = *A;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double s = 0.0;
      for (int p = j; p < n; ++p) s += W[static_cast<size_t>(p) * n + i] * W[static_cast<size_t>(p) * n + j];
      a[static_cast<size_t>(i) * n + j] = s;
      a[static_cast<size_t>(j) * n + i] = s;
    }
  return true;
}

void prolongation_1d(int k, int nc, Mat* P) {
  const std::vector<double> xi = gll_points(k);
  const int nf = 2 * k * nc + 1, ncn = k * nc + 1;
  P->assign(static_cast<size_t>(nf) * ncn, 0.0);
  for (int f = 0; f < nf; ++f) {
    // fine node f: fine cell fc = f / k (last node belongs to the last cell)
    int fc = f / k, a = f % k;
    if (fc == 2 * nc) { fc = 2 * nc - 1; a = k; }
    const double xf = (fc + xi[a]) / (2.0 * nc);
    const int c = std::min(fc / 2, nc - 1);
    const double loc = xf * nc - c;
    for (int b = 0; b <= k; ++b) (*P)[static_cast<size_t>(f) * ncn + c * k + b] = lagrange(xi, b, loc);
  }
}

}  // namespace vps

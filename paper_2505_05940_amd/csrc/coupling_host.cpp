// Host FP64 builder of the scaled von Karman coupling tensor for the sine
// in-plane family (paper: Sec. 3.1, coupling-coefficient equations).
//
// With Phi_i = c sin(al_i x) sin(be_i y), c = 2/sqrt(Lx Ly), al = m pi/Lx,
// be = q pi/Ly, the von Karman operator (paper: von Karman operator
// equation, f_xx g_yy + f_yy g_xx - 2 f_xy g_xy) gives
//   L(Phi_i, Phi_j) = c^2 (al_i^2 be_j^2 + be_i^2 al_j^2) s_i s_j s'_i s'_j
//                   - 2 c^2 al_i be_i al_j be_j  co_i co_j co'_i co'_j,
// so every entry factorises into 1-D integrals over x and over y of three
// trigonometric factors.  Those are tabulated once per instance, by
// Gauss-Legendre quadrature converged to rounding (exact integrals) or by
// the midpoint rule on the requested grid, and the N_in x N_t x N_t entries
// are assembled from the tables on several threads.
#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "../../include/modal.h"

namespace {

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Quadrature points/weights on [0, L]: midpoint (cells > 0) or Gauss.
void rule(double L, int cells, int gauss_n, std::vector<double>& x, std::vector<double>& w) {
  if (cells > 0) {
    x.resize(cells);
    w.assign(cells, L / cells);
    for (int i = 0; i < cells; ++i) x[i] = (i + 0.5) * L / cells;
    return;
  }
  gauss_legendre(gauss_n, x, w);
  for (size_t i = 0; i < x.size(); ++i) {
    x[i] = 0.5 * L * (x[i] + 1.0);
    w[i] *= 0.5 * L;
  }
}

// T_s[a][i][j] = int sin(a u) sin(i u) sin(j u),  T_c[a][i][j] = int sin(a u) cos(i u) cos(j u)
// over [0, L], u = pi x / L; a in 1..A, i, j in 1..M (index 0 unused).
struct Tables {
  int A, M;
  std::vector<double> s, c;
  double S(int a, int i, int j) const { return s[((size_t)a * (M + 1) + i) * (M + 1) + j]; }
  double C(int a, int i, int j) const { return c[((size_t)a * (M + 1) + i) * (M + 1) + j]; }
};

Tables tabulate(double L, int A, int M, int cells) {
  Tables t{A, M, {}, {}};
  const size_t sz = (size_t)(A + 1) * (M + 1) * (M + 1);
  t.s.assign(sz, 0.0);
  t.c.assign(sz, 0.0);
  std::vector<double> x, w;
  // the integrands are trigonometric polynomials of frequency <= A + 2M
  // half-waves; this many Gauss points integrates them to rounding
  rule(L, cells, 2 * (A + 2 * M) + 48, x, w);
  const size_t G = x.size();
  std::vector<double> sn((size_t)(std::max(A, M) + 1) * G), cs((size_t)(M + 1) * G);
  for (int k = 0; k <= std::max(A, M); ++k)
    for (size_t g = 0; g < G; ++g) sn[k * G + g] = std::sin(k * M_PI * x[g] / L);
  for (int k = 0; k <= M; ++k)
    for (size_t g = 0; g < G; ++g) cs[k * G + g] = std::cos(k * M_PI * x[g] / L);
  for (int a = 1; a <= A; ++a)
    for (int i = 1; i <= M; ++i)
      for (int j = i; j <= M; ++j) {
        double vs = 0.0, vc = 0.0;
        // Both integrands are sums of sin(k u) with k = a +- i +- j, all of
        // the parity of a + i + j; for even k each integral over [0, pi] is
        // zero, and so is its midpoint sum on the symmetric grid.  Those
        // entries are set to that exact value rather than left as rounding
        // noise, which keeps the tensor's parity blocks exactly empty.
        if ((a + i + j) % 2 == 0) continue;
        for (size_t g = 0; g < G; ++g) {
          const double wa = w[g] * sn[a * G + g];
          vs += wa * sn[i * G + g] * sn[j * G + g];
          vc += wa * cs[i * G + g] * cs[j * G + g];
        }
        const size_t ij = ((size_t)a * (M + 1) + i) * (M + 1) + j;
        const size_t ji = ((size_t)a * (M + 1) + j) * (M + 1) + i;
        t.s[ij] = t.s[ji] = vs;
        t.c[ij] = t.c[ji] = vc;
      }
  return t;
}

thread_local std::string g_cerr;

}  // namespace

extern "C" int modal_vk_coupling_sine(double Lx, double Ly, int32_t n_t, const int32_t* m,
                                      const int32_t* q, int32_t n_in, const int32_t* a,
                                      const int32_t* b, int32_t nx, int32_t ny,
                                      const double* scale_n, float* out, int32_t threads) {
  if (!(Lx > 0) || !(Ly > 0) || n_t < 1 || n_in < 1 || !m || !q || !a || !b || !scale_n || !out)
    return MODAL_EINVAL;
  if ((nx > 0) != (ny > 0) || nx < 0 || ny < 0) return MODAL_EINVAL;
  int Mx = 0, My = 0, Ax = 0, Ay = 0;
  for (int i = 0; i < n_t; ++i) {
    if (m[i] < 1 || q[i] < 1) return MODAL_EINVAL;
    Mx = std::max(Mx, (int)m[i]);
    My = std::max(My, (int)q[i]);
  }
  for (int i = 0; i < n_in; ++i) {
    if (a[i] < 1 || b[i] < 1) return MODAL_EINVAL;
    Ax = std::max(Ax, (int)a[i]);
    Ay = std::max(Ay, (int)b[i]);
  }
  const Tables tx = tabulate(Lx, Ax, Mx, nx);
  const Tables ty = tabulate(Ly, Ay, My, ny);
  const double c3 = std::pow(2.0 / std::sqrt(Lx * Ly), 3);
  std::vector<double> al(n_t), be(n_t);
  for (int i = 0; i < n_t; ++i) {
    al[i] = m[i] * M_PI / Lx;
    be[i] = q[i] * M_PI / Ly;
  }
  int nth = threads > 0 ? threads : (int)std::thread::hardware_concurrency();
  nth = std::max(1, std::min(nth, n_in));
  auto work = [&](int t) {
    for (int n = t; n < n_in; n += nth) {
      const double sc = scale_n[n] * c3;
      float* Hn = out + (size_t)n * n_t * n_t;
      for (int i = 0; i < n_t; ++i) {
        for (int j = i; j < n_t; ++j) {
          const double A = al[i] * al[i] * be[j] * be[j] + be[i] * be[i] * al[j] * al[j];
          const double B = 2.0 * al[i] * be[i] * al[j] * be[j];
          const double v = A * tx.S(a[n], m[i], m[j]) * ty.S(b[n], q[i], q[j]) -
                           B * tx.C(a[n], m[i], m[j]) * ty.C(b[n], q[i], q[j]);
          const float f = (float)(sc * v);
          Hn[(size_t)i * n_t + j] = f;
          Hn[(size_t)j * n_t + i] = f;
        }
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  return MODAL_OK;
}

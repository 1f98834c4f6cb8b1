// FP64 CPU oracle for batches of von Karman plates: the whole chain of the
// Python oracle (oracle/instances.py, oracle/coupling.py, oracle/simulate.py)
// written again as a plain C++ loop, for timing the oracle on all host cores.
//
// TEST INFRASTRUCTURE ONLY: called by tests/ (against the Python oracle) and
// by the CPU-baseline leg of bench.py; the product never links or runs it,
// and it shares no code with the product.
//
// Per plate (paper, Sec. 3 and Sec. 3.1-3.2):
//  * transverse modes of the simply supported rectangle, the n_t smallest
//    lambda = (m pi/Lx)^2 + (q pi/Ly)^2, ties broken by (lambda, m, q);
//  * the plate area that puts mode n_t at the target frequency
//    (rho_s w^2 S^2 - T0 Lam S - D Lam^2 = 0, Lam = lambda_N at unit area),
//    Lx = sqrt(S/a), Ly = sqrt(S a);
//  * omega^2 = (D lambda^2 + T0 lambda)/rho_s, gamma = g0 + g1 omega;
//  * in-plane modes of the sine family, the n_in smallest lambda_n, and the
//    scaled coupling tensor Ht[n][i][j] = sqrt(E/(2 rho)) H[n][i][j]/lambda_n
//    with H the exact integral of Psi_n L(Phi_i, Phi_j): with c = 2/sqrt(Lx Ly),
//    alpha = m pi/Lx, beta = q pi/Ly,
//      H = c^3 ((al_i^2 be_j^2 + be_i^2 al_j^2) Ixsss Iysss
//               - 2 al_i be_i al_j be_j Ixscc Iyscc),
//    each 1-D integral of three sines (or a sine and two cosines) a sum of
//    four integrals of single sines;
//  * the strike projection X_k = dA sum w0 Phi_k on the midpoint grid, the
//    pickup c_k = Phi_k(x_o), release from rest;
//  * the Stormer-Verlet recursion X+ = g X + p X- - r F(X) with
//    r = T^2/(1 + gamma T), g = r (2/T^2 - omega^2), p = r (gamma/T - 1/T^2),
//    F_k = sum_n eta_n V[n][k], V[n][k] = sum_j Ht[n][k][j] X_j,
//    eta_n = sum_k V[n][k] X_k, and the output y^n = c . X^n.
// OpenMP runs the plates on all threads, largest first.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <tuple>
#include <vector>

namespace {

struct Params {
  double aspect, top_hz, h, E, nu, rho, T0, g0, g1, xc, yc, amp, radius_rel, xo, yo;
  int n_t, n_in, nx, ny;
};

// parameter vector layout shared with the Python wrapper
constexpr int kDoubles = 15;
constexpr int kInts = 4;

Params unpack(const double* d, const int32_t* i) {
  return Params{d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7], d[8], d[9], d[10], d[11], d[12], d[13], d[14],
                i[0], i[1], i[2], i[3]};
}

void plate_modes(double Lx, double Ly, int n, std::vector<int>& m, std::vector<int>& q,
                 std::vector<double>& lam) {
  std::vector<std::tuple<double, int, int>> c;
  c.reserve((size_t)n * n);
  for (int a = 1; a <= n; ++a)
    for (int b = 1; b <= n; ++b) {
      const double l = (a * M_PI / Lx) * (a * M_PI / Lx) + (b * M_PI / Ly) * (b * M_PI / Ly);
      c.emplace_back(l, a, b);
    }
  std::partial_sort(c.begin(), c.begin() + n, c.end());
  m.resize(n);
  q.resize(n);
  lam.resize(n);
  for (int k = 0; k < n; ++k) std::tie(lam[k], m[k], q[k]) = c[k];
}

// integral over [0, L] of sin(k pi x / L): 2L/(k pi) for odd k, else 0
double sin_int(int k, double L) { return (k % 2 != 0) ? 2.0 * L / (M_PI * k) : 0.0; }
double int_sss(int a, int i, int j, double L) {
  return 0.25 * (sin_int(a + i - j, L) + sin_int(a - i + j, L) + sin_int(-a + i + j, L) - sin_int(a + i + j, L));
}
double int_scc(int a, int i, int j, double L) {
  return 0.25 * (sin_int(a + i - j, L) + sin_int(a - i + j, L) + sin_int(a + i + j, L) + sin_int(a - i - j, L));
}

struct Plate {
  int n, nin;
  double Lx, Ly;
  std::vector<double> omega, gamma, x0, c, Ht;  // Ht [nin][n][n]
};

void build(const Params& P, Plate& out) {
  const int n = P.n_t, nin = P.n_in;
  const double D = P.E * P.h * P.h * P.h / (12.0 * (1.0 - P.nu * P.nu));
  const double rho_s = P.rho * P.h;
  std::vector<int> m, q, ai, bi;
  std::vector<double> lam, lam_in;
  plate_modes(1.0 / std::sqrt(P.aspect), std::sqrt(P.aspect), n, m, q, lam);
  const double Lam = lam[n - 1];
  const double w = 2.0 * M_PI * P.top_hz;
  const double S = (P.T0 * Lam + std::sqrt((P.T0 * Lam) * (P.T0 * Lam) + 4.0 * rho_s * w * w * D * Lam * Lam)) /
                   (2.0 * rho_s * w * w);
  const double Lx = std::sqrt(S / P.aspect), Ly = std::sqrt(S * P.aspect);
  plate_modes(Lx, Ly, n, m, q, lam);
  plate_modes(Lx, Ly, nin, ai, bi, lam_in);
  out.n = n;
  out.nin = nin;
  out.Lx = Lx;
  out.Ly = Ly;
  out.omega.resize(n);
  out.gamma.resize(n);
  for (int k = 0; k < n; ++k) {
    out.omega[k] = std::sqrt((D * lam[k] * lam[k] + P.T0 * lam[k]) / rho_s);
    out.gamma[k] = P.g0 + P.g1 * out.omega[k];
  }
  // coupling tensor
  const double cc = 2.0 / std::sqrt(Lx * Ly);
  const double pref = std::sqrt(P.E / (2.0 * P.rho));
  std::vector<double> al(n), be(n);
  for (int k = 0; k < n; ++k) {
    al[k] = m[k] * M_PI / Lx;
    be[k] = q[k] * M_PI / Ly;
  }
  out.Ht.assign((size_t)nin * n * n, 0.0);
  for (int r = 0; r < nin; ++r) {
    const double s = pref / lam_in[r] * cc * cc * cc;
    double* Hr = &out.Ht[(size_t)r * n * n];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double A = al[i] * al[i] * be[j] * be[j] + be[i] * be[i] * al[j] * al[j];
        const double B = 2.0 * al[i] * be[i] * al[j] * be[j];
        Hr[(size_t)i * n + j] = s * (A * int_sss(ai[r], m[i], m[j], Lx) * int_sss(bi[r], q[i], q[j], Ly) -
                                     B * int_scc(ai[r], m[i], m[j], Lx) * int_scc(bi[r], q[i], q[j], Ly));
      }
  }
  // strike projection on the midpoint grid and pickup
  const double xc = P.xc * Lx, yc = P.yc * Ly, r0 = P.radius_rel * std::min(Lx, Ly);
  const double dA = Lx * Ly / ((double)P.nx * P.ny);
  out.x0.assign(n, 0.0);
  for (int ix = 0; ix < P.nx; ++ix) {
    const double x = (ix + 0.5) * Lx / P.nx;
    for (int iy = 0; iy < P.ny; ++iy) {
      const double y = (iy + 0.5) * Ly / P.ny;
      const double rr = std::hypot(x - xc, y - yc);
      if (!(rr < r0)) continue;
      const double w0 = 0.5 * P.amp * (1.0 + std::cos(M_PI * rr / r0));
      for (int k = 0; k < n; ++k) out.x0[k] += w0 * cc * std::sin(al[k] * x) * std::sin(be[k] * y) * dA;
    }
  }
  out.c.resize(n);
  const double xo = P.xo * Lx, yo = P.yo * Ly;
  for (int k = 0; k < n; ++k) out.c[k] = cc * std::sin(al[k] * xo) * std::sin(be[k] * yo);
}

void run(const Plate& pl, double fs, int n_steps, double* y) {
  const int n = pl.n, nin = pl.nin;
  const double T = 1.0 / fs;
  std::vector<double> g(n), p(n), r(n), X(pl.x0), Xm(pl.x0), Xn(n), V((size_t)nin * n), F(n), eta(nin);
  for (int k = 0; k < n; ++k) {
    r[k] = T * T / (1.0 + pl.gamma[k] * T);
    g[k] = r[k] * (2.0 / (T * T) - pl.omega[k] * pl.omega[k]);
    p[k] = r[k] * (pl.gamma[k] / T - 1.0 / (T * T));
  }
  for (int s = 0; s < n_steps; ++s) {
    double out = 0.0;
    for (int k = 0; k < n; ++k) out += pl.c[k] * X[k];
    y[s] = out;
    for (int a = 0; a < nin; ++a) {
      const double* Ha = &pl.Ht[(size_t)a * n * n];
      double e = 0.0;
      for (int k = 0; k < n; ++k) {
        const double* row = Ha + (size_t)k * n;
        double v = 0.0;
        for (int j = 0; j < n; ++j) v += row[j] * X[j];
        V[(size_t)a * n + k] = v;
        e += v * X[k];
      }
      eta[a] = e;
    }
    std::fill(F.begin(), F.end(), 0.0);
    for (int a = 0; a < nin; ++a)
      for (int k = 0; k < n; ++k) F[k] += eta[a] * V[(size_t)a * n + k];
    for (int k = 0; k < n; ++k) Xn[k] = g[k] * X[k] + p[k] * Xm[k] - r[k] * F[k];
    Xm.swap(X);
    X.swap(Xn);
  }
}

}  // namespace

extern "C" {

// One plate's omega, gamma, x0, c [n_t] and Ht [n_in][n_t][n_t] (caller
// memory).  Returns 0.
int oracle_vk_plate(const double* pd, const int32_t* pi, double* omega, double* gamma, double* x0, double* c,
                    double* Ht, double* LxLy) {
  Plate pl;
  build(unpack(pd, pi), pl);
  std::memcpy(omega, pl.omega.data(), sizeof(double) * pl.n);
  std::memcpy(gamma, pl.gamma.data(), sizeof(double) * pl.n);
  std::memcpy(x0, pl.x0.data(), sizeof(double) * pl.n);
  std::memcpy(c, pl.c.data(), sizeof(double) * pl.n);
  std::memcpy(Ht, pl.Ht.data(), sizeof(double) * pl.Ht.size());
  LxLy[0] = pl.Lx;
  LxLy[1] = pl.Ly;
  return 0;
}

// The batch: parameters pd [batch][15], pi [batch][4]; outputs y
// [batch][n_steps].  Builds every plate (timed in seconds[0]), then runs
// n_steps steps of every plate (seconds[1]) on `threads` OpenMP threads
// (0 = all), plates in decreasing order of n_in n_t^2.  Returns the number
// of threads used.
int oracle_vk_batch(int batch, const double* pd, const int32_t* pi, double fs, int n_steps, double* y,
                    int threads, double* seconds) {
  if (threads > 0) omp_set_num_threads(threads);
  std::vector<int> order(batch);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const double ca = (double)pi[kInts * a + 1] * pi[kInts * a] * pi[kInts * a];
    const double cb = (double)pi[kInts * b + 1] * pi[kInts * b] * pi[kInts * b];
    return ca > cb || (ca == cb && a < b);
  });
  std::vector<Plate> plates(batch);
  int used = 1;
  double t0 = omp_get_wtime();
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < batch; ++i) {
      const int b = order[i];
      build(unpack(pd + (size_t)kDoubles * b, pi + (size_t)kInts * b), plates[b]);
    }
  }
  double t1 = omp_get_wtime();
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < batch; ++i) {
    const int b = order[i];
    run(plates[b], fs, n_steps, y + (size_t)b * n_steps);
  }
  double t2 = omp_get_wtime();
  seconds[0] = t1 - t0;
  seconds[1] = t2 - t1;
  return used;
}

}  // extern "C"

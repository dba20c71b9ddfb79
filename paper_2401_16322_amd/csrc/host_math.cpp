// Host-side FP64 math of the library: damping profiles, spectrum rectangle,
// Faber ellipse and coefficients, Ricker derivatives, the source scalars of
// the augmented matrix, and the dense matrix exponential for the Krylov step.
// None of it touches the GPU.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace expw {

namespace {
thread_local std::string g_err;
}

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

const char* last_error() { return g_err.c_str(); }

bool stagger_weights(int order, double* alpha, int* K) {
  // Sec. 2.1: order 8 is printed by the paper; order 4 is the two-point
  // member of the same staggered family (exact for cubics).
  if (order == 4) {
    alpha[0] = 9.0 / 8.0;
    alpha[1] = -1.0 / 24.0;
    *K = 2;
    return true;
  }
  if (order == 8) {
    const double s = 1225.0 / 1024.0;
    alpha[0] = s;
    alpha[1] = -s / 15.0;
    alpha[2] = s / 125.0;
    alpha[3] = -s / 1715.0;
    *K = 4;
    return true;
  }
  return false;
}

bool stagger_weights_int(int order, double* w, double* beta, int* K) {
  // the same weights as integer multiples of one factor: alpha_l = beta w_l
  // (order 4: (27, -1) / 24; order 8: 1225 / (1024 * 128625) times
  // 128625 (1, -1/15, 1/125, -1/1715) = (128625, -8575, 1029, -75))
  if (order == 4) {
    w[0] = 27.0;
    w[1] = -1.0;
    *beta = 1.0 / 24.0;
    *K = 2;
    return true;
  }
  if (order == 8) {
    w[0] = 128625.0;
    w[1] = -8575.0;
    w[2] = 1029.0;
    w[3] = -75.0;
    *beta = 1225.0 / (1024.0 * 128625.0);
    *K = 4;
    return true;
  }
  return false;
}

void damping_profile(int64_t n, double h, int cells, double sigma_max, bool half, double* out) {
  // Sec. 2: sigma(d) = sigma_max (1 - d/delta)^2 for d < delta, 0 otherwise,
  // d = distance to the nearest outer node, clamped at 0 beyond the last node.
  const double delta = cells * h;
  for (int64_t i = 0; i < n; ++i) {
    const double pos = static_cast<double>(i) + (half ? 0.5 : 0.0);
    double d = std::fmin(pos, static_cast<double>(n - 1) - pos) * h;
    if (d < 0.0) d = 0.0;
    double s = 0.0;
    if (cells > 0 && sigma_max != 0.0 && d < delta) {
      const double r = 1.0 - d / delta;
      s = sigma_max * r * r;
    }
    out[i] = s;
  }
}

void faber_coefficients(double gamma, double c0, double c1, double dt, int m, double* a) {
  // Laurent coefficients of f(w) = exp(dt gamma (w + c0 + c1/w)) on |w| = 1 by
  // the trapezoidal rule, which converges geometrically for this entire
  // function of w and 1/w. M is chosen well past the decay point of the
  // coefficients (about e x / 2 with x = dt gamma max|1 -+ c1|), so aliasing
  // stays below rounding.
  const double z = dt * gamma;
  const double x = z * std::fmax(std::fabs(1.0 + c1), std::fabs(1.0 - c1));
  int M = 64;
  while (M < 2 * (m + static_cast<int>(2.0 * x) + 64)) M *= 2;
  const double two_pi = 6.283185307179586476925286766559;
  std::vector<double> mag(M), ph(M);
  for (int q = 0; q < M; ++q) {
    const double th = two_pi * q / M;
    mag[q] = std::exp(z * (c0 + (1.0 + c1) * std::cos(th)));
    ph[q] = z * (1.0 - c1) * std::sin(th);
  }
  for (int j = 0; j <= m; ++j) {
    double s = 0.0;
    for (int q = 0; q < M; ++q) {
      const double th = two_pi * q / M;
      s += mag[q] * std::cos(ph[q] - j * th);
    }
    a[j] = s / M;
  }
}

void ricker_derivatives(double t, double f_peak, double t_delay, int p, double* out) {
  // g = -(1/(2a)) d^2/dtau^2 exp(-a tau^2), and the n-th derivative of the
  // Gaussian is (-1)^n a^(n/2) H_n(sqrt(a) tau) exp(-a tau^2) with H_n the
  // physicists' Hermite polynomial, hence
  // g^(k) = -(1/(2a)) (-1)^k a^((k+2)/2) H_{k+2}(sqrt(a) tau) exp(-a tau^2).
  const double pi = 3.14159265358979323846264338327950;
  const double a = (pi * f_peak) * (pi * f_peak);
  const double tau = t - t_delay;
  const double xs = std::sqrt(a) * tau;
  const double e = std::exp(-a * tau * tau);
  std::vector<double> H(p + 3);
  H[0] = 1.0;
  H[1] = 2.0 * xs;
  for (int n = 1; n + 1 < p + 3; ++n) H[n + 1] = 2.0 * xs * H[n] - 2.0 * n * H[n - 1];
  double apow = a;  // a^((k+2)/2) for k = 0
  const double sa = std::sqrt(a);
  for (int k = 0; k < p; ++k) {
    const double sign = (k % 2 == 0) ? 1.0 : -1.0;
    out[k] = -(1.0 / (2.0 * a)) * sign * apow * H[k + 2] * e;
    apow *= sa;
  }
}

void faber_source_scalars(double gamma, double c0, double c1, int m, int p, const double* G,
                          double* q) {
  // The tail block of H~ is J (ones on the superdiagonal); the tail of the
  // Faber vectors obeys the same three-term recurrence with J in place of H.
  // The state part of H~ v_{j-1} gains W tau_{j-1}, i.e. the scalar
  // G . tau_{j-1} at the source node; divided by gamma it enters v_j.
  std::vector<double> t0(p, 0.0), t1(p, 0.0), t2(p, 0.0);
  t1[p - 1] = 1.0;  // tau_0 = e_p; t1 holds tau_{j-1}, t0 holds tau_{j-2}
  for (int j = 1; j <= m; ++j) {
    double dot = 0.0;
    for (int c = 0; c < p; ++c) dot += G[c] * t1[c];
    q[j - 1] = dot / gamma;
    const double cprev = (j == 1) ? 0.0 : (j == 2 ? 2.0 * c1 : c1);
    for (int c = 0; c < p; ++c) {
      const double Jt = (c + 1 < p) ? t1[c + 1] : 0.0;
      t2[c] = Jt / gamma - c0 * t1[c] - cprev * t0[c];
    }
    t0.swap(t1);
    t1.swap(t2);
  }
}

namespace {

void matmul(int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[i * k + l] * B[l * k + j];
      C[i * k + j] = s;
    }
}

// Solves A X = B in place (B overwritten by X) with partial pivoting.
bool lu_solve(int k, std::vector<double>& A, std::vector<double>& B) {
  for (int c = 0; c < k; ++c) {
    int piv = c;
    double best = std::fabs(A[c * k + c]);
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(A[r * k + c]) > best) {
        best = std::fabs(A[r * k + c]);
        piv = r;
      }
    if (best == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < k; ++j) {
        std::swap(A[c * k + j], A[piv * k + j]);
        std::swap(B[c * k + j], B[piv * k + j]);
      }
    for (int r = c + 1; r < k; ++r) {
      const double f = A[r * k + c] / A[c * k + c];
      if (f == 0.0) continue;
      for (int j = c; j < k; ++j) A[r * k + j] -= f * A[c * k + j];
      for (int j = 0; j < k; ++j) B[r * k + j] -= f * B[c * k + j];
    }
  }
  for (int r = k - 1; r >= 0; --r)
    for (int j = 0; j < k; ++j) {
      double s = B[r * k + j];
      for (int l = r + 1; l < k; ++l) s -= A[r * k + l] * B[l * k + j];
      B[r * k + j] = s / A[r * k + r];
    }
  return true;
}

}  // namespace

bool expm(int k, const double* A, double* E) {
  // Scaling and squaring with the diagonal [13/13] Pade approximant
  // (Higham, SIAM J. Matrix Anal. Appl. 26 (2005)): scale A by 2^-s so that
  // ||A||_1 <= theta_13, form R = (V - U)^{-1} (V + U) with U the odd and V
  // the even part of the Pade numerator, then square s times. The Pade
  // coefficients b_j = (26 - j)! 13! / (26! j! (13 - j)!) are generated here.
  const int mdeg = 13;
  const double theta13 = 5.371920351148152;
  double b[mdeg + 1];
  b[0] = 1.0;
  for (int j = 0; j < mdeg; ++j) b[j + 1] = b[j] * (mdeg - j) / ((j + 1.0) * (2.0 * mdeg - j));
  double norm1 = 0.0;
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += std::fabs(A[i * k + j]);
    norm1 = std::fmax(norm1, s);
  }
  if (!std::isfinite(norm1)) return false;
  int s = 0;
  if (norm1 > theta13) s = static_cast<int>(std::ceil(std::log2(norm1 / theta13)));
  const double scale = std::ldexp(1.0, -s);
  const size_t kk = static_cast<size_t>(k) * k;
  std::vector<double> As(kk), A2(kk), A4(kk), A6(kk), T1(kk), T2(kk), U(kk), V(kk), I(kk, 0.0);
  for (size_t i = 0; i < kk; ++i) As[i] = A[i] * scale;
  for (int i = 0; i < k; ++i) I[i * k + i] = 1.0;
  matmul(k, As.data(), As.data(), A2.data());
  matmul(k, A2.data(), A2.data(), A4.data());
  matmul(k, A4.data(), A2.data(), A6.data());
  // U = A [A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I]
  for (size_t i = 0; i < kk; ++i) T1[i] = b[13] * A6[i] + b[11] * A4[i] + b[9] * A2[i];
  matmul(k, A6.data(), T1.data(), T2.data());
  for (size_t i = 0; i < kk; ++i)
    T2[i] += b[7] * A6[i] + b[5] * A4[i] + b[3] * A2[i] + b[1] * I[i];
  matmul(k, As.data(), T2.data(), U.data());
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  for (size_t i = 0; i < kk; ++i) T1[i] = b[12] * A6[i] + b[10] * A4[i] + b[8] * A2[i];
  matmul(k, A6.data(), T1.data(), V.data());
  for (size_t i = 0; i < kk; ++i)
    V[i] += b[6] * A6[i] + b[4] * A4[i] + b[2] * A2[i] + b[0] * I[i];
  std::vector<double> P(kk), Q(kk);
  for (size_t i = 0; i < kk; ++i) {
    P[i] = V[i] + U[i];
    Q[i] = V[i] - U[i];
  }
  if (!lu_solve(k, Q, P)) return false;
  for (int r = 0; r < s; ++r) {
    matmul(k, P.data(), P.data(), T1.data());
    P.swap(T1);
  }
  std::memcpy(E, P.data(), kk * sizeof(double));
  return true;
}


void step_ellipse(int dtype, double gamma, double c0, double c1, double* gs, double* c0s,
                  double* c1s) {
  if (dtype == EXPW_F32) {
    const float ig = static_cast<float>(1.0 / gamma);
    *gs = 1.0 / static_cast<double>(ig);
    *c0s = static_cast<double>(static_cast<float>(c0));
    *c1s = static_cast<double>(static_cast<float>(c1));
  } else {
    *gs = gamma;
    *c0s = c0;
    *c1s = c1;
  }
}
// ------------------------------------------------------------ PML operator

// Fornberg's recursion for finite-difference weights of derivative orders
// 0..m at z0 on arbitrary nodes: c[k * n + i] weighs f(nodes[i]) in the k-th
// derivative. Each node added updates the weights of all previous ones.
void fd_weights(double z0, const double* nodes, int n, int m, double* c) {
  for (int k = 0; k <= m; ++k)
    for (int i = 0; i < n; ++i) c[k * n + i] = 0.0;
  c[0] = 1.0;
  double prod_prev = 1.0;
  double off_new = nodes[0] - z0;
  for (int i = 1; i < n; ++i) {
    const int top = i < m ? i : m;
    double prod = 1.0;
    const double off_last = off_new;
    off_new = nodes[i] - z0;
    for (int j = 0; j < i; ++j) {
      const double gap = nodes[i] - nodes[j];
      prod *= gap;
      if (j == i - 1) {
        // the new node's weights from the previous node's (before they change)
        for (int k = top; k >= 1; --k)
          c[k * n + i] = prod_prev * (k * c[(k - 1) * n + i - 1] - off_last * c[k * n + i - 1]) / prod;
        c[i] = -prod_prev * off_last * c[i - 1] / prod;
      }
      for (int k = top; k >= 1; --k) c[k * n + j] = (off_new * c[k * n + j] - k * c[(k - 1) * n + j]) / gap;
      c[j] = off_new * c[j] / gap;
    }
    prod_prev = prod;
  }
}

void pml_surface_tables(double d2[4][9], double d1[3][8], double dw[4][8]) {
  // appendix on the free surface, u_i = u(x, -i h), y up: d_yy u at
  // y = 0, -h, -2h, -3h (times 1/h^2) and d_y u at y = -h/2, -3h/2, -5h/2
  // (times 1/h)
  static const double D2[4][9] = {
      {-3144919.0 / 352800.0, 16.0, -14.0, 112.0 / 9.0, -35.0 / 4.0, 112.0 / 25.0, -14.0 / 9.0, 16.0 / 49.0, -1.0 / 32.0},
      {271343.0 / 156800.0, -1991.0 / 630.0, 57.0 / 40.0, 13.0 / 60.0, -109.0 / 288.0, 6.0 / 25.0, -11.0 / 120.0, 179.0 / 8820.0, -9.0 / 4480.0},
      {-18519.0 / 78400.0, 58.0 / 35.0, -251.0 / 90.0, 22.0 / 15.0, -1.0 / 16.0, -14.0 / 225.0, 1.0 / 30.0, -2.0 / 245.0, 17.0 / 20160.0},
      {74801.0 / 1411200.0, -37.0 / 140.0, 67.0 / 40.0, -263.0 / 90.0, 53.0 / 32.0, -23.0 / 100.0, 13.0 / 360.0, -1.0 / 245.0, 1.0 / 4480.0}};
  static const double D1[3][8] = {
      {5034629.0 / 3763200.0, -23533.0 / 15360.0, 4259.0 / 15360.0, -1103.0 / 9216.0, 151.0 / 3072.0, -1171.0 / 76800.0, 139.0 / 46080.0, -211.0 / 752640.0},
      {-363509.0 / 3763200.0, 6297.0 / 5120.0, -6147.0 / 5120.0, 211.0 / 3072.0, 3.0 / 1024.0, -153.0 / 25600.0, 29.0 / 15360.0, -57.0 / 250880.0},
      {4631.0 / 250880.0, -305.0 / 3072.0, 1245.0 / 1024.0, -3725.0 / 3072.0, 275.0 / 3072.0, -69.0 / 5120.0, 5.0 / 3072.0, -5.0 / 50176.0}};
  std::memcpy(d2, D2, sizeof(D2));
  std::memcpy(d1, D1, sizeof(D1));
  // d_y w_y at y = -j h, j = 0..3: Fornberg on the surface point (w_y = 0
  // there, so its weight drops out) and the half rows -(i + 1/2) h, i = 0..7,
  // nine nodes for order 8
  double nodes[9], c[2 * 9];
  nodes[0] = 0.0;
  for (int i = 0; i < 8; ++i) nodes[i + 1] = -(i + 0.5);
  for (int j = 0; j < 4; ++j) {
    fd_weights(-static_cast<double>(j), nodes, 9, 1, c);
    for (int i = 0; i < 8; ++i) dw[j][i] = c[9 + i + 1];
  }
}

void bottom_profile(int64_t n, double h, int cells, double beta0, bool half, double* out) {
  // Sec. 2: no layer at the free surface, so beta_y grows towards the bottom
  // row only: beta0 (1 - d/delta)^2 with d the distance to row n - 1
  const double delta = cells * h;
  for (int64_t i = 0; i < n; ++i) {
    const double pos = static_cast<double>(i) + (half ? 0.5 : 0.0);
    double d = (static_cast<double>(n - 1) - pos) * h;
    if (d < 0.0) d = 0.0;
    double s = 0.0;
    if (cells > 0 && beta0 != 0.0 && d < delta) {
      const double r = 1.0 - d / delta;
      s = beta0 * r * r;
    }
    out[i] = s;
  }
}

}  // namespace expw

// ------------------------------------------------------------------ C ABI (host only)

// The one-sided surface rows raise the largest frequency of the PML operator
// about 22 % above the interior symbol bound (dense spectra of small grids);
// B carries this margin so that the Faber ellipse, whose height at Re = 0 is
// B, still encloses the spectrum.
constexpr double kPmlSurfaceMargin = 1.25;

extern "C" {

int32_t expw_version(void) { return 1; }

const char* expw_last_error(void) { return expw::last_error(); }

int32_t expw_damping_profile(int64_t n, double h, int32_t cells, double sigma_max, int32_t half,
                             double* out) {
  if (n < 1 || !(h > 0.0) || cells < 0 || !(sigma_max >= 0.0) || !out)
    return expw::fail(EXPW_EINVAL, "expw_damping_profile: invalid argument");
  expw::damping_profile(n, h, cells, sigma_max, half != 0, out);
  return EXPW_OK;
}

int32_t expw_ellipse(double x_lo, double B, double* gamma, double* c0, double* c1) {
  // Minimum-area ellipse through the corners of [x_lo, 0] x i[-B, B]: centre
  // x_lo/2, semi-axes sqrt(2) |x_lo|/2 (real) and sqrt(2) B (imaginary); the
  // degenerate rectangle x_lo = 0 gives the segment i[-B, B]. psi(w) =
  // gamma (w + c0 + c1/w) maps |w| = 1 onto it.
  if (!(x_lo <= 0.0) || !(B > 0.0) || !gamma || !c0 || !c1 || !std::isfinite(x_lo) ||
      !std::isfinite(B))
    return expw::fail(EXPW_EINVAL, "expw_ellipse: need x_lo <= 0 < B, finite");
  const double r2 = std::sqrt(2.0);
  const double ar = (x_lo < 0.0) ? r2 * 0.5 * std::fabs(x_lo) : 0.0;
  const double bi = (x_lo < 0.0) ? r2 * B : B;
  *gamma = 0.5 * (ar + bi);
  *c1 = (ar - bi) / (ar + bi);
  *c0 = 0.5 * x_lo / *gamma;
  return EXPW_OK;
}

int32_t expw_spectrum_rectangle(const expw_grid* g, double c2_max, double* x_lo, double* B) {
  if (!g || !x_lo || !B || !(c2_max > 0.0) || !std::isfinite(c2_max))
    return expw::fail(EXPW_EINVAL, "expw_spectrum_rectangle: invalid argument");
  double alpha[4];
  int K = 0;
  if (!expw::stagger_weights(g->order, alpha, &K))
    return expw::fail(EXPW_EINVAL, "expw_spectrum_rectangle: order must be 4 or 8");
  if (g->ndim != 2 && g->ndim != 3)
    return expw::fail(EXPW_EINVAL, "expw_spectrum_rectangle: ndim must be 2 or 3");
  double sa = 0.0;
  for (int l = 0; l < K; ++l) sa += std::fabs(alpha[l]);
  *B = std::sqrt(c2_max) * std::sqrt(static_cast<double>(g->ndim)) * (2.0 / g->h) * sa;
  double smax_p = 0.0, smax_v = 0.0;
  for (int a = 0; a < g->ndim; ++a) {
    std::vector<double> si(g->n[a]), sh(g->n[a]);
    expw::damping_profile(g->n[a], g->h, g->abc_cells, g->sigma_max, false, si.data());
    expw::damping_profile(g->n[a], g->h, g->abc_cells, g->sigma_max, true, sh.data());
    double mi = 0.0, mh = 0.0;
    for (int64_t i = 0; i < g->n[a]; ++i) {
      mi = std::fmax(mi, si[i]);
      mh = std::fmax(mh, sh[i]);
    }
    smax_p += mi;  // sigma_p = sum over axes, separable: its max is the sum of maxima
    smax_v = std::fmax(smax_v, mh);
  }
  *x_lo = -std::fmax(smax_p, smax_v);
  return EXPW_OK;
}

int32_t expw_spectrum_rectangle_profiles(const expw_grid* g, double c2_max,
                                         const double* const* sigma_host, double* x_lo,
                                         double* B) {
  if (!sigma_host) return expw_spectrum_rectangle(g, c2_max, x_lo, B);
  if (int32_t rc = expw_spectrum_rectangle(g, c2_max, x_lo, B)) return rc;
  // x_lo = -(largest damping): sigma_p sums the axes' integer-point values (its
  // maximum is the sum of their maxima), v_a takes axis a's half-point values
  double smax_p = 0.0, smax_v = 0.0;
  for (int a = 0; a < g->ndim; ++a) {
    const double* si = sigma_host[2 * a];
    const double* sh = sigma_host[2 * a + 1];
    if (!si || !sh) return expw::fail(EXPW_EINVAL, "expw_spectrum_rectangle_profiles: NULL profile");
    double mi = 0.0, mh = 0.0;
    for (int64_t i = 0; i < g->n[a]; ++i) {
      if (!(si[i] >= 0.0) || !(sh[i] >= 0.0) || !std::isfinite(si[i]) || !std::isfinite(sh[i]))
        return expw::fail(EXPW_EINVAL, "expw_spectrum_rectangle_profiles: profile values must be finite and >= 0");
      mi = std::fmax(mi, si[i]);
      mh = std::fmax(mh, sh[i]);
    }
    smax_p += mi;
    smax_v = std::fmax(smax_v, mh);
  }
  *x_lo = -std::fmax(smax_p, smax_v);
  return EXPW_OK;
}

int32_t expw_faber_coefficients(double gamma, double c0, double c1, double dt, int32_t m,
                                double* a) {
  if (!(gamma > 0.0) || !(dt > 0.0) || m < 0 || !a || !(std::fabs(c1) <= 1.0) ||
      !std::isfinite(c0))
    return expw::fail(EXPW_EINVAL, "expw_faber_coefficients: invalid argument");
  expw::faber_coefficients(gamma, c0, c1, dt, m, a);
  return EXPW_OK;
}

int32_t expw_step_ellipse(int32_t dtype, double gamma, double c0, double c1, double* gs,
                          double* c0s, double* c1s) {
  if ((dtype != EXPW_F32 && dtype != EXPW_F64) || !(gamma > 0.0) || !std::isfinite(gamma) ||
      !std::isfinite(c0) || !(std::fabs(c1) <= 1.0) || !gs || !c0s || !c1s)
    return expw::fail(EXPW_EINVAL, "expw_step_ellipse: invalid argument");
  expw::step_ellipse(dtype, gamma, c0, c1, gs, c0s, c1s);
  return EXPW_OK;
}

int32_t expw_faber_dense_coefficients(double gamma, double c0, double c1, int32_t m, int32_t n_tau,
                                      const double* taus, double* coef) {
  if (!(gamma > 0.0) || !std::isfinite(gamma) || m < 0 || n_tau < 0 || !(std::fabs(c1) <= 1.0) ||
      !std::isfinite(c0) || (n_tau > 0 && (!taus || !coef)))
    return expw::fail(EXPW_EINVAL, "expw_faber_dense_coefficients: invalid argument");
  for (int32_t t = 0; t < n_tau; ++t)
    if (!(taus[t] >= 0.0) || !std::isfinite(taus[t]))
      return expw::fail(EXPW_EINVAL, "expw_faber_dense_coefficients: tau must be finite and >= 0");
  for (int32_t t = 0; t < n_tau; ++t) {
    double* a = coef + static_cast<int64_t>(t) * (m + 1);
    if (taus[t] == 0.0) {  // exp(0) = I: only F_0 = I contributes
      for (int j = 0; j <= m; ++j) a[j] = j == 0 ? 1.0 : 0.0;
    } else {
      expw::faber_coefficients(gamma, c0, c1, taus[t], m, a);
    }
  }
  return EXPW_OK;
}

int32_t expw_ricker_derivatives(double t, double f_peak, double t_delay, int32_t p, double* out) {
  if (!(f_peak > 0.0) || p < 1 || p > 64 || !out)
    return expw::fail(EXPW_EINVAL, "expw_ricker_derivatives: invalid argument");
  expw::ricker_derivatives(t, f_peak, t_delay, p, out);
  return EXPW_OK;
}

int32_t expw_faber_source_scalars(double gamma, double c0, double c1, int32_t m, int32_t p,
                                  const double* G, double* q) {
  if (!(gamma > 0.0) || m < 1 || p < 1 || p > EXPW_MAX_TAYLOR || !G || !q)
    return expw::fail(EXPW_EINVAL, "expw_faber_source_scalars: invalid argument");
  expw::faber_source_scalars(gamma, c0, c1, m, p, G, q);
  return EXPW_OK;
}

int32_t expw_expm(int32_t k, const double* A, double* E) {
  if (k < 1 || k > EXPW_MAX_KRYLOV + 1 || !A || !E)
    return expw::fail(EXPW_EINVAL, "expw_expm: need 1 <= k <= %d", EXPW_MAX_KRYLOV + 1);
  if (!expw::expm(k, A, E)) return expw::fail(EXPW_ENONFINITE, "expw_expm: singular or non-finite");
  return EXPW_OK;
}

int32_t expw_pml_check_grid(const expw_pml_grid* g) {
  if (!g) return expw::fail(EXPW_EINVAL, "grid is NULL");
  if (g->ny < 9) return expw::fail(EXPW_EINVAL, "the free-surface stencils need ny >= 9 (got %lld)", (long long)g->ny);
  if (g->nx < 1) return expw::fail(EXPW_EINVAL, "nx must be >= 1");
  if (g->nx > (int64_t(1) << 30) || g->ny > (int64_t(1) << 30) || g->nx * g->ny > (int64_t(1) << 31))
    return expw::fail(EXPW_EINVAL, "grid too large");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return expw::fail(EXPW_EINVAL, "h must be > 0");
  if (g->dtype != EXPW_F32 && g->dtype != EXPW_F64) return expw::fail(EXPW_EINVAL, "bad dtype");
  if (g->abc_cells < 0) return expw::fail(EXPW_EINVAL, "abc_cells must be >= 0");
  if (!(g->beta0 >= 0.0) || !std::isfinite(g->beta0)) return expw::fail(EXPW_EINVAL, "beta0 must be >= 0");
  return EXPW_OK;
}

int32_t expw_pml_spectrum_rectangle(const expw_pml_grid* g, double c2_max, double* x_lo, double* B) {
  if (int32_t rc = expw_pml_check_grid(g)) return rc;
  if (!(c2_max > 0.0) || !std::isfinite(c2_max) || !x_lo || !B)
    return expw::fail(EXPW_EINVAL, "expw_pml_spectrum_rectangle: invalid argument");
  // largest symbol of the centred second derivative along one axis
  const double sym = (205.0 / 72.0 + 2.0 * (8.0 / 5.0 + 1.0 / 5.0 + 8.0 / 315.0 + 1.0 / 560.0)) / (g->h * g->h);
  *B = kPmlSurfaceMargin * std::sqrt(c2_max) * std::sqrt(2.0 * sym);
  std::vector<double> pr(std::max(g->nx, g->ny));
  double bx = 0.0, by = 0.0;
  for (int hf = 0; hf < 2; ++hf) {
    expw::damping_profile(g->nx, g->h, g->abc_cells, g->beta0, hf == 1, pr.data());
    for (int64_t i = 0; i < g->nx; ++i) bx = std::fmax(bx, pr[i]);
    expw::bottom_profile(g->ny, g->h, g->abc_cells, g->beta0, hf == 1, pr.data());
    for (int64_t i = 0; i < g->ny; ++i) by = std::fmax(by, pr[i]);
  }
  *x_lo = -(bx + by);
  return EXPW_OK;
}

int32_t expw_pml_surface_weights(double* d2, double* d1, double* dw) {
  if (!d2 || !d1 || !dw) return expw::fail(EXPW_EINVAL, "NULL output");
  double a[4][9], b[3][8], c[4][8];
  expw::pml_surface_tables(a, b, c);
  std::memcpy(d2, a, sizeof(a));
  std::memcpy(d1, b, sizeof(b));
  std::memcpy(dw, c, sizeof(c));
  return EXPW_OK;
}

}  // extern "C"

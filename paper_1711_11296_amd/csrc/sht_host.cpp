// Host-side planning for the Clenshaw-Curtis spherical-harmonic transform:
// latitude nodes, quadrature weights and the table of normalised associated
// Legendre functions, all in extended precision, rounded to double once.
//
// Nodes:   Sec. 3.1 eq. cc-points (pole-free grid, theta_j = j pi/(J+1)) and
//          the classical grid with the poles, theta_j = j pi/(J-1).
// Weights: Sec. 3.1 eq. cc-wgt (derivation in App. A) for the pole-free
//          grid; the classical Clenshaw-Curtis rule for the grid with poles.
// P~_n^m:  the three-term recurrence named in Sec. 4.1, normalised as in
//          eq. pnm-ortho, carried as (mantissa, binary exponent) pairs so
//          that the sectoral starting values of high m never underflow.

#include <cmath>
#include <cstdint>
#include <numeric>
#include <thread>
#include <vector>

#include "sht_internal.h"

namespace sht {

namespace {

// sin(pi * a / b) with a/b reduced by its gcd; exactly odd in a.
double sinpi_frac(long a, long b) {
  if (a == 0) return 0.0;
  long g = std::gcd(a < 0 ? -a : a, b);
  long aa = (a < 0 ? -a : a) / g;
  long bb = b / g;
  double s = std::sin(M_PI * (double)aa / (double)bb);
  return a > 0 ? s : -s;
}

long double sinpi_frac_l(long a, long b) {
  // reduce a into [0, 2b) first; sin has period 2 in units of pi
  long m = 2 * b;
  a %= m;
  if (a < 0) a += m;
  if (a == 0) return 0.0L;
  long g = std::gcd(a, b);
  return sinl(3.141592653589793238462643383279502884L * (long double)(a / g) /
              (long double)(b / g));
}

// theta_j = pi p / q
void node_pq(int J, int kind, int j, long* p, long* q) {
  if (kind == SHT_GRID_CC_POLES) {
    *p = j;
    *q = J - 1;
  } else if (kind == SHT_GRID_FEJER1) {  // Sec. 3.3, eq. fejer1-points
    *p = 2 * j + 1;
    *q = 2 * J;
  } else {  // Sec. 3.1, eq. cc-points
    *p = j + 1;
    *q = J + 1;
  }
}

}  // namespace

bool grid_args_ok(int J, int kind) {
  if (kind == SHT_GRID_CC_POLES) return J >= 2;
  if (kind == SHT_GRID_FEJER2 || kind == SHT_GRID_FEJER1 || kind == SHT_GRID_GAUSS) return J >= 1;
  return false;
}

namespace {
// Gauss-Legendre nodes (roots of P_J, descending: north first) and weights
// 2 / (sin^2(theta) P_J'(x)^2), by Newton's method in the colatitude theta
// on the three-term recurrence of P_J in extended precision, from Tricomi's
// estimate theta = pi (j + 3/4) / (J + 1/2).  Iterating on theta rather than
// on x = cos(theta) keeps sin(theta) accurate to its own relative precision
// near the poles, where 1 - x is tiny.  The southern half is the exact
// mirror and the middle node of odd J is 0.
void gauss_nodes_weights(int J, long double* x, long double* w, long double* st) {
  const long double PI = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < (J + 1) / 2; ++j) {
    long double th = PI * ((long double)j + 0.75L) / ((long double)J + 0.5L);
    long double z = cosl(th), s = sinl(th);
    // quadratic convergence: one more step once the step is below 1e-12 th
    // brings theta to rounding level
    bool last = false;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;  // P_0, P_1
      for (int n = 2; n <= J; ++n) {
        const long double p2 = ((2.0L * n - 1.0L) * z * p1 - (n - 1.0L) * p0) / (long double)n;
        p0 = p1;
        p1 = p2;
      }
      if (J == 1) p0 = 1.0L;  // P_{J-1} = P_0
      // P_J'(z) = J (P_{J-1} - z P_J) / sin^2(theta); dP_J/dtheta = -sin(theta) P_J'(z)
      const long double dp = (long double)J * (p0 - z * p1) / (s * s);
      const long double dth = p1 / (s * dp);
      th += dth;
      z = cosl(th);
      s = sinl(th);
      if (last) break;
      last = fabsl(dth) < 1e-12L * th;
    }
    if (2 * j + 1 == J) {
      z = 0.0L;
      s = 1.0L;
    }
    // the weight from P_J' at the final theta
    long double q0 = 1.0L, q1 = z;
    for (int n = 2; n <= J; ++n) {
      const long double q2 = ((2.0L * n - 1.0L) * z * q1 - (n - 1.0L) * q0) / (long double)n;
      q0 = q1;
      q1 = q2;
    }
    if (J == 1) q0 = 1.0L;
    x[j] = z;
    x[J - 1 - j] = -z;
    if (st) st[j] = st[J - 1 - j] = s;
    const long double dq = (long double)J * (q0 - z * q1) / (s * s);
    w[j] = w[J - 1 - j] = 2.0L / (s * s * dq * dq);
  }
}
}  // namespace

void grid_nodes(int J, int kind, double* mu, double* sint) {
  if (kind == SHT_GRID_GAUSS) {
    std::vector<long double> x(J), w(J), st(J);
    gauss_nodes_weights(J, x.data(), w.data(), st.data());
    for (int j = 0; j < J; ++j) {
      mu[j] = (double)x[j];
      sint[j] = (double)st[j];
    }
    return;
  }
  for (int j = 0; j < J; ++j) {
    long p, q;
    node_pq(J, kind, j, &p, &q);
    // mu = cos(pi p/q) = sin(pi (q - 2p) / (2q))
    mu[j] = sinpi_frac(q - 2 * p, 2 * q);
    long r = p < q - p ? p : q - p;
    sint[j] = sinpi_frac(r, q);
  }
}

void grid_weights(int J, int kind, double* w) {
  const long double PI = 3.141592653589793238462643383279502884L;
  if (kind == SHT_GRID_GAUSS) {
    std::vector<long double> x(J), wl(J);
    gauss_nodes_weights(J, x.data(), wl.data(), nullptr);
    for (int j = 0; j < J; ++j) w[j] = (double)wl[j];
    return;
  }
  if (kind == SHT_GRID_FEJER2) {
    // w_j = 4 sin(theta_j)/(J+1) * sum_{p odd <= J} sin(p theta_j)/p
    for (int j = 0; j < J; ++j) {
      long p0, q;
      node_pq(J, kind, j, &p0, &q);
      long double s = 0.0L;
      for (long p = 1; p <= J; p += 2) s += sinpi_frac_l(p * p0, q) / (long double)p;
      w[j] = (double)(4.0L * sinpi_frac_l(p0, q) / (long double)(J + 1) * s);
    }
    return;
  }
  if (kind == SHT_GRID_FEJER1) {
    // Fejer's first rule (Sec. 3.3, eq. fejer1-wgt, with the factor 2 before
    // the sum that makes the rule interpolatory):
    // w_j = (2/J) [1 - 2 sum_{p=1}^{J/2} cos(2 p theta_j) / (4 p^2 - 1)],
    // 2 p theta_j = pi p (2j+1) / J
    for (long j = 0; j < J; ++j) {
      long double s = 0.0L;
      for (long p = 1; p <= J / 2; ++p) {
        const long r = (p * (2 * j + 1)) % (2L * J);
        s += cosl(PI * (long double)r / (long double)J) / (4.0L * (long double)p * (long double)p - 1.0L);
      }
      w[j] = (double)(2.0L / (long double)J * (1.0L - 2.0L * s));
    }
    return;
  }
  // classical Clenshaw-Curtis on n+1 = J points:
  // w_k = (c_k/n) [1 - sum_{l=1}^{n/2} b_l cos(2 l theta_k) / (4 l^2 - 1)]
  const long n = J - 1;
  for (long k = 0; k < J; ++k) {
    long double c = (k == 0 || k == n) ? 1.0L : 2.0L;
    long double s = 0.0L;
    for (long l = 1; l <= n / 2; ++l) {
      long double b = (2 * l == n) ? 1.0L : 2.0L;
      long r = (l * k) % n;
      s += b * cosl(2.0L * PI * (long double)r / (long double)n) /
           (4.0L * (long double)l * (long double)l - 1.0L);
    }
    w[k] = (double)(c / (long double)n * (1.0L - s));
  }
}

namespace {

// Extended-range number: value = x * 2^(SCALE * e).
constexpr int SCALE = 4096;

struct XNum {
  long double x;
  int e;
};

inline void xnorm(XNum& v) {
  const long double hi = ldexpl(1.0L, SCALE);
  const long double lo = ldexpl(1.0L, -SCALE);
  if (v.x == 0.0L) {
    v.e = 0;
    return;
  }
  while (fabsl(v.x) >= hi) {
    v.x *= lo;
    v.e += 1;
  }
  while (fabsl(v.x) < lo) {
    v.x *= hi;
    v.e -= 1;
  }
}

inline double xval(const XNum& v) {
  if (v.e == 0) return (double)v.x;
  return (double)ldexpl(v.x, SCALE * v.e);
}

}  // namespace

// P~_n^m(mu_r) for n = m..N and the `nr` rows given; out[(n-m)*ld + r].
void alf_column(int N, int m, int nr, const double* mu, const double* sint,
                double* out, long ld) {
  std::vector<XNum> p0(nr), p1(nr);
  // sectoral start: P~_m^m = prod_{k=1}^m sqrt((2k+1)/(2k)) sin^m / sqrt(2)
  for (int r = 0; r < nr; ++r) {
    XNum v{1.0L / sqrtl(2.0L), 0};
    const long double s = sint[r];
    for (int k = 1; k <= m; ++k) {
      v.x *= sqrtl((2.0L * k + 1.0L) / (2.0L * k)) * s;
      xnorm(v);
    }
    p0[r] = v;
    out[r] = xval(v);
  }
  if (N == m) return;
  const long double a1 = sqrtl(2.0L * m + 3.0L);
  for (int r = 0; r < nr; ++r) {
    XNum v{a1 * (long double)mu[r] * p0[r].x, p0[r].e};
    xnorm(v);
    p1[r] = v;
    out[ld + r] = xval(v);
  }
  long double aprev = a1;  // a_{m+1}^m = sqrt(2m+3)
  for (int n = m + 2; n <= N; ++n) {
    const long double nn = (long double)n * n, mm = (long double)m * m;
    const long double a = sqrtl((4.0L * nn - 1.0L) / (nn - mm));
    const long double inv = 1.0L / aprev;
    double* o = out + (long)(n - m) * ld;
    for (int r = 0; r < nr; ++r) {
      // p_n = a (mu p_{n-1} - p_{n-2} / a_{n-1}), both terms brought to a
      // common exponent (a zero mantissa carries no exponent)
      const XNum& q1 = p1[r];
      const XNum& q0 = p0[r];
      long double x1 = q1.x, x0 = q0.x;
      int ew = q1.e;
      if (q0.e != q1.e) {
        if (q1.x == 0.0L) ew = q0.e;
        else if (q0.x != 0.0L && q0.e > q1.e) ew = q0.e;
        x1 = (q1.x == 0.0L) ? 0.0L : ldexpl(q1.x, SCALE * (q1.e - ew));
        x0 = (q0.x == 0.0L) ? 0.0L : ldexpl(q0.x, SCALE * (q0.e - ew));
      }
      XNum v{a * ((long double)mu[r] * x1 - x0 * inv), ew};
      xnorm(v);
      p0[r] = q1;
      p1[r] = v;
      o[r] = xval(v);
    }
    aprev = a;
  }
}

void alf_table(int N, int nr, const double* mu, const double* sint,
               double* out, int nthreads) {
  // out: spec order, row (m, n) of length nr at offset idx(m,n)*nr
  if (nthreads < 1) nthreads = 1;
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t) {
    pool.emplace_back([=]() {
      // interleave m and N-m so that every thread gets a similar share
      for (int k = t; k <= N; k += nthreads) {
        int m = (k % 2 == 0) ? k / 2 : N - k / 2;
        long off = (long)m * (2 * N + 3 - m) / 2 * nr;
        alf_column(N, m, nr, mu, sint, out + off, nr);
      }
    });
  }
  for (auto& th : pool) th.join();
}

bool factor_radices(int I, int* rad, int* nrad) {
  int n = I, k = 0;
  while (n % 8 == 0) {
    rad[k++] = 8;
    n /= 8;
  }
  while (n % 4 == 0) {
    rad[k++] = 4;
    n /= 4;
  }
  while (n % 2 == 0) {
    rad[k++] = 2;
    n /= 2;
  }
  while (n % 3 == 0) {
    rad[k++] = 3;
    n /= 3;
  }
  while (n % 5 == 0) {
    rad[k++] = 5;
    n /= 5;
  }
  if (n != 1 || k > SHT_MAX_RADICES) return false;
  *nrad = k;
  return true;
}

}  // namespace sht

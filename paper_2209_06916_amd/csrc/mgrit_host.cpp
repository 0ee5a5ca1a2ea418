// Host side of the MGRIT library: problem setup (coefficients, level
// hierarchy, factorisations of the periodic banded operators), the MGRIT
// schedule, and the C ABI declared in include/mgrit.h.
#include "mgrit.h"
#include "mgrit_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

using namespace mgrit;

namespace {

using ld = long double;
using cld = std::complex<long double>;

// ---------------------------------------------------------------------------
// Dense helpers (tiny systems only)
// ---------------------------------------------------------------------------

// Solve A x = b (n x n, row-major) by Gaussian elimination with partial pivoting.
bool dense_solve(std::vector<ld> A, std::vector<ld> &b, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const ld f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    ld s = b[c];
    for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
    b[c] = s / A[c * n + c];
  }
  return true;
}

std::vector<ld> matmul(const std::vector<ld> &A, const std::vector<ld> &B, int k) {
  std::vector<ld> C(k * k, 0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      ld s = 0;
      for (int t = 0; t < k; ++t) s += A[i * k + t] * B[t * k + j];
      C[i * k + j] = s;
    }
  return C;
}

std::vector<ld> identity(int k) {
  std::vector<ld> I(k * k, 0);
  for (int i = 0; i < k; ++i) I[i * k + i] = 1;
  return I;
}

bool invert(const std::vector<ld> &A, int k, std::vector<ld> &inv) {
  inv.assign(k * k, 0);
  for (int c = 0; c < k; ++c) {
    std::vector<ld> e(k, 0);
    e[c] = 1;
    if (!dense_solve(A, e, k)) return false;
    for (int r = 0; r < k; ++r) inv[r * k + c] = e[r];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Upwind stencil L_p (Sec. 4.1): differentiate the degree-p interpolant at
// x_i.  Weights from the moment conditions sum_j w_j j^k = [k == 1], k = 0..p.
// ---------------------------------------------------------------------------

void upwind_stencil(int p, int &l, int &r, std::vector<double> &w) {
  if (p % 2) {
    l = (p + 1) / 2;
    r = l - 1;
  } else {
    l = p / 2 + 1;
    r = l - 2;
  }
  const int n = p + 1;
  std::vector<ld> V(n * n), rhs(n, 0);
  for (int k = 0; k < n; ++k)
    for (int c = 0; c < n; ++c) {
      const int j = c - l;
      ld v = 1;
      for (int e = 0; e < k; ++e) v *= j;
      V[k * n + c] = v;
    }
  rhs[1] = 1;
  dense_solve(V, rhs, n);
  w.assign(n, 0.0);
  for (int c = 0; c < n; ++c) w[c] = (double)rhs[c];
}

// ---------------------------------------------------------------------------
// Runge-Kutta tableaux (Sec. 4.2).  ERK1-4: forward Euler, Heun, the
// three-stage SSP method, classical RK4 (R = Taylor polynomial of exp).
// ERK5: six stages, sub-diagonal coupling (3/32, 1/5, 1/4, 1/3, 1/2), b = e_6,
// so R = T_5 + z^6/1280, matching Table 1's e_RK.  SDIRK1-3: backward Euler;
// gamma = 1 - 1/sqrt(2); the L-stable three-stage method with
// 6 g^3 - 18 g^2 + 9 g - 1 = 0.
// ---------------------------------------------------------------------------

struct Tableau {
  int s = 0;
  std::vector<ld> A, b;
  ld gamma = 0;  // SDIRK diagonal
};

ld sdirk3_gamma() {
  ld g = 0.4358665215L;  // Newton on the cubic from a bracketing start
  for (int i = 0; i < 60; ++i) {
    const ld f = ((6 * g - 18) * g + 9) * g - 1;
    const ld df = (18 * g - 36) * g + 9;
    g -= f / df;
  }
  return g;
}

bool make_tableau(int kind, int q, Tableau &T) {
  auto set = [&](int s) {
    T.s = s;
    T.A.assign(s * s, 0);
    T.b.assign(s, 0);
  };
  if (kind == MGRIT_ERK) {
    switch (q) {
      case 1: set(1); T.b[0] = 1; return true;
      case 2: set(2); T.A[1 * 2 + 0] = 1; T.b[0] = 0.5L; T.b[1] = 0.5L; return true;
      case 3:
        set(3);
        T.A[1 * 3 + 0] = 1;
        T.A[2 * 3 + 0] = 0.25L;
        T.A[2 * 3 + 1] = 0.25L;
        T.b[0] = 1.0L / 6;
        T.b[1] = 1.0L / 6;
        T.b[2] = 2.0L / 3;
        return true;
      case 4:
        set(4);
        T.A[1 * 4 + 0] = 0.5L;
        T.A[2 * 4 + 1] = 0.5L;
        T.A[3 * 4 + 2] = 1;
        T.b[0] = 1.0L / 6;
        T.b[1] = 1.0L / 3;
        T.b[2] = 1.0L / 3;
        T.b[3] = 1.0L / 6;
        return true;
      case 5: {
        set(6);
        const ld sub[5] = {3.0L / 32, 1.0L / 5, 1.0L / 4, 1.0L / 3, 1.0L / 2};
        for (int i = 0; i < 5; ++i) T.A[(i + 1) * 6 + i] = sub[i];
        T.b[5] = 1;
        return true;
      }
      default: return false;
    }
  }
  if (kind == MGRIT_SDIRK) {
    switch (q) {
      case 1: set(1); T.A[0] = 1; T.b[0] = 1; T.gamma = 1; return true;
      case 2: {
        set(2);
        const ld g = 1 - 1 / std::sqrt((ld)2);
        T.A[0] = g;
        T.A[1 * 2 + 0] = 1 - g;
        T.A[1 * 2 + 1] = g;
        T.b[0] = 1 - g;
        T.b[1] = g;
        T.gamma = g;
        return true;
      }
      case 3: {
        set(3);
        const ld g = sdirk3_gamma();
        const ld b1 = -(6 * g * g - 16 * g + 1) / 4, b2 = (6 * g * g - 20 * g + 5) / 4;
        T.A[0] = g;
        T.A[1 * 3 + 0] = (1 - g) / 2;
        T.A[1 * 3 + 1] = g;
        T.A[2 * 3 + 0] = b1;
        T.A[2 * 3 + 1] = b2;
        T.A[2 * 3 + 2] = g;
        T.b[0] = b1;
        T.b[1] = b2;
        T.b[2] = g;
        T.gamma = g;
        return true;
      }
      default: return false;
    }
  }
  return false;
}

// A caller's Butcher tableau (rk_stages > 0): explicit = strictly lower
// triangular A; singly diagonally implicit = lower triangular A with one
// diagonal value gamma > 0 (every stage then solves with the same matrix,
// which the polynomial-in-W form of the step needs).
bool custom_tableau(const mgrit_problem &P, Tableau &T, std::string &err) {
  const int s = P.rk_stages;
  if (s < 1 || s > MAXCOEF - 1 || !P.rk_A || !P.rk_b) {
    err = "custom tableau: rk_stages must be in 1..7 with rk_A and rk_b given";
    return false;
  }
  T.s = s;
  T.A.assign(s * s, 0);
  T.b.assign(s, 0);
  for (int i = 0; i < s * s; ++i) T.A[i] = P.rk_A[i];
  for (int i = 0; i < s; ++i) T.b[i] = P.rk_b[i];
  for (int i = 0; i < s * s; ++i)
    if (!std::isfinite((double)T.A[i])) err = "custom tableau: non-finite entry";
  for (int i = 0; i < s; ++i)
    if (!std::isfinite((double)T.b[i])) err = "custom tableau: non-finite weight";
  if (!err.empty()) return false;
  for (int i = 0; i < s; ++i)
    for (int j = i + 1; j < s; ++j)
      if (T.A[i * s + j] != 0) {
        err = "custom tableau: rk_A must be lower triangular";
        return false;
      }
  if (P.rk_kind == MGRIT_ERK) {
    for (int i = 0; i < s; ++i)
      if (T.A[i * s + i] != 0) {
        err = "custom explicit tableau: rk_A must be strictly lower triangular";
        return false;
      }
  } else {
    const ld g = T.A[0];
    for (int i = 0; i < s; ++i)
      if (T.A[i * s + i] != g) {
        err = "custom implicit tableau: every diagonal entry of rk_A must equal the same gamma";
        return false;
      }
    if (!(g > 0)) {
      err = "custom implicit tableau: gamma must be positive";
      return false;
    }
    T.gamma = g;
  }
  return true;
}

// Taylor coefficients beta_j of R(z) = 1 + z b^T (I - zA)^{-1} 1:
// beta_0 = 1, beta_j = b^T A^{j-1} 1 (eq. RK_stab_def).
std::vector<ld> rk_series(const Tableau &T, int jmax) {
  std::vector<ld> beta(jmax + 1, 0);
  beta[0] = 1;
  std::vector<ld> v(T.s, 1);  // A^{j-1} 1
  for (int j = 1; j <= jmax; ++j) {
    ld s = 0;
    for (int i = 0; i < T.s; ++i) s += T.b[i] * v[i];
    beta[j] = s;
    std::vector<ld> nv(T.s, 0);
    for (int i = 0; i < T.s; ++i)
      for (int k = 0; k < T.s; ++k) nv[i] += T.A[i * T.s + k] * v[k];
    v = nv;
  }
  return beta;
}

// R(z) for complex z (lower-triangular A: forward substitution).
std::complex<double> rk_R(const Tableau &T, std::complex<double> z) {
  std::vector<std::complex<double>> y(T.s);
  for (int i = 0; i < T.s; ++i) {
    std::complex<double> s = 1.0;
    for (int k = 0; k < i; ++k) s += z * (double)T.A[i * T.s + k] * y[k];
    y[i] = s / (1.0 - z * (double)T.A[i * T.s + i]);
  }
  std::complex<double> acc = 0.0;
  for (int i = 0; i < T.s; ++i) acc += (double)T.b[i] * y[i];
  return 1.0 + z * acc;
}

ld factorial(int n) {
  ld f = 1;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// ---------------------------------------------------------------------------
// Semi-Lagrangian interpolation (Sec. 3) and f_{p+1} (eq. fpoly_def), odd p:
// nodes j = -(p+1)/2 .. (p-1)/2 around the east neighbour of the departure
// point x_i - shift*h = x_{i-K} - eps*h.
// ---------------------------------------------------------------------------

void sl_weights(int p, ld eps, int &l, int &r, std::vector<double> &w) {
  l = (p + 1) / 2;
  r = (p - 1) / 2;
  w.assign(l + r + 1, 0.0);
  const ld x = -eps;
  for (int j = -l; j <= r; ++j) {
    ld v = 1;
    for (int k = -l; k <= r; ++k)
      if (k != j) v *= (x - k) / (ld)(j - k);
    w[j + l] = (double)v;
  }
}

ld f_poly(int p, ld z) {
  const int l = (p + 1) / 2, r = (p - 1) / 2;
  ld v = 1;
  for (int j = -l; j <= r; ++j) v *= (j + z);
  return v / factorial(p + 1);
}

// Symmetric second-order D^(k) for even k: centred k-th difference.
std::map<int, ld> dmat(int k) {
  std::map<int, ld> d;
  ld binom = 1;
  for (int n = 0; n <= k; ++n) {
    d[k / 2 - n] = (n % 2 ? -binom : binom);
    binom = binom * (k - n) / (n + 1);
  }
  return d;
}

// ---------------------------------------------------------------------------
// Factorisation of a periodic banded (circulant) operator
//   (T v)_i = sum_j t_j v_{i+j},  symbol T(w) = sum_j t_j w^j,
// as T = C * F(S^-1) * B(S): F(x) = prod(1 - rho x) over the roots |rho| < 1
// of w^{l} T(w), B(w) = prod(1 - w/sigma) over the roots |sigma| > 1.
// Requires winding number zero (exactly l roots inside the unit circle).
// ---------------------------------------------------------------------------

std::vector<cld> poly_roots(const std::vector<ld> &c) {
  const int n = (int)c.size() - 1;
  std::vector<cld> mon(n + 1);
  for (int i = 0; i <= n; ++i) mon[i] = c[i] / c[n];
  auto eval = [&](cld z, cld &p, cld &dp) {
    p = mon[n];
    dp = 0;
    for (int i = n - 1; i >= 0; --i) {
      dp = dp * z + p;
      p = p * z + mon[i];
    }
  };
  // |p(z)| at or below this bound is rounding noise of the Horner evaluation
  auto noise = [&](cld z) {
    const ld az = std::abs(z);
    ld s = std::fabs(std::abs(mon[n])), t = 1;
    for (int i = n - 1; i >= 0; --i) s = s * az + std::abs(mon[i]), t = t * az + 1;
    return 8 * (ld)std::numeric_limits<ld>::epsilon() * (s + t) * (2 * n + 1);
  };
  const ld rad = std::pow(std::abs(mon[0]) + 1e-300L, 1.0L / n);
  std::vector<cld> z(n);
  std::vector<char> done(n, 0);
  for (int k = 0; k < n; ++k) z[k] = std::polar(rad * (1 + 0.1L * k), (ld)(2 * M_PI * k / n + 0.4));
  for (int it = 0; it < 500; ++it) {
    int live = 0;
    for (int k = 0; k < n; ++k) {
      if (done[k]) continue;
      cld p, dp;
      eval(z[k], p, dp);
      if (std::abs(p) <= noise(z[k])) {
        done[k] = 1;
        continue;
      }
      ++live;
      const cld ratio = p / dp;
      cld sum = 0;
      for (int j = 0; j < n; ++j)
        if (j != k) sum += 1.0L / (z[k] - z[j]);
      const cld step = ratio / (1.0L - ratio * sum);
      z[k] -= step;
    }
    if (live == 0) break;
  }
  for (int k = 0; k < n; ++k)  // Newton polish
    for (int it = 0; it < 3; ++it) {
      cld p, dp;
      eval(z[k], p, dp);
      if (dp != cld(0)) z[k] -= p / dp;
    }
  return z;
}

struct Factor {
  int kf = 0, kb = 0;
  ld a[KMAX] = {0, 0, 0};  // forward: y_i = x_i + sum a_m y_{i-m}
  ld b[KMAX] = {0, 0, 0};  // backward: y_i = x_i + sum b_m y_{i+m}
  ld C = 1;
};

bool factorize(const std::map<int, ld> &taps_in, Factor &F, std::string &err) {
  std::map<int, ld> taps;
  ld tmax = 0;
  for (auto &kv : taps_in) tmax = std::max(tmax, std::fabs(kv.second));
  for (auto &kv : taps_in)
    if (std::fabs(kv.second) > 1e-18L * tmax) taps[kv.first] = kv.second;
  if (taps.empty()) {
    err = "zero operator";
    return false;
  }
  const int jmin = taps.begin()->first, jmax = taps.rbegin()->first;
  if (jmin > 0 || jmax < 0) {
    err = "operator is not diagonally centred";
    return false;
  }
  if (jmin == 0 && jmax == 0) {
    F.C = taps[0];
    return true;
  }
  const int n = jmax - jmin;
  std::vector<ld> c(n + 1, 0);
  for (auto &kv : taps) c[kv.first - jmin] = kv.second;
  std::vector<cld> rts = poly_roots(c);
  std::vector<cld> in, out;
  for (auto &z : rts) {
    const ld a = std::abs(z);
    if (std::fabs(a - 1) < 1e-12L) {
      err = "operator is singular or nearly so (root on the unit circle)";
      return false;
    }
    (a < 1 ? in : out).push_back(z);
  }
  if ((int)in.size() != -jmin) {
    err = "operator has nonzero winding number";
    return false;
  }
  if ((int)in.size() > KMAX || (int)out.size() > KMAX) {
    err = "band too wide";
    return false;
  }
  // F(x) = prod (1 - rho x)
  std::vector<cld> pf(1, 1), pb(1, 1);
  for (auto &rho : in) {
    std::vector<cld> nx(pf.size() + 1, 0);
    for (size_t i = 0; i < pf.size(); ++i) {
      nx[i] += pf[i];
      nx[i + 1] -= rho * pf[i];
    }
    pf = nx;
  }
  for (auto &sg : out) {
    std::vector<cld> nx(pb.size() + 1, 0);
    for (size_t i = 0; i < pb.size(); ++i) {
      nx[i] += pb[i];
      nx[i + 1] -= pb[i] / sg;
    }
    pb = nx;
  }
  cld C = taps[jmax];
  for (auto &sg : out) C *= -sg;
  F.kf = (int)in.size();
  F.kb = (int)out.size();
  for (int m = 1; m <= F.kf; ++m) F.a[m - 1] = -pf[m].real();
  for (int m = 1; m <= F.kb; ++m) F.b[m - 1] = -pb[m].real();
  F.C = C.real();
  // verify: C * F(w^-1) * B(w) reproduces the taps
  std::map<int, ld> back;
  for (int i = 0; i <= F.kf; ++i)
    for (int k = 0; k <= F.kb; ++k) {
      const ld fi = i == 0 ? 1 : -F.a[i - 1];
      const ld bk = k == 0 ? 1 : -F.b[k - 1];
      back[k - i] += F.C * fi * bk;
    }
  ld worst = 0;
  for (int j = jmin; j <= jmax; ++j) {
    const ld want = taps.count(j) ? taps[j] : 0;
    worst = std::max(worst, std::fabs(back[j] - want));
  }
  if (worst > 1e-13L * tmax) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "factorisation check failed (error %.3Le)", worst);
    err = buf;
    return false;
  }
  return true;
}

// Scan tables of one recurrence for a chunk layout (see mgrit_internal.h).
void recurrence_tables(int k, const ld *a, const Layout &lay, std::vector<double> &out) {
  std::vector<ld> M(k * k, 0);
  for (int m = 0; m < k; ++m) M[m] = a[m];
  for (int i = 1; i < k; ++i) M[i * k + (i - 1)] = 1;
  auto mpow = [&](const std::vector<ld> &B0, long e) {
    std::vector<ld> R = identity(k), B = B0;
    while (e > 0) {
      if (e & 1) R = matmul(R, B, k);
      B = matmul(B, B, k);
      e >>= 1;
    }
    return R;
  };
  const std::vector<ld> H = mpow(M, lay.L);
  std::vector<ld> P = identity(k);
  out.clear();
  for (int t = 0; t <= WAVE; ++t) {
    for (ld v : P) out.push_back((double)v);
    P = matmul(H, P, k);
  }
  const std::vector<ld> Hlast = mpow(M, lay.Llast);
  std::vector<ld> Iw = identity(k);
  const std::vector<ld> HH = matmul(Hlast, mpow(H, lay.A - 1), k);
  for (int i = 0; i < k * k; ++i) Iw[i] -= HH[i];
  std::vector<ld> Wwrap;
  invert(Iw, k, Wwrap);
  for (ld v : Hlast) out.push_back((double)v);
  for (ld v : Wwrap) out.push_back((double)v);
  for (ld v : mpow(M, lay.L / 2)) out.push_back((double)v);
  const std::vector<ld> H64 = mpow(H, WAVE);
  P = identity(k);
  for (int w = 0; w < MAXWAVES; ++w) {
    for (ld v : P) out.push_back((double)v);
    P = matmul(H64, P, k);
  }
}

// Truncated-carry plan of one recurrence (order k, coefficients a) on n
// points in chunks of L (the windowed step kernel).  H = M^L: the state
// entering a chunk is sum_{d < D} H^d Z_{t-1-d} up to H^D E, so D is the
// first power with ||H^D||_inf <= 2^-60 (the error relative to max |y|, well
// below float64 rounding).  Tables: H^1..H^{D-1}, then M^{L/2} (the kernel
// runs the two halves of a chunk as separate chains).  Fails when the carry
// would reach round the whole periodic mesh or past WIN_DMAX chunks.
bool window_tables(int k, const ld *a, int L, int n, int &D, std::vector<double> &out) {
  const ld eps = std::ldexp((ld)1, -60);
  std::vector<ld> M(k * k, 0);
  for (int m = 0; m < k; ++m) M[m] = a[m];
  for (int i = 1; i < k; ++i) M[i * k + (i - 1)] = 1;
  auto norm_inf = [&](const std::vector<ld> &A) {
    ld best = 0;
    for (int r = 0; r < k; ++r) {
      ld s = 0;
      for (int c = 0; c < k; ++c) s += std::fabs(A[r * k + c]);
      best = std::max(best, s);
    }
    return best;
  };
  std::vector<ld> H = identity(k);
  for (int i = 0; i < L; ++i) H = matmul(H, M, k);
  out.clear();
  std::vector<ld> P = H;
  D = 1;
  while (norm_inf(P) > eps) {
    for (ld v : P) out.push_back((double)v);
    P = matmul(P, H, k);
    if (++D > WIN_DMAX || (int64_t)(D + 1) * L > n) return false;
  }
  std::vector<ld> G = identity(k);
  for (int i = 0; i < L / 2; ++i) G = matmul(G, M, k);
  for (ld v : G) out.push_back((double)v);
  return true;
}

// Work distribution: L points per thread (a kernel template parameter).
Layout choose_layout(int nx, int Lpref) {
  static const int Ls[4] = {16, 8, 4, 2};
  Layout best{};
  bool found = false;
  int bestdist = 1 << 30;
  for (int L : Ls) {
    if (nx % (WAVE * L) == 0 && nx / L <= 1024) {
      const int dist = std::abs(L - Lpref);
      if (dist < bestdist) {
        bestdist = dist;
        best = Layout{nx, L, nx / L, nx / L, L, 0, 0};
        found = true;
      }
    }
  }
  if (found) return best;
  int L = 16;
  for (int cand : Ls)
    if ((nx + cand - 1) / cand <= 1024 && std::abs(cand - Lpref) <= std::abs(L - Lpref)) L = cand;
  const int A = (nx + L - 1) / L;
  const int T = ((A + WAVE - 1) / WAVE) * WAVE;
  return Layout{nx, L, A, T, nx - (A - 1) * L, 1, 0};
}

constexpr size_t LDS_LIMIT = 160 * 1024;

// Tile geometry of the level-0 explicit relaxation: the halo is what m steps
// of (Horner depth) stencil applications consume; pick the points per lane
// that minimise redundant lane-work (ties: fewer points, more wavefronts).
bool choose_tiles(int nx, int m, int depth, int sl, int sr, int Pforce, TileGeom &tg, int comp = 0) {
  static const int Ps[2] = {8, 16};
  const int HL = m * depth * sl, HR = m * depth * sr;
  long best = -1;
  for (int P : Ps) {
    if (Pforce && P != Pforce) continue;
    const int avail = WAVE * P - HL - HR;
    if (avail < 32) continue;
    const int ntiles = (nx + avail - 1) / avail;
    const long work = (long)ntiles * WAVE * P;
    if (best < 0 || work < best) {
      best = work;
      tg = TileGeom{P, HL, HR, (nx + ntiles - 1) / ntiles, ntiles, sl, sr, comp};
    }
  }
  return best >= 0;
}

// Sequential stepping in blocks of T steps through the tile kernel (one
// launch per block, the halo covering T steps).  Pick (P, T) minimising a
// model of nt/T dependent launches: a fixed cost per launch (dispatch and
// drain, about 2.5 us) plus one wavefront's instruction stream (about 5
// cycles per instruction at 2.4 GHz), the tiles running side by side.
bool choose_seq_tiles(int nx, int64_t nt, int depth, int sl, int sr, int Pforce, int Tforce, TileGeom &tg, int &T) {
  static const int Ps[3] = {4, 8, 16};
  static const int Ts[5] = {2, 4, 8, 16, 32};
  double best = -1;
  for (int P : Ps) {
    if (Pforce && P != Pforce) continue;
    for (int Tc : Ts) {
      if (Tforce && Tc != Tforce) continue;
      const int HL = Tc * depth * sl, HR = Tc * depth * sr;
      const int avail = WAVE * P - HL - HR;
      if (avail < 32) continue;
      const int ntiles = (nx + avail - 1) / avail;
      const double instr = (double)Tc * depth * (P * (sl + sr + 2) + 2 * (sl + sr));
      const double rounds = std::ceil(ntiles / 1024.0);  // 256 CUs x 4 SIMDs, one wavefront each
      const double launch_us = 2.5 + rounds * instr * 5.0 / 2400.0;
      const double cost = std::ceil((double)nt / Tc) * launch_us;
      if (best < 0 || cost < best) {
        best = cost;
        tg = TileGeom{P, HL, HR, (nx + ntiles - 1) / ntiles, ntiles, sl, sr};
        T = Tc;
      }
    }
  }
  return best >= 0;
}

// Level sizes (Sec. 2.2): nt_0 = nt, nt_{l+1} = nt_l / m_l while the level
// has more than min_coarse_nt steps and m_l divides it; a zero m[l] repeats
// the previous factor.
bool level_hierarchy(const mgrit_problem &P, const mgrit_options &O, std::vector<int64_t> &nts, std::vector<int> &ms,
                     std::string &err) {
  nts.assign(1, P.nt);
  ms.clear();
  int mprev = 0;
  for (int l = 0; l < O.max_levels - 1; ++l) {
    const int m = O.m[l] > 0 ? O.m[l] : mprev;
    if (m < 2) {
      if (l == 0) {
        err = "m[0] must be >= 2";
        return false;
      }
      break;
    }
    mprev = m;
    const int64_t cur = nts.back();
    if (l > 0 && cur <= O.min_coarse_nt) break;
    if (cur % m != 0) {
      if (l == 0) {
        err = "nt must be divisible by m[0]";
        return false;
      }
      break;
    }
    ms.push_back(m);
    nts.push_back(cur / m);
  }
  return true;
}

int env_int(const char *name, int def) {
  const char *v = std::getenv(name);
  return (v && *v) ? std::atoi(v) : def;
}

struct Level {
  bool tiles = false;  // level-0 explicit relaxation through tile_kernel
  TileGeom tg{};
  int t_depth = 0, t_sl = 0, t_sr = 0, t_comp = 0;  // the tiles' operator: Horner depth, extents, written out
  bool seq_tiles = false;  // sequential stepping through tile_kernel, seq_T steps per launch
  TileGeom seq_tg{};
  int seq_T = 0;
  int64_t nt = 0;
  int m = 0;  // to the next level, 0 on the coarsest
  StepOp op{};
  Layout lay{};
  double shift = 0, eps = 0, phi_p = 0, phi_q = 0;
  int64_t K = 0;
  double *tabs = nullptr;
  LevelDesc *desc = nullptr;  // device copy of (op, lay)
  double *c[2] = {nullptr, nullptr};
  double *r = nullptr;
  // float32 copies for the inner solves of mixed precision
  float *tabs32 = nullptr;
  LevelDesc *desc32 = nullptr;  // (op, lay) with the tables' float32 copy
  float *c32[2] = {nullptr, nullptr};
  float *r32 = nullptr;
};

}  // namespace

struct mgrit_handle {
  mgrit_problem prob{};
  mgrit_options opt{};
  hipStream_t stream = nullptr;
  std::vector<Level> lv;
  double *normpart = nullptr;
  int64_t normpart_len = 0;
  double *normsum = nullptr;
  double *normsum_host = nullptr;
  SolveCtl *ctl = nullptr;       // device iteration state of mgrit_solve
  SolveCtl *ctl_host = nullptr;  // pinned coherent copy, read once per iteration
  SolveCtl *ctl_host_dev = nullptr;  // the same memory as the device addresses it
  // mixed precision: the outer refinement loop's state, on the device, and
  // its pinned copy
  SolveCtl *octl = nullptr;
  SolveCtl *octl_host = nullptr, *octl_host_dev = nullptr;
  hipEvent_t ctl_ev = nullptr;
  const int *guard = nullptr;    // stop flag handed to the passes being queued
  // persistent coarse V-cycle (one cooperative launch per iteration)
  bool cv_ok = false;
  size_t cv_lds = 0;
  int64_t cv_grid = 0;
  GridSync *gsync = nullptr;
  // mixed precision: the inner right-hand side (the outer residual, which
  // the residual kernel writes rounded) and solution (float32) and, when the
  // caller keeps no u_out, the outer iterate
  float *g32 = nullptr, *e32 = nullptr;
  double *u64 = nullptr;
  char *arena = nullptr;       // every device buffer of the handle
  size_t arena_bytes = 0;
  bool owns_arena = false;     // false: the caller's workspace (mgrit_setup_ws)
  char *host_arena = nullptr;  // pinned words: normsum_host, ctl_host
  // allocation-free mode (mgrit_solve_noalloc): no pinned words and no
  // events; the iteration state is copied to this host word after each
  // stopping test and the host waits for it
  bool noalloc = false;
  SolveCtl ctl_local{};
  double norm_local = 0;
  std::string err;
  // the solve in progress (mgrit_solve_start .. mgrit_solve_finish)
  struct {
    bool active = false, finished = false;
    double *u_out = nullptr, *u_final = nullptr;
    int cur = 0;
    double prev = NAN;
    SolveCtl hc{};  // float64: the iteration state; mixed: the outer state
    std::vector<double> hist;
    mgrit_status status = MGRIT_OK;
    std::chrono::steady_clock::time_point t0;
    // mixed precision
    bool mixed = false;
    double *U = nullptr;  // the outer iterate
    int rk = 1;           // time points per residual workgroup
    int icur = 0;         // the inner C-point buffer
    int outer = 0, inner_total = 0;
  } ss;
  // profiler
  uint32_t prof_mask = 0;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  mgrit_profile prof{};
};

namespace {

mgrit_status fail(mgrit_handle *h, mgrit_status s, const std::string &msg) {
  if (h) h->err = msg;
  return s;
}

mgrit_status hipfail(mgrit_handle *h, hipError_t e, const char *where) {
  return fail(h, MGRIT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                 \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hipfail((h), e_, #expr); \
  } while (0)

thread_local std::string g_setup_error;

// Pinned, mapped, coherent host memory in 256-byte slots, one per handle.
// Blocks are taken from the runtime 64 KiB at a time and kept for the life
// of the process, so creating and destroying handles never frees pinned
// memory (which would synchronise the device).
std::mutex g_pinned_mu;
std::vector<std::pair<char *, char *>> g_pinned_free;  // (host, device) addresses
std::map<char *, char *> g_pinned_dev;                 // host slot -> device address

bool pinned_slot_take(char *&host, char *&dev) {
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  if (g_pinned_free.empty()) {
    const size_t block = 64 << 10;
    char *hb = nullptr, *db = nullptr;
    if (hipHostMalloc((void **)&hb, block, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return false;
    if (hipHostGetDevicePointer((void **)&db, hb, 0) != hipSuccess) return false;
    for (size_t o = block; o > 0; o -= 256) g_pinned_free.push_back({hb + o - 256, db + o - 256});
  }
  host = g_pinned_free.back().first;
  dev = g_pinned_free.back().second;
  g_pinned_free.pop_back();
  g_pinned_dev[host] = dev;
  std::memset(host, 0, 256);
  return true;
}

void pinned_slot_give(char *host) {
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  auto it = g_pinned_dev.find(host);
  if (it == g_pinned_dev.end()) return;
  g_pinned_free.push_back({host, it->second});
  g_pinned_dev.erase(it);
}

mgrit_status setup_impl(const mgrit_problem *P, const mgrit_options *O, void *stream, void *ws, uint64_t ws_bytes,
                        mgrit_handle **out, bool noalloc = false);

// Build the StepOp of a solve-free or solve-carrying operator.
bool attach_solve(StepOp &op, const std::map<int, ld> &taps, const Layout &lay, std::vector<double> &tabs,
                  std::vector<size_t> &offsets, std::string &err) {
  Factor F;
  if (!factorize(taps, F, err)) return false;
  op.has_solve = (F.kf + F.kb) > 0 || std::fabs(F.C - 1) > 0;
  op.cinv = (double)(1 / F.C);
  op.fw.k = F.kf;
  op.bw.k = F.kb;
  for (int m = 0; m < KMAX; ++m) {
    op.fw.a[m] = (double)F.a[m];
    op.bw.a[m] = (double)F.b[m];
  }
  std::vector<double> t;
  if (F.kf > 0) {
    recurrence_tables(F.kf, F.a, lay, t);
    offsets.push_back(tabs.size());
    tabs.insert(tabs.end(), t.begin(), t.end());
  } else {
    offsets.push_back((size_t)-1);
  }
  if (F.kb > 0) {
    recurrence_tables(F.kb, F.b, lay, t);
    offsets.push_back(tabs.size());
    tabs.insert(tabs.end(), t.begin(), t.end());
  } else {
    offsets.push_back((size_t)-1);
  }
  // truncated-carry plan for the windowed kernel: 32 points per thread where
  // that still gives at least 256 threads, else 16 (MGRIT_WIN_L = 16 or 32
  // forces one, MGRIT_WIN_L_COARSE for the coarse operators only), and only
  // when both recurrences have a short enough carry
  op.win_L = 0;
  const int nx = lay.nx;
  const int Lenv = (op.kind == OP_SLC && env_int("MGRIT_WIN_L_COARSE", 0)) ? env_int("MGRIT_WIN_L_COARSE", 0)
                                                                          : env_int("MGRIT_WIN_L", 0);
  if (env_int("MGRIT_NO_WINDOW", 0) == 0 && op.has_solve && (op.kind == OP_POLY_W || op.kind == OP_SLC)) {
    for (int Lw : {32, 16}) {
      if (Lenv ? Lw != Lenv : (Lw == 32 && nx < 32 * 256)) continue;
      const int nthr = nx / Lw;
      if (nx != nthr * Lw || nthr % WAVE || nthr > (Lw == 32 ? 512 : 1024) || nthr < WAVE) continue;
      if (!window_instance(op.kind, F.kf, F.kb, Lw)) continue;
      if (op.kind == OP_SLC && op.sl_l + op.sl_r + 1 != 2 * F.kf) continue;
      std::vector<double> tf, tb;
      int Df = 1, Db = 1;
      if (F.kf > 0 && !window_tables(F.kf, F.a, Lw, nx, Df, tf)) continue;
      if (F.kb > 0 && !window_tables(F.kb, F.b, Lw, nx, Db, tb)) continue;
      op.win_L = Lw;
      op.fw.D = Df;
      op.bw.D = Db;
      offsets.push_back(tf.empty() ? (size_t)-1 : tabs.size());
      tabs.insert(tabs.end(), tf.begin(), tf.end());
      offsets.push_back(tb.empty() ? (size_t)-1 : tabs.size());
      tabs.insert(tabs.end(), tb.begin(), tb.end());
      break;
    }
  }
  if (op.kind == OP_POLY_W) {
    ld ci = 1;
    for (int i = 0; i < op.ncoef; ++i) {
      op.wcoef[i] = (double)((ld)op.coef[i] * ci);
      ci /= F.C;
    }
  }
  return true;
}

struct FineInfo {
  int l = 0, r = 0;
  std::vector<double> w;  // upwind weights, offsets -l..r
  Tableau tab;
  std::vector<ld> beta;
  ld efd = 0, erk = 0;
};

mgrit_status fine_info(const mgrit_problem &P, FineInfo &fi, std::string &err) {
  if (P.upwind_order < 1 || P.upwind_order > 5) {
    err = "upwind_order must be in 1..5";
    return MGRIT_EINVAL;
  }
  if (P.rk_kind != MGRIT_ERK && P.rk_kind != MGRIT_SDIRK) {
    err = "rk_kind must be MGRIT_ERK or MGRIT_SDIRK";
    return MGRIT_EINVAL;
  }
  if (P.rk_stages != 0) {
    if (!custom_tableau(P, fi.tab, err)) return MGRIT_EINVAL;
    if (P.rk_order < 1 || P.rk_order > 2 * MAXCOEF) {
      err = "custom tableau: rk_order out of range";
      return MGRIT_EINVAL;
    }
    // the linear order conditions b^T A^{j-1} 1 = 1/j!, j = 1..q (Sec. 4.2)
    const std::vector<ld> beta = rk_series(fi.tab, P.rk_order);
    for (int j = 1; j <= P.rk_order; ++j)
      if (std::fabs(beta[j] - 1 / factorial(j)) > 1e-12L / factorial(j)) {
        err = "custom tableau fails the linear order condition b^T A^" + std::to_string(j - 1) + " 1 = 1/" +
              std::to_string(j) + "!";
        return MGRIT_EINVAL;
      }
  } else if (!make_tableau(P.rk_kind, P.rk_order, fi.tab)) {
    err = "unsupported Runge-Kutta method (ERK 1..5, SDIRK 1..3)";
    return MGRIT_EINVAL;
  }
  upwind_stencil(P.upwind_order, fi.l, fi.r, fi.w);
  const int q = P.rk_order, p = P.upwind_order;
  fi.beta = rk_series(fi.tab, std::max(q + 1, fi.tab.s + 1));
  fi.erk = fi.beta[q + 1] - 1 / factorial(q + 1);
  // eq. (e_FD_def)
  fi.efd = ((fi.r % 2) ? -1 : 1) * factorial(fi.l) * factorial(fi.r) / factorial(p + 1);
  return MGRIT_OK;
}

std::complex<double> upwind_symbol(const FineInfo &fi, double om) {
  std::complex<double> s = 0;
  for (int j = -fi.l; j <= fi.r; ++j) s += fi.w[j + fi.l] * std::polar(1.0, j * om);
  return s;
}

// ERK stability: max over omega of |R(-c Lhat(omega))| <= 1 (Sec. 4.3, Table 2).
// R is the degree-s polynomial sum_j beta_j z^j of an explicit tableau.  The
// samples om_k = pi k / N take the phasors e^{i j om_k} from one table of
// e^{i pi n / N}, n < 2N (built once), so each sample is a few complex
// multiply-adds, written on real pairs.
bool erk_stable(const FineInfo &fi, double c) {
  constexpr int N = 16384;
  static const std::vector<double> ph = [] {
    std::vector<double> t(4 * N);
    for (int n = 0; n < 2 * N; ++n) {
      t[2 * n] = std::cos(M_PI * n / N);
      t[2 * n + 1] = std::sin(M_PI * n / N);
    }
    return t;
  }();
  const int s = fi.tab.s;
  const std::vector<ld> beta_l = rk_series(fi.tab, s);
  double beta[16];
  for (int j = 0; j <= s; ++j) beta[j] = (double)beta_l[j];
  const int nt = fi.l + fi.r + 1;
  double cw[16];
  for (int t = 0; t < nt; ++t) cw[t] = -c * fi.w[t];
  bool ok = true;
  for (int k = 1; k <= N; ++k) {
    double zr = 0, zi = 0;
    for (int t = 0; t < nt; ++t) {
      const int n = ((t - fi.l) * k) & (2 * N - 1);  // phase index of e^{i (t - l) om_k} (2N = 2^15)
      zr += cw[t] * ph[2 * n];
      zi += cw[t] * ph[2 * n + 1];
    }
    double ar = beta[s], ai = 0;
    for (int j = s - 1; j >= 0; --j) {
      const double nr = ar * zr - ai * zi + beta[j];
      ai = ar * zi + ai * zr;
      ar = nr;
    }
    ok &= ar * ar + ai * ai <= (1 + 1e-10) * (1 + 1e-10);
  }
  return ok;
}

// The corrected semi-Lagrangian coarse step of every coarse level
// (eqs. MOL-SL-corrected, MOL-SL-corrected-multilevel) for the 1D problem at
// CFL c on n points: level l (1-based) steps by m_1...m_l fine steps, its
// shift is c m_1...m_l, and phi follows the recursion over the levels
// (phi_q carries the Runge-Kutta term separately when q != p).  plain: phi = 0.
struct SlLevel {
  double shift = 0, eps = 0, phi_p = 0, phi_q = 0;
  int64_t K = 0;
  StepOp op{};
  Layout lay{};
  std::vector<double> tabs;
  std::vector<size_t> offs;
};

bool sl_chain(const FineInfo &fi, int p, int q, double c, const std::vector<int> &ms, int n, int Lcoarse, bool plain,
              std::vector<SlLevel> &out, std::string &err) {
  const int sgn = ((p + 1) % 2) ? -1 : 1;  // (-1)^{p+1}
  ld prod = 1, phi_p = 0, phi_q = 0, eps_prev = 0;
  out.assign(ms.size(), SlLevel{});
  for (size_t i = 0; i < ms.size(); ++i) {
    SlLevel &Lv = out[i];
    const int mcur = ms[i];
    prod *= mcur;
    const ld shift = (ld)c * prod;
    const ld Kf = std::floor(shift);
    const ld eps = shift - Kf;
    if (i == 0) {
      if (q == p) {
        phi_p = mcur * ((ld)c * fi.efd + std::pow(-(ld)c, (ld)(p + 1)) * fi.erk) + sgn * f_poly(p, eps);
        phi_q = 0;
      } else {
        phi_p = mcur * (ld)c * fi.efd + sgn * f_poly(p, eps);
        phi_q = mcur * std::pow(-(ld)c, (ld)(q + 1)) * fi.erk;
      }
    } else {
      phi_p = sgn * (-mcur * f_poly(p, eps_prev) + f_poly(p, eps)) + mcur * phi_p;
      phi_q = mcur * phi_q;
    }
    eps_prev = eps;
    Lv.shift = (double)shift;
    Lv.K = (int64_t)Kf;
    Lv.eps = (double)eps;
    Lv.phi_p = plain ? 0.0 : (double)phi_p;
    Lv.phi_q = plain ? 0.0 : (double)phi_q;
    StepOp &op = Lv.op;
    op = StepOp{};
    op.kind = OP_SLC;
    op.repeat = 1;
    std::vector<double> slw;
    sl_weights(p, eps, op.sl_l, op.sl_r, slw);
    for (size_t j = 0; j < slw.size(); ++j) op.slw[j] = slw[j];
    op.sl_K = (int)(((int64_t)Kf) % n);
    std::map<int, ld> taps;
    taps[0] += 1;
    for (auto &kv : dmat(p + 1)) taps[kv.first] -= (ld)Lv.phi_p * kv.second;
    if (Lv.phi_q != 0)
      for (auto &kv : dmat(q + 1)) taps[kv.first] -= (ld)Lv.phi_q * kv.second;
    Lv.lay = choose_layout(n, Lcoarse);
    Lv.lay.dbuf = 1;
    if (lds_bytes_for(Lv.lay, 1) > LDS_LIMIT) Lv.lay.dbuf = 0;
    if (!attach_solve(op, taps, Lv.lay, Lv.tabs, Lv.offs, err)) {
      err = "coarse operator: " + err;
      return false;
    }
  }
  return true;
}

// An explicit step R(Z) = sum_i beta_i Z^i, Z = -c L_p (eq. MOL_M_def), written
// out as one circulant stencil: the powers of Z's stencil are convolved and
// summed in extended precision, offsets -s l .. s r (s = degree of R).  The
// same operator as the Horner form up to rounding, with s(l + r) + 1 products
// per point instead of s(l + r + 2).
void write_out_erk(const FineInfo &fi, double c, StepOp &op) {
  const int s = fi.tab.s, cl = s * fi.l, cr = s * fi.r, n = cl + cr + 1;
  std::vector<ld> pw(n, 0), acc(n, 0);  // index: offset + cl
  pw[cl] = 1;
  acc[cl] = fi.beta[0];
  for (int i = 1; i <= s; ++i) {
    std::vector<ld> nxt(n, 0);
    for (int o = -(i - 1) * fi.l; o <= (i - 1) * fi.r; ++o)
      for (int j = -fi.l; j <= fi.r; ++j) nxt[o + j + cl] += pw[o + cl] * (-(ld)c * (ld)fi.w[j + fi.l]);
    pw.swap(nxt);
    for (int k = 0; k < n; ++k) acc[k] += fi.beta[i] * pw[k];
  }
  op.ct_l = cl;
  op.ct_r = cr;
  for (int k = 0; k < n; ++k) op.ctaps[k] = (double)acc[k];
}

// One Runge-Kutta step of the upwind semi-discretisation at CFL c
// (eq. MOL_M_def), as a Horner form: ERK R(z) in z = -c L_p (OP_POLY_Z);
// SDIRK R as a polynomial in w = (I + gamma c L_p)^{-1} (OP_POLY_W), every
// stage solving with the same periodic banded matrix.
bool build_mol_step(const FineInfo &fi, int rk_kind, double c, int nx, int Lpref, StepOp &op, Layout &lay,
                    std::vector<double> &tabs, std::vector<size_t> &offs, std::string &err) {
  op = StepOp{};
  op.repeat = 1;
  if (rk_kind == MGRIT_ERK) {
    lay = choose_layout(nx, Lpref);
    lay.dbuf = 1;
    if (lds_bytes_for(lay, 0) > LDS_LIMIT) lay.dbuf = 0;
    op.kind = OP_POLY_Z;
    op.ncoef = fi.tab.s + 1;
    for (int i = 0; i <= fi.tab.s; ++i) op.coef[i] = (double)fi.beta[i];
    op.st_l = fi.l;
    op.st_r = fi.r;
    for (int j = 0; j <= fi.l + fi.r; ++j) op.taps[j] = -c * fi.w[j];
    return true;
  }
  // R(z) = P(z) / (1 - g z)^s as a polynomial in w = 1/(1 - g z):
  // z = (w - 1)/(g w)  =>  R = sum_n P_n g^-n (w - 1)^n w^(s-n).
  lay = choose_layout(nx, Lpref);
  const int s = fi.tab.s;
  const ld g = fi.tab.gamma;
  std::vector<ld> beta = rk_series(fi.tab, s);
  std::vector<ld> Q(s + 1, 0), Pc(s + 1, 0), coefw(s + 1, 0);
  for (int n = 0; n <= s; ++n) {
    ld bin = 1;
    for (int i = 0; i < n; ++i) bin = bin * (s - i) / (i + 1);
    Q[n] = bin * std::pow(-g, (ld)n);
  }
  for (int n = 0; n <= s; ++n)
    for (int j = 0; j <= n; ++j) Pc[n] += beta[j] * Q[n - j];
  for (int n = 0; n <= s; ++n) {
    ld bin = 1;
    for (int k = 0; k <= n; ++k) {
      coefw[k + s - n] += Pc[n] * std::pow(g, (ld)-n) * bin * (((n - k) % 2) ? -1 : 1);
      bin = bin * (n - k) / (k + 1);
    }
  }
  op.kind = OP_POLY_W;
  op.ncoef = s + 1;
  for (int i = 0; i <= s; ++i) op.coef[i] = (double)coefw[i];
  std::map<int, ld> taps;
  taps[0] += 1;
  for (int j = -fi.l; j <= fi.r; ++j) taps[j] += g * c * fi.w[j + fi.l];
  if (!attach_solve(op, taps, lay, tabs, offs, err)) {
    err = "SDIRK stage operator: " + err;
    return false;
  }
  // self-check of the w-polynomial against R(z)
  for (double zr : {-0.3, -2.0, -7.5}) {
    const std::complex<double> z(zr, 0.7);
    const std::complex<double> w = 1.0 / (1.0 - (double)g * z);
    std::complex<double> acc = 0;
    for (int i = s; i >= 0; --i) acc = acc * w + (double)coefw[i];
    const std::complex<double> ref = rk_R(fi.tab, z);
    if (std::abs(acc - ref) > 1e-11 * (1 + std::abs(ref))) {
      err = "internal: SDIRK rational form check failed";
      return false;
    }
  }
  return true;
}


}  // namespace

extern "C" {

const char *mgrit_status_string(mgrit_status s) {
  switch (s) {
    case MGRIT_OK: return "ok";
    case MGRIT_ENOTCONVERGED: return "not converged within max_iter";
    case MGRIT_EINVAL: return "invalid argument";
    case MGRIT_EUNSTABLE: return "explicit scheme above its CFL limit";
    case MGRIT_ENOMEM: return "device allocation failed";
    case MGRIT_EDEVICE: return "HIP runtime error";
    case MGRIT_EDIVERGED: return "diverged";
  }
  return "unknown status";
}

const char *mgrit_last_error(const mgrit_handle *h) {
  if (!h) return g_setup_error.c_str();
  return h->err.c_str();
}

void mgrit_destroy(mgrit_handle *h) {
  if (!h) return;
  // work still queued on the handle's stream may write its workspace and
  // its pinned words (an abandoned incremental solve): wait for it before
  // either is reused
  if (h->arena) (void)hipStreamSynchronize(h->stream);
  if (h->arena && h->owns_arena) (void)hipFree(h->arena);
  if (h->host_arena) pinned_slot_give(h->host_arena);
  if (h->ctl_ev) (void)hipEventDestroy(h->ctl_ev);
  for (auto &pe : h->ev_pending) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (auto e : h->ev_free) (void)hipEventDestroy(e);
  delete h;
}

mgrit_status mgrit_setup(const mgrit_problem *P, const mgrit_options *O, void *stream, mgrit_handle **out) {
  return setup_impl(P, O, stream, nullptr, 0, out);
}

mgrit_status mgrit_setup_ws(const mgrit_problem *P, const mgrit_options *O, void *stream, void *workspace,
                            uint64_t workspace_bytes, mgrit_handle **out) {
  if (!workspace) {
    g_setup_error = "workspace is required";
    if (out) *out = nullptr;
    return MGRIT_EINVAL;
  }
  return setup_impl(P, O, stream, workspace, workspace_bytes, out);
}

}  // extern "C"

namespace {

// The kernels' LDS attribute is process-wide and always raised to LDS_LIMIT:
// set it once per device, before the first handle on that device launches
// anything, and never again while other threads may be launching.
std::mutex g_config_mu;
std::vector<int> g_configured;  // devices done

hipError_t configure_once() {
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  std::lock_guard<std::mutex> lk(g_config_mu);
  for (int d : g_configured)
    if (d == dev) return hipSuccess;
  if (hipError_t e = configure_kernels(LDS_LIMIT)) return e;
  if (hipError_t e = configure_2d_kernels(LDS_LIMIT)) return e;
  g_configured.push_back(dev);
  return hipSuccess;
}

// Tile-width autotuner of the level-0 explicit relaxation: time pass A with
// every candidate width on the handle's own buffers (zeroed C-points, three
// launches after one warm-up) and keep the fastest.  The choice is cached per
// process by (nx, m, Horner depth, stencil extents, N_c), the things the
// launch shape depends on; every width gives the same bits, so the choice
// changes only the time.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, int> g_tune_cache;

hipError_t tune_tiles(mgrit_handle *h) {
  Level &L0 = h->lv[0];
  const int depth = L0.t_depth, sl = L0.t_sl, sr = L0.t_sr, comp = L0.t_comp;
  const int nx = (int)h->prob.nx;
  const int64_t nc = L0.nt / L0.m;
  const std::vector<int64_t> key{nx, L0.m, depth, sl, sr, comp, nc};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      choose_tiles(nx, L0.m, depth, sl, sr, it->second, L0.tg, comp);
      return hipSuccess;
    }
  }
  hipError_t e = launch_fill(L0.c[0], (nc + 1) * (int64_t)nx, 0.0, h->stream);
  if (e) return e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1))) return e;
  int best_p = L0.tg.P;
  float best_ms = -1;
  for (int cand : {8, 16}) {
    TileGeom tg{};
    if (!choose_tiles(nx, L0.m, depth, sl, sr, cand, tg, comp)) continue;
    TileArgs ta{};
    ta.mode = MODE_PASS_A;
    ta.m = L0.m;
    ta.nint = nc;
    ta.cin = L0.c[0];
    ta.cout = L0.c[1];
    ta.normpart = h->normpart;
    if ((e = launch_tiles(L0.desc, tg, ta, h->stream))) break;
    if ((e = hipEventRecord(e0, h->stream))) break;
    for (int r = 0; r < 3 && !e; ++r) e = launch_tiles(L0.desc, tg, ta, h->stream);
    if (e || (e = hipEventRecord(e1, h->stream)) || (e = hipEventSynchronize(e1))) break;
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, e0, e1))) break;
    if (best_ms < 0 || ms < best_ms) {
      best_ms = ms;
      best_p = cand;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e) return e;
  choose_tiles(nx, L0.m, depth, sl, sr, best_p, L0.tg, comp);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best_p;
  return hipSuccess;
}

mgrit_status setup_impl(const mgrit_problem *P, const mgrit_options *O, void *stream, void *ws, uint64_t ws_bytes,
                        mgrit_handle **out, bool noalloc) {
  g_setup_error.clear();
  if (out) *out = nullptr;
  if (!P || !O || !out) {
    g_setup_error = "null argument";
    return MGRIT_EINVAL;
  }
  auto bad = [&](mgrit_status s, const std::string &m) {
    g_setup_error = m;
    return s;
  };
  if (!(P->velocity > 0) || !(P->x_hi > P->x_lo) || !(P->cfl > 0)) return bad(MGRIT_EINVAL, "need velocity > 0, x_hi > x_lo, cfl > 0");
  if (P->nx < 1 || P->nx > MGRIT_MAX_NX) return bad(MGRIT_EINVAL, "nx must be in 1..16384");
  if (P->nt < 1) return bad(MGRIT_EINVAL, "nt must be >= 1");
  if (O->max_levels < 2 || O->max_levels > MGRIT_MAX_LEVELS) return bad(MGRIT_EINVAL, "max_levels must be in 2..16");
  if (O->nu < 0 || O->nu > 8) return bad(MGRIT_EINVAL, "nu must be in 0..8");
  if (O->max_iter < 0) return bad(MGRIT_EINVAL, "max_iter must be >= 0");
  if (!(O->rtol >= 0)) return bad(MGRIT_EINVAL, "rtol must be >= 0");
  if (O->cg_kind < 0 || O->cg_kind > 3) return bad(MGRIT_EINVAL, "unknown coarse operator");
  if (O->coarse_launch < 0 || O->coarse_launch > 1) return bad(MGRIT_EINVAL, "coarse_launch must be 0 or 1");
  if (O->tile_tune < 0 || O->tile_tune > 1) return bad(MGRIT_EINVAL, "tile_tune must be 0 or 1");
  if (O->precision != MGRIT_PREC_FP64 && O->precision != MGRIT_PREC_MIXED) return bad(MGRIT_EINVAL, "unknown precision");
  if (O->precision == MGRIT_PREC_MIXED && !(O->inner_rtol > 0 && O->inner_rtol < 1))
    return bad(MGRIT_EINVAL, "mixed precision needs 0 < inner_rtol < 1");
  if (O->precision == MGRIT_PREC_MIXED && O->inner_max_iter < 1)
    return bad(MGRIT_EINVAL, "mixed precision needs inner_max_iter >= 1");
  if (O->coarse_solve < 0 || O->coarse_solve > 1) return bad(MGRIT_EINVAL, "coarse_solve must be 0 or 1");
  if (O->coarse_solve == 1) {
    if (O->cg_kind != MGRIT_CG_SL_CORRECTED)
      return bad(MGRIT_EINVAL, "GMRES coarse solves apply to the corrected semi-Lagrangian operator only");
    if (O->precision != MGRIT_PREC_FP64) return bad(MGRIT_EINVAL, "GMRES coarse solves run in float64 only");
    if (O->gmres_max_iter < 1 || O->gmres_max_iter > GMRES_MAX) return bad(MGRIT_EINVAL, "gmres_max_iter must be in 1..32");
    if (!(O->gmres_rtol > 0 && O->gmres_rtol < 1)) return bad(MGRIT_EINVAL, "gmres_rtol must be in (0, 1)");
  }
  const bool sl_coarse = O->cg_kind == MGRIT_CG_SL_CORRECTED || O->cg_kind == MGRIT_CG_SL_PLAIN;
  if (sl_coarse && P->upwind_order % 2 == 0)
    return bad(MGRIT_EINVAL, "semi-Lagrangian coarse operators need odd upwind order");
  if (O->cg_kind == MGRIT_CG_IDEAL && O->max_levels != 2) return bad(MGRIT_EINVAL, "ideal coarse operator: two levels only");

  FineInfo fi;
  std::string err;
  mgrit_status st = fine_info(*P, fi, err);
  if (st != MGRIT_OK) return bad(st, err);
  const double c = P->cfl;
  const int p = P->upwind_order, q = P->rk_order;
  if (P->rk_kind == MGRIT_ERK && !erk_stable(fi, c)) return bad(MGRIT_EUNSTABLE, "CFL number above the stability limit of the explicit scheme");
  if (q != p && (q % 2 == 0) && sl_coarse)
    return bad(MGRIT_EINVAL, "mixed orders need an odd Runge-Kutta order for the correction");

  // level hierarchy
  std::vector<int64_t> nts;
  std::vector<int> ms;
  if (!level_hierarchy(*P, *O, nts, ms, err)) return bad(MGRIT_EINVAL, err);
  const int nlev = (int)nts.size();

  mgrit_handle *h = new mgrit_handle();
  h->prob = *P;
  h->opt = *O;
  h->stream = (hipStream_t)stream;
  h->lv.resize(nlev);
  const int nx = (int)P->nx;
  // Points per thread of the coarse step kernels: 8 up to nx = 2048 (two to
  // four wavefronts per interval hide more of a step's latency than one or
  // two; measured 8-13% faster coarse cycles at nx = 1024 and 2048), else 16.
  const int Lfine = env_int("MGRIT_L_FINE", 16), Lcoarse = env_int("MGRIT_L_COARSE", nx <= 2048 ? 8 : 16);

  // ---- fine operator (eq. MOL_M_def)
  std::vector<std::vector<double>> tabs(nlev);
  std::vector<std::vector<size_t>> offs(nlev);
  {
    Level &L0 = h->lv[0];
    L0.nt = nts[0];
    L0.m = ms[0];
    StepOp &op = L0.op;
    op = StepOp{};
    op.repeat = 1;
    if (P->rk_kind == MGRIT_ERK) {
      // the tiles apply the step written out as one stencil where an
      // instance exists for its extents (ERK3 + U3), else by Horner; the
      // halo, m (depth x extent), is the same either way
      const int s = fi.tab.s;
      L0.t_comp = env_int("MGRIT_TILE_COMPOSE", 1) != 0 && s * fi.l == 6 && s * fi.r == 3;
      L0.t_depth = L0.t_comp ? 1 : s;
      L0.t_sl = L0.t_comp ? s * fi.l : fi.l;
      L0.t_sr = L0.t_comp ? s * fi.r : fi.r;
      L0.tiles = env_int("MGRIT_NO_TILES", 0) == 0 &&
                 choose_tiles(nx, ms[0], L0.t_depth, L0.t_sl, L0.t_sr, env_int("MGRIT_TILE_P", 0), L0.tg, L0.t_comp);
      L0.seq_tiles = env_int("MGRIT_NO_TILES", 0) == 0 &&
                     choose_seq_tiles(nx, P->nt, fi.tab.s, fi.l, fi.r, env_int("MGRIT_SEQ_P", 0),
                                      env_int("MGRIT_SEQ_T", 0), L0.seq_tg, L0.seq_T);
    }
    if (!build_mol_step(fi, P->rk_kind, c, nx, P->rk_kind == MGRIT_ERK ? Lfine : Lcoarse, op, L0.lay, tabs[0],
                        offs[0], err)) {
      mgrit_destroy(h);
      return bad(MGRIT_EINVAL, err);
    }
    if (L0.t_comp) write_out_erk(fi, c, op);
  }

  // ---- coarse operators (eqs. MOL-SL-corrected, MOL-SL-corrected-multilevel)
  if (O->cg_kind == MGRIT_CG_SL_CORRECTED || O->cg_kind == MGRIT_CG_SL_PLAIN) {
    std::vector<SlLevel> chain;
    if (!sl_chain(fi, p, q, c, std::vector<int>(ms.begin(), ms.begin() + (nlev - 1)), nx, Lcoarse,
                  O->cg_kind == MGRIT_CG_SL_PLAIN, chain, err)) {
      mgrit_destroy(h);
      return bad(MGRIT_EINVAL, err);
    }
    for (int l = 1; l < nlev; ++l) {
      Level &Lv = h->lv[l];
      SlLevel &S = chain[l - 1];
      Lv.nt = nts[l];
      Lv.m = (l < nlev - 1) ? ms[l] : 0;
      Lv.shift = S.shift;
      Lv.K = S.K;
      Lv.eps = S.eps;
      Lv.phi_p = S.phi_p;
      Lv.phi_q = S.phi_q;
      Lv.op = S.op;
      Lv.lay = S.lay;
      // From nx = 8192 the lean kernel needs 8 wavefronts and its registers
      // spill; the windowed kernel (32 points per thread) measured 6-15%
      // faster there, so it takes the coarse steps where it has a plan.
      const int no_lean_env = env_int("MGRIT_NO_LEAN", -1);
      Lv.op.no_lean = no_lean_env >= 0 ? no_lean_env : (nx >= 8192 && window_applies(Lv.op, Lv.lay) ? 1 : 0);
      tabs[l] = std::move(S.tabs);
      offs[l] = std::move(S.offs);
      if (O->coarse_solve == 1) {
        // T = I - phi_p D^(p+1) - phi_q D^(q+1) applied as its stencil,
        // solved by GMRES (Sec. 6.3)
        std::map<int, ld> t;
        t[0] += 1;
        for (auto &kv : dmat(p + 1)) t[kv.first] -= (ld)Lv.phi_p * kv.second;
        if (Lv.phi_q != 0)
          for (auto &kv : dmat(q + 1)) t[kv.first] -= (ld)Lv.phi_q * kv.second;
        int tk = 0;
        for (auto &kv : t) tk = std::max(tk, std::abs(kv.first));
        StepOp &op = Lv.op;
        op.gmres_max = O->gmres_max_iter;
        op.gmres_rtol = O->gmres_rtol;
        op.t_k = tk;
        for (int j = 0; j < MAXTAPS; ++j) op.ttaps[j] = 0;
        for (auto &kv : t) op.ttaps[kv.first + tk] = (double)kv.second;
        op.win_L = 0;
        if (2 * tk + 1 > MAXTAPS || Lv.lay.ragged || gmres_lds_bytes(Lv.lay, op.gmres_max) > LDS_LIMIT) {
          mgrit_destroy(h);
          return bad(MGRIT_EINVAL, "GMRES coarse solves need nx a multiple of 128 and at most 16384 points");
        }
      }
    }
  } else {
    ld prod = 1;
    for (int l = 1; l < nlev; ++l) {
      Level &Lv = h->lv[l];
      Lv.nt = nts[l];
      Lv.m = (l < nlev - 1) ? ms[l] : 0;
      const int mcur = ms[l - 1];
      prod *= mcur;
      if (O->cg_kind == MGRIT_CG_IDEAL) {
        Lv.op = h->lv[0].op;
        Lv.op.repeat = ms[0];
        Lv.lay = h->lv[0].lay;
        tabs[l] = tabs[0];
        offs[l] = offs[0];
        continue;
      }
      // MGRIT_CG_REDISC: the fine scheme rediscretised with the level's step
      // (Sec. 5, Theorem 1)
      const double cl = (double)((ld)c * prod);
      if (P->rk_kind == MGRIT_ERK && !erk_stable(fi, cl)) {
        mgrit_destroy(h);
        return bad(MGRIT_EUNSTABLE, "rediscretised explicit coarse step above its CFL limit");
      }
      Lv.shift = cl;
      if (!build_mol_step(fi, P->rk_kind, cl, nx, Lcoarse, Lv.op, Lv.lay, tabs[l], offs[l], err)) {
        mgrit_destroy(h);
        return bad(MGRIT_EINVAL, "coarse operator: " + err);
      }
    }
  }

  // Every layout chosen above needs at most LDS_LIMIT bytes; the attribute is
  // per kernel and process-wide, so it is always raised to that limit.
  if (hipError_t e = configure_once()) {
    mgrit_destroy(h);
    return bad(MGRIT_EDEVICE, std::string("configure: ") + hipGetErrorString(e));
  }
  // Persistent coarse V-cycle: every coarse level takes the lean kernel, the
  // tables of all of them fit in LDS beside the vector, and the largest
  // level's intervals can all be resident at once.
  if (nlev >= 2 && O->coarse_launch == 0 && env_int("MGRIT_NO_PERSISTENT", 0) == 0) {
    bool all_lean = true;
    for (int l = 1; l < nlev; ++l) all_lean = all_lean && lean_slc_applies(h->lv[l].op, h->lv[l].lay);
    const size_t lds = all_lean ? coarse_vcycle_lds(h->lv[1].op, h->lv[1].lay, nlev - 1) : 0;
    int64_t grid = 1;
    int64_t longest = h->lv[nlev - 1].nt;  // steps of the longest phase (the barrier wait bound assumes <= 256)
    for (int l = 1; l + 1 < nlev; ++l) {
      grid = std::max<int64_t>(grid, h->lv[l].nt / h->lv[l].m);
      longest = std::max<int64_t>(longest, h->lv[l].m);
    }
    // A grid barrier costs about 35 ns per workgroup (every workgroup's
    // device-scope release; measured 3 us at 64 workgroups, 9.5 us at 256,
    // 36 us at 1024), a kernel boundary about 5 us: past 128 workgroups one
    // launch per pass is faster.
    const int64_t fast_grid = std::min<int64_t>(MAX_PERSISTENT_GRID, env_int("MGRIT_PERSISTENT_MAX_GRID", 128));
    if (lds > 0 && longest <= 256 && grid <= fast_grid &&
        grid <= coarse_vcycle_max_grid(h->lv[1].op, h->lv[1].lay, lds)) {
      h->cv_ok = true;
      h->cv_lds = lds;
      h->cv_grid = grid;
    }
  }

  // ---- device data: one allocation carved into 256-byte aligned pieces.
  // Its head (scan tables, level descriptors, grid-barrier state) is
  // uploaded in one copy; the iterate, residual and norm buffers follow.
  auto al = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
  const size_t none = (size_t)-1;
  std::vector<size_t> o_tab(nlev, none), o_desc(nlev, none), o_c0(nlev, none), o_c1(nlev, none), o_r(nlev, none);
  size_t off = 0;
  for (int l = 0; l < nlev; ++l)
    if (!tabs[l].empty()) o_tab[l] = off, off += al(tabs[l].size() * sizeof(double));
  for (int l = 0; l < nlev; ++l) o_desc[l] = off, off += al(sizeof(LevelDesc));
  const bool mixed = O->precision == MGRIT_PREC_MIXED;
  std::vector<size_t> o_tab32(nlev, none), o_desc32(nlev, none);
  if (mixed) {
    for (int l = 0; l < nlev; ++l)
      if (!tabs[l].empty()) o_tab32[l] = off, off += al(tabs[l].size() * sizeof(float));
    for (int l = 0; l < nlev; ++l) o_desc32[l] = off, off += al(sizeof(LevelDesc));
  }
  size_t o_gs = none;
  if (h->cv_ok) o_gs = off, off += al(sizeof(GridSync));
  const size_t head = off;
  for (int l = 0; l + 1 < nlev; ++l) {
    const size_t rows = (size_t)(h->lv[l].nt / h->lv[l].m);
    o_c0[l] = off, off += al((rows + 1) * nx * sizeof(double));
    o_c1[l] = off, off += al((rows + 1) * nx * sizeof(double));
    o_r[l] = off, off += al(std::max<size_t>(rows * nx, 1) * sizeof(double));
  }
  std::vector<size_t> o_kry(nlev, none);  // GMRES bases of the coarse levels
  for (int l = 1; l < nlev; ++l)
    if (h->lv[l].op.gmres_max > 0) {
      const int64_t cap = (l < nlev - 1) ? h->lv[l].nt / h->lv[l].m : 1;
      h->lv[l].op.krylov_cap = cap;
      o_kry[l] = off, off += al((size_t)cap * (h->lv[l].op.gmres_max + 1) * nx * sizeof(double));
    }
  std::vector<size_t> o_c32a(nlev, none), o_c32b(nlev, none), o_r32(nlev, none);
  size_t o_g32 = none, o_e32 = none, o_u64 = none;
  if (mixed) {
    for (int l = 0; l + 1 < nlev; ++l) {
      const size_t rows = (size_t)(h->lv[l].nt / h->lv[l].m);
      o_c32a[l] = off, off += al((rows + 1) * nx * sizeof(float));
      o_c32b[l] = off, off += al((rows + 1) * nx * sizeof(float));
      o_r32[l] = off, off += al(std::max<size_t>(rows * nx, 1) * sizeof(float));
    }
    const size_t pts = (size_t)P->nt * nx;
    o_g32 = off, off += al(pts * sizeof(float));
    o_e32 = off, off += al((pts + nx) * sizeof(float));
    o_u64 = off, off += al((pts + nx) * sizeof(double));
  }
  h->normpart_len = std::max<int64_t>(P->nt, 1);
  if (h->lv[0].tiles) {
    h->normpart_len = std::max<int64_t>(h->normpart_len, (P->nt / ms[0]) * h->lv[0].tg.ntiles);
    if (O->tile_tune)  // room for every candidate width
      for (int cand : {8, 16}) {
        TileGeom tg{};
        if (choose_tiles(nx, ms[0], h->lv[0].t_depth, h->lv[0].t_sl, h->lv[0].t_sr, cand, tg, h->lv[0].t_comp))
          h->normpart_len = std::max<int64_t>(h->normpart_len, (P->nt / ms[0]) * tg.ntiles);
      }
  }
  const size_t o_np = off;
  off += al(h->normpart_len * sizeof(double));
  const size_t o_ns = off;
  off += al(sizeof(double));
  const size_t o_ctl = off;
  off += al(sizeof(SolveCtl));
  const size_t o_octl = off;
  off += al(sizeof(SolveCtl));
  if (ws) {
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) {
      mgrit_destroy(h);
      return bad(MGRIT_EINVAL, "workspace must be 256-byte aligned");
    }
    if (ws_bytes < off) {
      mgrit_destroy(h);
      return bad(MGRIT_EINVAL, "workspace too small: " + std::to_string(off) + " bytes needed");
    }
    h->arena = (char *)ws;
    h->owns_arena = false;
  } else {
    if (hipMalloc((void **)&h->arena, off) != hipSuccess) {
      mgrit_destroy(h);
      return bad(MGRIT_ENOMEM, "device workspace");
    }
    h->owns_arena = true;
  }
  h->arena_bytes = off;
  char *base = h->arena;
  std::vector<char> up(head, 0);
  for (int l = 0; l < nlev; ++l) {
    Level &Lv = h->lv[l];
    if (o_tab[l] != none) {
      Lv.tabs = (double *)(base + o_tab[l]);
      std::memcpy(up.data() + o_tab[l], tabs[l].data(), tabs[l].size() * sizeof(double));
    }
    if (offs[l].size() >= 2) {
      Lv.op.fw.tab = offs[l][0] == none ? nullptr : Lv.tabs + offs[l][0];
      Lv.op.bw.tab = offs[l][1] == none ? nullptr : Lv.tabs + offs[l][1];
    }
    if (offs[l].size() >= 4) {
      Lv.op.fw.wtab = offs[l][2] == none ? nullptr : Lv.tabs + offs[l][2];
      Lv.op.bw.wtab = offs[l][3] == none ? nullptr : Lv.tabs + offs[l][3];
    }
    if (o_kry[l] != none) Lv.op.krylov = (double *)(base + o_kry[l]);
    Lv.desc = (LevelDesc *)(base + o_desc[l]);
    const LevelDesc hd{Lv.op, Lv.lay};
    std::memcpy(up.data() + o_desc[l], &hd, sizeof(LevelDesc));
    if (o_c0[l] != none) {
      Lv.c[0] = (double *)(base + o_c0[l]);
      Lv.c[1] = (double *)(base + o_c1[l]);
      Lv.r = (double *)(base + o_r[l]);
    }
    if (mixed) {
      LevelDesc hd32{Lv.op, Lv.lay};
      if (o_tab32[l] != none) {
        Lv.tabs32 = (float *)(base + o_tab32[l]);
        float *dst = (float *)(up.data() + o_tab32[l]);
        for (size_t i = 0; i < tabs[l].size(); ++i) dst[i] = (float)tabs[l][i];
      }
      if (offs[l].size() >= 2) {
        hd32.op.fw.tab = offs[l][0] == none ? nullptr : Lv.tabs32 + offs[l][0];
        hd32.op.bw.tab = offs[l][1] == none ? nullptr : Lv.tabs32 + offs[l][1];
      }
      if (offs[l].size() >= 4) {
        hd32.op.fw.wtab = offs[l][2] == none ? nullptr : Lv.tabs32 + offs[l][2];
        hd32.op.bw.wtab = offs[l][3] == none ? nullptr : Lv.tabs32 + offs[l][3];
      }
      Lv.desc32 = (LevelDesc *)(base + o_desc32[l]);
      std::memcpy(up.data() + o_desc32[l], &hd32, sizeof(LevelDesc));
      if (o_c32a[l] != none) {
        Lv.c32[0] = (float *)(base + o_c32a[l]);
        Lv.c32[1] = (float *)(base + o_c32b[l]);
        Lv.r32 = (float *)(base + o_r32[l]);
      }
    }
  }
  if (mixed) {
    h->g32 = (float *)(base + o_g32);
    h->e32 = (float *)(base + o_e32);
    h->u64 = (double *)(base + o_u64);
  }
  if (o_gs != none) h->gsync = (GridSync *)(base + o_gs);  // zero from the upload
  h->normpart = (double *)(base + o_np);
  h->normsum = (double *)(base + o_ns);
  h->ctl = (SolveCtl *)(base + o_ctl);
  h->octl = (SolveCtl *)(base + o_octl);
  // on the handle's stream, where all of its work goes; the source is
  // pageable, so the call returns once it has been staged
  if (hipMemcpyAsync(base, up.data(), head, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
    mgrit_destroy(h);
    return bad(MGRIT_EDEVICE, "table upload");
  }
  // pinned host words: the norm read back by mgrit_residual and the mapped,
  // coherent copy of the iteration state (allocation-free mode: plain host
  // words, filled by copies the host waits for)
  if (noalloc) {
    h->noalloc = true;
    h->normsum_host = &h->norm_local;
    h->ctl_host = &h->ctl_local;
    h->ctl_host_dev = nullptr;
    *out = h;
    return MGRIT_OK;
  }
  char *slot_dev = nullptr;
  if (!pinned_slot_take(h->host_arena, slot_dev) ||
      hipEventCreateWithFlags(&h->ctl_ev, hipEventDisableTiming) != hipSuccess) {
    mgrit_destroy(h);
    return bad(MGRIT_ENOMEM, "pinned host words");
  }
  static_assert(sizeof(SolveCtl) <= 64, "pinned slot layout: norm at 0, outer state at 64, state at 128");
  h->normsum_host = (double *)h->host_arena;
  h->octl_host = (SolveCtl *)(h->host_arena + 64);
  h->octl_host_dev = (SolveCtl *)(slot_dev + 64);
  h->ctl_host = (SolveCtl *)(h->host_arena + 128);
  h->ctl_host_dev = (SolveCtl *)(slot_dev + 128);
  if (O->tile_tune && h->lv[0].tiles && nlev >= 2) {
    const hipError_t e = tune_tiles(h);
    if (e != hipSuccess) {
      mgrit_destroy(h);
      return bad(MGRIT_EDEVICE, std::string("tile tuning: ") + hipGetErrorString(e));
    }
  }
  *out = h;
  return MGRIT_OK;
}

}  // namespace

extern "C" {

int32_t mgrit_num_levels(const mgrit_handle *h) { return h ? (int32_t)h->lv.size() : 0; }

mgrit_status mgrit_level_info(const mgrit_handle *h, int32_t level, mgrit_level_desc *out) {
  if (!h || !out || level < 0 || level >= (int32_t)h->lv.size()) return MGRIT_EINVAL;
  const Level &L = h->lv[level];
  out->nt = L.nt;
  out->m = L.m;
  out->shift = L.shift;
  out->K = L.K;
  out->eps = L.eps;
  out->phi_p = L.phi_p;
  out->phi_q = L.phi_q;
  out->tile_p = (level == 0 && L.tiles) ? L.tg.P : 0;
  const bool win = window_applies(L.op, L.lay) && !(level >= 1 && lean_slc_applies(L.op, L.lay));
  out->win_L = win ? L.op.win_L : 0;
  out->win_D[0] = win && L.op.fw.k > 0 ? L.op.fw.D : 0;
  out->win_D[1] = win && L.op.bw.k > 0 ? L.op.bw.D : 0;
  out->gmres_max_iter = (level >= 1 && L.op.kind == OP_SLC) ? L.op.gmres_max : 0;
  return MGRIT_OK;
}

}  // extern "C"

namespace {

hipEvent_t take_event(mgrit_handle *h) {
  if (!h->ev_free.empty()) {
    hipEvent_t e = h->ev_free.back();
    h->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold finished event pairs into the profile (call after a stream sync).
void harvest_events(mgrit_handle *h) {
  for (auto &pe : h->ev_pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      h->prof.launches[pe.first] += 1;
      h->prof.total_ms[pe.first] += ms;
    }
    h->ev_free.push_back(pe.second.first);
    h->ev_free.push_back(pe.second.second);
  }
  h->ev_pending.clear();
}

hipError_t run_pass(mgrit_handle *h, const Level &L, int phase, int mode, int m, int64_t nint, const double *cin,
                    double *cout, const double *g, double *r, double *parent, double *out, int zero_init,
                    float *r32 = nullptr) {
  PassArgs pa{};
  pa.mode = mode;
  pa.m = m;
  pa.zero_init = zero_init;
  pa.nint = nint;
  pa.cin = cin;
  pa.cout = cout;
  pa.g = g;
  pa.r = r;
  pa.r32 = r32;
  pa.parent = parent;
  pa.out = out;
  pa.normpart = h->normpart;
  pa.stop = h->guard;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof_mask & (1u << phase)) {
    e0 = take_event(h);
    e1 = take_event(h);
    if (e0 && e1) (void)hipEventRecord(e0, h->stream);
  }
  hipError_t err = launch_pass(L.desc, L.op, L.lay, pa, h->stream);
  if (e0 && e1) {
    (void)hipEventRecord(e1, h->stream);
    h->ev_pending.push_back({phase, {e0, e1}});
  }
  return err;
}

// Level-0 pass through the tile kernel when it applies, else the slab kernel.
hipError_t run_fine(mgrit_handle *h, int phase, int mode, const double *cin, double *cout, double *r, double *out) {
  const Level &L0 = h->lv[0];
  const int64_t nc = L0.nt / L0.m;
  if (!L0.tiles) return run_pass(h, L0, phase, mode, L0.m, nc, cin, cout, nullptr, r, nullptr, out, 0);
  TileArgs ta{};
  ta.mode = mode;
  ta.m = L0.m;
  ta.nint = nc;
  ta.cin = cin;
  ta.cout = cout;
  ta.r = r;
  ta.out = out;
  ta.normpart = h->normpart;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof_mask & (1u << phase)) {
    e0 = take_event(h);
    e1 = take_event(h);
    if (e0 && e1) (void)hipEventRecord(e0, h->stream);
  }
  hipError_t err = launch_tiles(L0.desc, L0.tg, ta, h->stream);
  if (e0 && e1) {
    (void)hipEventRecord(e1, h->stream);
    h->ev_pending.push_back({phase, {e0, e1}});
  }
  return err;
}

int64_t fine_norm_parts(const mgrit_handle *h) {
  const Level &L0 = h->lv[0];
  return (L0.nt / L0.m) * (L0.tiles ? L0.tg.ntiles : 1);
}

// Approximate solve of level l >= 1 with rhs g (rows 1..nt_l) and zero initial
// guess; the result is added into `parent` rows 0..nt_l (the C-points of
// level l-1).
struct PhaseRec {
  int kind;  // CP_PASS or CP_FILL
  int level;
  PassArgs pa;
};

// The coarse passes of a V-cycle below level l-1, in launch order: level l
// relaxes (F(CF)^nu, then F and the C-point residual), recurses on its
// residual, and post-relaxes into its parent's C-points; the last level is
// solved by sequential stepping (Sec. 2.2).
void vcycle_plan(mgrit_handle *h, int l, const double *g, double *parent, std::vector<PhaseRec> &out) {
  Level &L = h->lv[l];
  const int nlev = (int)h->lv.size();
  const int nx = (int)h->prob.nx;
  auto pass = [&](int mode, int m, int64_t nint, const double *cin, double *cout, double *r, double *par,
                  int zero_init) {
    PhaseRec p{CP_PASS, l, PassArgs{}};
    p.pa.mode = mode;
    p.pa.m = m;
    p.pa.zero_init = zero_init;
    p.pa.nint = nint;
    p.pa.cin = cin;
    p.pa.cout = cout;
    p.pa.g = g;
    p.pa.r = r;
    p.pa.parent = par;
    p.pa.normpart = h->normpart;
    out.push_back(p);
  };
  if (l == nlev - 1) {
    pass(MODE_SEQ, (int)L.nt, 1, nullptr, nullptr, nullptr, parent, 1);
    return;
  }
  const int64_t nc = L.nt / L.m;
  int cur = 0;
  if (h->opt.nu == 0) {
    PhaseRec f{CP_FILL, l, PassArgs{}};
    f.pa.cout = L.c[0];
    f.pa.nint = (nc + 1) * (int64_t)nx;
    out.push_back(f);
  }
  for (int s = 0; s < h->opt.nu; ++s) {
    pass(MODE_PASS_A, L.m, nc, s == 0 ? nullptr : L.c[cur], L.c[1 - cur], nullptr, nullptr, s == 0);
    cur = 1 - cur;
  }
  pass(MODE_PASS_B, L.m, nc, L.c[cur], nullptr, L.r, nullptr, 0);
  vcycle_plan(h, l + 1, L.r, L.c[cur], out);
  pass(MODE_POST_F, L.m, nc, L.c[cur], nullptr, nullptr, parent, 0);
}

// Queue the coarse-grid correction of one iteration: one persistent launch
// when it applies, else one launch per pass.
mgrit_status vcycle(mgrit_handle *h, const double *g, double *parent) {
  std::vector<PhaseRec> ph;
  vcycle_plan(h, 1, g, parent, ph);
  if (h->cv_ok && (int)ph.size() <= MAX_COARSE_PHASES) {
    CoarsePlan plan{};
    plan.nphases = (int)ph.size();
    plan.nlevels = (int)h->lv.size() - 1;
    for (int l = 1; l < (int)h->lv.size(); ++l) plan.desc[l - 1] = h->lv[l].desc;
    for (size_t i = 0; i < ph.size(); ++i) plan.ph[i] = CoarsePhase{ph[i].kind, ph[i].level - 1, ph[i].pa};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->prof_mask & (1u << MGRIT_PROF_COARSE)) {
      e0 = take_event(h);
      e1 = take_event(h);
      if (e0 && e1) (void)hipEventRecord(e0, h->stream);
    }
    const hipError_t e = launch_coarse_vcycle(plan, h->lv[1].op, h->lv[1].lay, h->cv_grid, h->cv_lds, h->gsync,
                                              h->guard, h->stream);
    if (e0 && e1) {
      (void)hipEventRecord(e1, h->stream);
      h->ev_pending.push_back({MGRIT_PROF_COARSE, {e0, e1}});
    }
    if (e == hipSuccess) return MGRIT_OK;
    // the launch was refused: fall back to one launch per pass
    (void)hipGetLastError();
    h->cv_ok = false;
  }
  for (const PhaseRec &p : ph) {
    const Level &L = h->lv[p.level];
    if (p.kind == CP_FILL) {
      HIPCHK(h, launch_fill(p.pa.cout, p.pa.nint, 0.0, h->stream, h->guard));
    } else {
      HIPCHK(h, run_pass(h, L, MGRIT_PROF_COARSE, p.pa.mode, p.pa.m, p.pa.nint, p.pa.cin, p.pa.cout, p.pa.g, p.pa.r,
                         p.pa.parent, nullptr, p.pa.zero_init));
    }
  }
  return MGRIT_OK;
}

// One MGRIT iteration of the solve in progress: level-0 relaxation (F(CF)^nu
// then F and the C-point residual), the norm and stopping test on the
// device (its state also lands in pinned host memory, with an event behind
// it), and the coarse-grid correction, queued before the decision is known
// and skipping itself once a stop is recorded.
mgrit_status queue_iteration(mgrit_handle *h) {
  auto &ss = h->ss;
  Level &L0 = h->lv[0];
  const StopRule rule{h->opt.rtol, h->opt.diverge_factor, h->opt.max_iter, 0.0};
  for (int s = 0; s < h->opt.nu; ++s) {
    HIPCHK(h, run_fine(h, MGRIT_PROF_FINE_RELAX, MODE_PASS_A, L0.c[ss.cur], L0.c[1 - ss.cur], nullptr, nullptr));
    ss.cur = 1 - ss.cur;
  }
  HIPCHK(h, run_fine(h, MGRIT_PROF_FINE_RELAX, MODE_PASS_B, L0.c[ss.cur], nullptr, L0.r, nullptr));
  HIPCHK(h, launch_solve_ctl(h->normpart, fine_norm_parts(h), h->ctl, h->ctl_host_dev, h->gsync, rule, h->stream));
  if (h->noalloc) {
    // the state the host reads once the correction below has been queued
    HIPCHK(h, hipMemcpyAsync(&h->ctl_local, h->ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, h->stream));
  } else {
    HIPCHK(h, hipEventRecord(h->ctl_ev, h->stream));
  }
  h->guard = &h->ctl->stop;
  const mgrit_status st = vcycle(h, L0.r, L0.c[ss.cur]);
  h->guard = nullptr;
  return st;
}

// Read the stopping decision of the last queued iteration (its event has
// completed); on a stop, queue the outputs and mark the solve finished.
mgrit_status take_decision(mgrit_handle *h) {
  auto &ss = h->ss;
  Level &L0 = h->lv[0];
  const int nx = (int)h->prob.nx;
  const int64_t nc = L0.nt / L0.m;
  ss.prev = ss.hc.rho;
  ss.hc = *h->ctl_host;
  ss.hist.push_back(ss.hc.rho);
  if (ss.hc.stop == STOP_NONE) return MGRIT_OK;
  ss.finished = true;
  switch (ss.hc.stop) {
    case STOP_NONFINITE: ss.status = fail(h, MGRIT_EDIVERGED, "non-finite residual"); break;
    case STOP_MAX_ITER:
      ss.status = MGRIT_ENOTCONVERGED;
      h->err = "max_iter reached";
      break;
    case STOP_DIVERGED: ss.status = fail(h, MGRIT_EDIVERGED, "residual grew past diverge_factor * res0"); break;
    case STOP_DEVICE:
      // a persistent launch gave up waiting at a grid barrier: reset the
      // barrier state so that later solves start clean; no outputs
      (void)hipStreamSynchronize(h->stream);
      (void)hipMemset(h->gsync, 0, sizeof(GridSync));
      ss.status = fail(h, MGRIT_EDEVICE, "coarse-level grid barrier timed out");
      return MGRIT_OK;
    default: break;
  }
  if (ss.u_out) HIPCHK(h, run_fine(h, MGRIT_PROF_FINAL, MODE_FINAL_F, L0.c[ss.cur], nullptr, nullptr, ss.u_out));
  if (ss.u_final)
    HIPCHK(h, hipMemcpyAsync(ss.u_final, L0.c[ss.cur] + nc * (int64_t)nx, nx * sizeof(double),
                             hipMemcpyDeviceToDevice, h->stream));
  return MGRIT_OK;
}

double reduce_norm(mgrit_handle *h, int64_t n, hipError_t &e) {
  e = launch_reduce(h->normpart, n, h->normsum, h->stream);
  if (e) return NAN;
  e = hipMemcpyAsync(h->normsum_host, h->normsum, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e) return NAN;
  e = hipStreamSynchronize(h->stream);
  if (e) return NAN;
  harvest_events(h);
  return std::sqrt(*h->normsum_host);
}

// ---------------------------------------------------------------------------
// Mixed precision: float32 MGRIT on the correction equation A e = r inside a
// float64 refinement loop (see mgrit_precision).
// ---------------------------------------------------------------------------
hipError_t run_pass32(mgrit_handle *h, const Level &L, int phase, int mode, int m, int64_t nint, const float *cin,
                      float *cout, const float *g, float *r, float *parent, float *out, int zero_init) {
  PassArgs32 pa{};
  pa.mode = mode;
  pa.m = m;
  pa.zero_init = zero_init;
  pa.nint = nint;
  pa.cin = cin;
  pa.cout = cout;
  pa.g = g;
  pa.r = r;
  pa.parent = parent;
  pa.out = out;
  pa.normpart = h->normpart;
  pa.stop = h->guard;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof_mask & (1u << phase)) {
    e0 = take_event(h);
    e1 = take_event(h);
    if (e0 && e1) (void)hipEventRecord(e0, h->stream);
  }
  hipError_t err = launch_pass32(L.desc32, L.op, L.lay, pa, h->stream);
  if (e0 && e1) {
    (void)hipEventRecord(e1, h->stream);
    h->ev_pending.push_back({phase, {e0, e1}});
  }
  return err;
}

// Level-0 float32 pass (inner solves of mixed precision) through the tile
// kernel when the float64 passes use it, else the slab kernel; g: the inner
// right-hand side at every point.
hipError_t run_fine32(mgrit_handle *h, int phase, int mode, const float *cin, float *cout, const float *g, float *r,
                      float *out) {
  const Level &L0 = h->lv[0];
  const int64_t nc = L0.nt / L0.m;
  if (!L0.tiles) return run_pass32(h, L0, phase, mode, L0.m, nc, cin, cout, g, r, nullptr, out, 0);
  TileArgs32 ta{};
  ta.mode = mode;
  ta.m = L0.m;
  ta.nint = nc;
  ta.cin = cin;
  ta.cout = cout;
  ta.r = r;
  ta.out = out;
  ta.g = g;
  ta.normpart = h->normpart;
  ta.stop = h->guard;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof_mask & (1u << phase)) {
    e0 = take_event(h);
    e1 = take_event(h);
    if (e0 && e1) (void)hipEventRecord(e0, h->stream);
  }
  hipError_t err = launch_tiles32(L0.desc, L0.tg, ta, h->stream);
  if (e0 && e1) {
    (void)hipEventRecord(e1, h->stream);
    h->ev_pending.push_back({phase, {e0, e1}});
  }
  return err;
}

// The float32 coarse-grid correction below level l-1: the passes of
// vcycle_plan, one launch each.
mgrit_status vcycle32(mgrit_handle *h, int l, const float *g, float *parent) {
  Level &L = h->lv[l];
  const int nlev = (int)h->lv.size();
  const int nx = (int)h->prob.nx;
  const int ph = MGRIT_PROF_COARSE;
  if (l == nlev - 1) {
    HIPCHK(h, run_pass32(h, L, ph, MODE_SEQ, (int)L.nt, 1, nullptr, nullptr, g, nullptr, parent, nullptr, 1));
    return MGRIT_OK;
  }
  const int64_t nc = L.nt / L.m;
  int cur = 0;
  if (h->opt.nu == 0) HIPCHK(h, launch_fill32(L.c32[0], (nc + 1) * (int64_t)nx, h->stream, h->guard));
  for (int s = 0; s < h->opt.nu; ++s) {
    HIPCHK(h, run_pass32(h, L, ph, MODE_PASS_A, L.m, nc, s == 0 ? nullptr : L.c32[cur], L.c32[1 - cur], g, nullptr,
                         nullptr, nullptr, s == 0));
    cur = 1 - cur;
  }
  HIPCHK(h, run_pass32(h, L, ph, MODE_PASS_B, L.m, nc, L.c32[cur], nullptr, g, L.r32, nullptr, nullptr, 0));
  const mgrit_status st = vcycle32(h, l + 1, L.r32, L.c32[cur]);
  if (st != MGRIT_OK) return st;
  HIPCHK(h, run_pass32(h, L, ph, MODE_POST_F, L.m, nc, L.c32[cur], nullptr, g, nullptr, parent, nullptr, 0));
  return MGRIT_OK;
}

// Float32 MGRIT for A e = g32 (rows 1..nt), e_0 = 0, zero initial iterate,
// until the C-point residual falls by inner_rtol (or inner_max_iter); every
// row of e lands in e32.  Queued behind the outer stopping decision: every
// launch skips itself once *gate (the outer stop flag) is set, which the
// inner state reports as STOP_OUTER.  Returns the iterations performed in
// *iters and the inner stop code in *stop.
// Mixed precision in steps (mgrit_solve and mgrit_solve_start/_advance/
// _finish): an outer step queues the float64 residual with its norm and
// stopping test, then the float32 inner solve of A e = r from zero, one
// iteration at a time (each skips itself once the inner state, or the outer
// one through the gate, has stopped); the host reads each inner decision
// from pinned memory behind an event while the correction runs.  When the
// inner solve stops, its final F-pass writes e, the host reads the outer
// decision (current by then) and either finishes or queues u += e and the
// next outer step.
mgrit_status mp_queue_inner_iteration(mgrit_handle *h) {
  auto &ss = h->ss;
  Level &L0 = h->lv[0];
  const StopRule rule{h->opt.inner_rtol, h->opt.diverge_factor, h->opt.inner_max_iter, 0.5};
  h->guard = &h->ctl->stop;
  for (int s = 0; s < h->opt.nu; ++s) {
    HIPCHK(h, run_fine32(h, MGRIT_PROF_FINE_RELAX, MODE_PASS_A, L0.c32[ss.icur], L0.c32[1 - ss.icur], h->g32, nullptr,
                         nullptr));
    ss.icur = 1 - ss.icur;
  }
  HIPCHK(h, run_fine32(h, MGRIT_PROF_FINE_RELAX, MODE_PASS_B, L0.c32[ss.icur], nullptr, h->g32, L0.r32, nullptr));
  HIPCHK(h, launch_solve_ctl(h->normpart, fine_norm_parts(h), h->ctl, h->ctl_host_dev, nullptr, rule, h->stream));
  HIPCHK(h, hipEventRecord(h->ctl_ev, h->stream));
  const mgrit_status st = vcycle32(h, 1, L0.r32, L0.c32[ss.icur]);
  h->guard = nullptr;
  return st;
}

// the outer step: float64 r = g - A u at every time point (written rounded
// to float32 as the inner right-hand side), its norm and the test; then the
// inner solve's start
mgrit_status mp_queue_outer(mgrit_handle *h) {
  auto &ss = h->ss;
  Level &L0 = h->lv[0];
  const int nx = (int)h->prob.nx;
  const int64_t nt = h->prob.nt;
  const int64_t nc = L0.nt / L0.m;
  const StopRule orule{h->opt.rtol, h->opt.diverge_factor, h->opt.max_iter, 0.0};
  HIPCHK(h, run_pass(h, L0, MGRIT_PROF_RESIDUAL, MODE_RESID, ss.rk, nt / ss.rk, ss.U, nullptr, nullptr, nullptr,
                     nullptr, nullptr, 0, h->g32));
  HIPCHK(h, launch_solve_ctl(h->normpart, nt / ss.rk, h->octl, h->octl_host_dev, nullptr, orule, h->stream));
  const int *ostop = &h->octl->stop;
  HIPCHK(h, launch_ctl_reset(h->ctl, ostop, h->stream));
  ss.icur = 0;
  HIPCHK(h, launch_fill32(L0.c32[0], (nc + 1) * (int64_t)nx, h->stream, &h->ctl->stop));
  return mp_queue_inner_iteration(h);
}

mgrit_status mp_start(mgrit_handle *h, const double *u0, const double *v_init, double *u_out, double *u_final) {
  auto &ss = h->ss;
  ss = {};
  ss.t0 = std::chrono::steady_clock::now();
  ss.mixed = true;
  ss.u_out = u_out;
  ss.u_final = u_final;
  ss.hc.rho = NAN;
  const int nx = (int)h->prob.nx;
  const int64_t nt = h->prob.nt;
  const int64_t pts = nt * nx;
  ss.U = u_out ? u_out : h->u64;
  // outer iterate: v_init (or the seeded U[0,1), or zero) with row 0 = u0
  if (v_init && v_init != ss.U) {
    HIPCHK(h, hipMemcpyAsync(ss.U, v_init, (pts + nx) * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  } else if (!v_init && h->opt.init_seed) {
    HIPCHK(h, launch_splitmix_rows(ss.U + nx, nt, 1, 1, nx, h->opt.init_seed, h->stream));
  } else if (!v_init) {
    HIPCHK(h, launch_fill(ss.U, pts + nx, 0.0, h->stream));
  }
  HIPCHK(h, hipMemcpyAsync(ss.U, u0, nx * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  // each residual workgroup takes rk consecutive time points, so that every
  // row of the iterate is read once (plus one row per workgroup), while
  // keeping at least 1024 workgroups (four per CU)
  ss.rk = 1;
  for (int k : {16, 8, 4, 2})
    if (nt % k == 0 && nt / k >= 1024) {
      ss.rk = k;
      break;
    }
  HIPCHK(h, hipMemsetAsync(h->octl, 0, sizeof(SolveCtl), h->stream));
  ss.active = true;
  const mgrit_status st = mp_queue_outer(h);
  if (st != MGRIT_OK) ss.active = false;
  return st;
}

// The inner decision of the last queued iteration (its event has completed).
mgrit_status mp_take_decision(mgrit_handle *h) {
  auto &ss = h->ss;
  Level &L0 = h->lv[0];
  const int nx = (int)h->prob.nx;
  const int64_t nt = h->prob.nt;
  const SolveCtl ic = *h->ctl_host;
  if (ic.stop == STOP_NONE) return mp_queue_inner_iteration(h);
  // the inner solve has stopped: its final F-pass writes e at every point
  // (skipped after an outer stop)
  const int *ostop = &h->octl->stop;
  h->guard = ostop;
  HIPCHK(h, run_fine32(h, MGRIT_PROF_FINAL, MODE_FINAL_F, L0.c32[ss.icur], nullptr, h->g32, nullptr, h->e32));
  h->guard = nullptr;
  // the outer state in pinned memory is current: the inner decisions came
  // after it
  const SolveCtl oc = *h->octl_host;
  ss.prev = ss.hc.rho;
  ss.hc = oc;
  ss.hist.push_back(oc.rho);
  if (oc.stop != STOP_NONE) {
    ss.finished = true;
    if (oc.stop == STOP_NONFINITE) ss.status = fail(h, MGRIT_EDIVERGED, "non-finite residual");
    if (oc.stop == STOP_MAX_ITER) {
      ss.status = MGRIT_ENOTCONVERGED;
      h->err = "max_iter reached";
    }
    if (oc.stop == STOP_DIVERGED) ss.status = fail(h, MGRIT_EDIVERGED, "residual grew past diverge_factor * res0");
    if (ss.u_final)
      HIPCHK(h, hipMemcpyAsync(ss.u_final, ss.U + nt * (int64_t)nx, nx * sizeof(double), hipMemcpyDeviceToDevice,
                               h->stream));
    return MGRIT_OK;
  }
  ss.inner_total += ic.it;
  if (ic.stop == STOP_NONFINITE || ic.stop == STOP_DIVERGED) {
    ss.finished = true;
    ss.status = fail(h, MGRIT_EDIVERGED, "the float32 inner solve diverged");
    return MGRIT_OK;
  }
  HIPCHK(h, launch_add32(ss.U, h->e32, nt * (int64_t)nx + nx, h->stream, ostop));
  ++ss.outer;
  return mp_queue_outer(h);
}

}  // namespace

extern "C" {

mgrit_status mgrit_solve_start(mgrit_handle *h, const double *u0, const double *v_init, double *u_out,
                               double *u_final) {
  if (!h) return MGRIT_EINVAL;
  if (!u0) return fail(h, MGRIT_EINVAL, "u0 is required");
  if (h->ss.active) return fail(h, MGRIT_EINVAL, "a solve is already in progress on this handle");
  if (h->opt.precision == MGRIT_PREC_MIXED) return mp_start(h, u0, v_init, u_out, u_final);
  auto &ss = h->ss;
  ss = {};
  ss.t0 = std::chrono::steady_clock::now();
  ss.u_out = u_out;
  ss.u_final = u_final;
  ss.hc.rho = NAN;
  Level &L0 = h->lv[0];
  const int nx = (int)h->prob.nx;
  const int64_t nc = L0.nt / L0.m;
  // initial C-points: v_init's, seeded U[0,1), or zero
  if (v_init) {
    HIPCHK(h, launch_gather_rows(v_init, L0.m, L0.c[0], nc + 1, nx, h->stream));
  } else if (h->opt.init_seed) {
    HIPCHK(h, launch_splitmix_rows(L0.c[0] + nx, nc, L0.m, L0.m, nx, h->opt.init_seed, h->stream));
  } else {
    HIPCHK(h, launch_fill(L0.c[0], (nc + 1) * (int64_t)nx, 0.0, h->stream));
  }
  HIPCHK(h, hipMemcpyAsync(L0.c[0], u0, nx * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipMemsetAsync(h->ctl, 0, sizeof(SolveCtl), h->stream));
  ss.active = true;
  const mgrit_status st = queue_iteration(h);
  if (st != MGRIT_OK) ss.active = false;
  return st;
}

mgrit_status mgrit_solve_advance(mgrit_handle *h, int32_t *done) {
  if (!h || !done) return MGRIT_EINVAL;
  auto &ss = h->ss;
  if (!ss.active) return fail(h, MGRIT_EINVAL, "no solve in progress");
  *done = 0;
  if (ss.finished) {
    *done = 1;
    return MGRIT_OK;
  }
  const hipError_t q = hipEventQuery(h->ctl_ev);
  if (q == hipErrorNotReady) return MGRIT_OK;
  if (q != hipSuccess) return hipfail(h, q, "stopping-test event");
  if (ss.mixed) {
    const mgrit_status st = mp_take_decision(h);
    if (st != MGRIT_OK) return st;
    *done = ss.finished ? 1 : 0;
    return MGRIT_OK;
  }
  const mgrit_status st = take_decision(h);
  if (st != MGRIT_OK) return st;
  if (ss.finished) {
    *done = 1;
    return MGRIT_OK;
  }
  return queue_iteration(h);
}

mgrit_status mgrit_solve_finish(mgrit_handle *h, mgrit_stats *stats) {
  if (!h) return MGRIT_EINVAL;
  auto &ss = h->ss;
  if (!ss.active) return fail(h, MGRIT_EINVAL, "no solve in progress");
  while (!ss.finished) {
    HIPCHK(h, hipEventSynchronize(h->ctl_ev));
    int32_t done = 0;
    const mgrit_status st = mgrit_solve_advance(h, &done);
    if (st != MGRIT_OK) {
      (void)hipStreamSynchronize(h->stream);
      ss.active = false;
      return st;
    }
  }
  ss.active = false;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_events(h);
  if (stats) {
    const auto &hc = ss.hc;
    stats->iterations = ss.mixed ? ss.outer : hc.it;
    stats->inner_iterations = ss.mixed ? ss.inner_total : 0;
    stats->res0 = hc.res0;
    stats->res_final = hc.rho;
    stats->conv_factor = ss.prev > 0 ? hc.rho / ss.prev : NAN;
    const int len = (int)ss.hist.size();
    if (stats->res_history)
      for (int i = 0; i < std::min(len, stats->res_history_cap); ++i) stats->res_history[i] = ss.hist[i];
    stats->res_history_len = std::min(len, std::max(stats->res_history_cap, 0));
    stats->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - ss.t0).count();
  }
  return ss.status;
}

mgrit_status mgrit_solve(mgrit_handle *h, const double *u0, const double *v_init, double *u_out, double *u_final,
                         mgrit_stats *stats) {
  const mgrit_status st = mgrit_solve_start(h, u0, v_init, u_out, u_final);
  if (st != MGRIT_OK) return st;
  return mgrit_solve_finish(h, stats);
}

mgrit_status mgrit_workspace_bytes(const mgrit_problem *P, const mgrit_options *O, uint64_t *bytes) {
  if (!P || !O || !bytes) return MGRIT_EINVAL;
  std::vector<int64_t> nts;
  std::vector<int> ms;
  std::string err;
  if (P->nx < 1 || P->nt < 1 || O->max_levels < 2 || O->max_levels > MGRIT_MAX_LEVELS ||
      !level_hierarchy(*P, *O, nts, ms, err))
    return MGRIT_EINVAL;
  uint64_t n = 0;
  for (size_t l = 0; l + 1 < nts.size(); ++l) {
    const uint64_t nc = (uint64_t)(nts[l] / ms[l]);
    n += (2 * (nc + 1) + nc) * (uint64_t)P->nx;  // two C-point arrays and the residual
  }
  n += (uint64_t)std::max<int64_t>(P->nt, 1) * 64;  // norm partials (bound)
  // per level: scan tables, descriptor and the alignment of five pieces;
  // once: the grid-barrier state and the alignment of the norm pieces
  *bytes = n * sizeof(double) +
           (uint64_t)nts.size() * (2 * RTAB_ALL * KMAX * KMAX * sizeof(double) + sizeof(LevelDesc) + 5 * 256) +
           sizeof(GridSync) + 4 * 256 + sizeof(SolveCtl);
  if (O->coarse_solve == 1) {  // GMRES bases: (gmres_max + 1) vectors per interval of each coarse level
    for (size_t l = 1; l < nts.size(); ++l) {
      const uint64_t cap = (l + 1 < nts.size()) ? (uint64_t)(nts[l] / ms[l]) : 1;
      *bytes += cap * (uint64_t)(std::max(O->gmres_max_iter, 1) + 1) * (uint64_t)P->nx * sizeof(double) + 256;
    }
  }
  if (O->precision == MGRIT_PREC_MIXED) {
    // float32 copies of the level arrays and tables, the inner right-hand
    // side and solution (float32), the outer iterate (float64)
    uint64_t n32 = 0;
    for (size_t l = 0; l + 1 < nts.size(); ++l) {
      const uint64_t nc = (uint64_t)(nts[l] / ms[l]);
      n32 += (2 * (nc + 1) + nc) * (uint64_t)P->nx;
    }
    const uint64_t pts = (uint64_t)P->nt * (uint64_t)P->nx;
    *bytes += n32 * sizeof(float) + (2 * pts + P->nx) * sizeof(float) + (pts + P->nx) * sizeof(double) +
              (uint64_t)nts.size() * (2 * RTAB_ALL * KMAX * KMAX * sizeof(float) + sizeof(LevelDesc) + 5 * 256) +
              4 * 256;
  }
  return MGRIT_OK;
}

mgrit_status mgrit_residual(mgrit_handle *h, const double *u, double *r, double *norm2) {
  if (!h || !u) return MGRIT_EINVAL;
  const Level &L0 = h->lv[0];
  HIPCHK(h, run_pass(h, L0, MGRIT_PROF_RESIDUAL, MODE_RESID, 1, h->prob.nt, u, nullptr, nullptr, r, nullptr, nullptr, 0));
  hipError_t e;
  const double n = reduce_norm(h, h->prob.nt, e);
  if (e) return hipfail(h, e, "residual norm");
  if (norm2) *norm2 = n;
  return MGRIT_OK;
}

mgrit_status mgrit_sequential(mgrit_handle *h, const double *u0, double *u_out) {
  if (!h || !u0 || !u_out) return MGRIT_EINVAL;
  const Level &L0 = h->lv[0];
  if (L0.seq_tiles) {
    // blocks of seq_T steps, each launch reading the row the previous wrote
    const int64_t nx = h->prob.nx, nt = h->prob.nt;
    HIPCHK(h, hipMemcpyAsync(u_out, u0, nx * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    for (int64_t k = 0; k < nt; k += L0.seq_T) {
      TileArgs ta{};
      ta.mode = MODE_SEQ;
      ta.m = (int)std::min<int64_t>(L0.seq_T, nt - k);
      ta.nint = 1;
      ta.cin = u_out + k * nx;
      ta.out = u_out + k * nx;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (h->prof_mask & (1u << MGRIT_PROF_SEQUENTIAL)) {
        e0 = take_event(h);
        e1 = take_event(h);
        if (e0 && e1) (void)hipEventRecord(e0, h->stream);
      }
      HIPCHK(h, launch_tiles(L0.desc, L0.seq_tg, ta, h->stream));
      if (e0 && e1) {
        (void)hipEventRecord(e1, h->stream);
        h->ev_pending.push_back({MGRIT_PROF_SEQUENTIAL, {e0, e1}});
      }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    harvest_events(h);
    return MGRIT_OK;
  }
  HIPCHK(h, run_pass(h, L0, MGRIT_PROF_SEQUENTIAL, MODE_SEQ, (int)h->prob.nt, 1, u0, nullptr, nullptr, nullptr, nullptr, u_out, 0));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_events(h);
  return MGRIT_OK;
}

mgrit_status mgrit_apply_step(mgrit_handle *h, int32_t level, const double *v_in, double *v_out, int64_t count,
                              int32_t nsteps) {
  if (!h || level < 0 || level >= (int32_t)h->lv.size() || !v_in || !v_out || count < 0 || nsteps < 0)
    return fail(h, MGRIT_EINVAL, "bad apply_step arguments");
  if (count == 0) return MGRIT_OK;
  const Level &L = h->lv[level];
  HIPCHK(h, run_pass(h, L, MGRIT_PROF_OTHER, MODE_APPLY, nsteps, count, v_in, v_out, nullptr, nullptr, nullptr, nullptr, 0));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_events(h);
  return MGRIT_OK;
}

mgrit_status mgrit_profile_enable(mgrit_handle *h, uint32_t mask) {
  if (!h) return MGRIT_EINVAL;
  h->prof_mask = mask;
  return MGRIT_OK;
}

mgrit_status mgrit_profile_read(mgrit_handle *h, mgrit_profile *out, int32_t reset) {
  if (!h || !out) return MGRIT_EINVAL;
  if (hipError_t e = hipStreamSynchronize(h->stream)) return hipfail(h, e, "profile sync");
  harvest_events(h);
  *out = h->prof;
  if (reset) h->prof = mgrit_profile{};
  return MGRIT_OK;
}

mgrit_status mgrit_lfa_rho(const mgrit_problem *P, const mgrit_options *O, double *rho) {
  if (!P || !O || !rho) return MGRIT_EINVAL;
  FineInfo fi;
  std::string err;
  if (fine_info(*P, fi, err) != MGRIT_OK) return MGRIT_EINVAL;
  const int p = P->upwind_order, q = P->rk_order, m = O->m[0], nu = O->nu;
  if (m < 2) return MGRIT_EINVAL;
  const double c = P->cfl;
  const int sgn = ((p + 1) % 2) ? -1 : 1;
  const ld shift = (ld)c * m;
  const ld eps = shift - std::floor(shift);
  const long K = (long)std::floor(shift);
  ld phi_p, phi_q;
  if (q == p) {
    phi_p = m * ((ld)c * fi.efd + std::pow(-(ld)c, (ld)(p + 1)) * fi.erk) + sgn * f_poly(p, eps);
    phi_q = 0;
  } else {
    phi_p = m * (ld)c * fi.efd + sgn * f_poly(p, eps);
    phi_q = m * std::pow(-(ld)c, (ld)(q + 1)) * fi.erk;
  }
  if (O->cg_kind == MGRIT_CG_SL_PLAIN) phi_p = phi_q = 0;
  int sl_l = 0, sl_r = 0;
  std::vector<double> slw;
  if (O->cg_kind == MGRIT_CG_SL_CORRECTED || O->cg_kind == MGRIT_CG_SL_PLAIN) sl_weights(p, eps, sl_l, sl_r, slw);
  const int N = 1 << 11;
  std::vector<std::pair<double, double>> oms;  // (|omega|, omega)
  for (int k = 0; k < N; ++k) {
    const double om = -M_PI + 2 * M_PI * k / N;
    oms.push_back({std::fabs(om), om});
  }
  std::sort(oms.begin(), oms.end());
  double best = 0;
  for (size_t i = 11; i < oms.size(); ++i) {
    const double om = oms[i].second;
    const std::complex<double> lam = rk_R(fi.tab, -c * upwind_symbol(fi, om));
    std::complex<double> mu;
    const std::complex<double> lamm = std::pow(lam, m);
    if (O->cg_kind == MGRIT_CG_IDEAL) {
      mu = lamm;
    } else if (O->cg_kind == MGRIT_CG_REDISC) {
      mu = rk_R(fi.tab, -(c * m) * upwind_symbol(fi, om));
    } else {
      std::complex<double> S = 0;
      for (int j = -sl_l; j <= sl_r; ++j) S += slw[j + sl_l] * std::polar(1.0, (double)(j - K) * om);
      const double dp = std::pow(2 * std::cos(om) - 2, (p + 1) / 2);
      const double dq = q % 2 ? std::pow(2 * std::cos(om) - 2, (q + 1) / 2) : 0.0;
      mu = S / (1.0 - (double)phi_p * dp - (double)phi_q * dq);
    }
    const double val = std::pow(std::abs(lam), m * nu) * std::abs(lamm - mu) / (1 - std::abs(mu));
    best = std::max(best, val);
  }
  *rho = best;
  return MGRIT_OK;
}

}  // extern "C"

// ===========================================================================
// 2D extension (dimension-split reading; see mgrit.h)
// ===========================================================================
namespace {

struct Line1D {  // a 1D coarse step applied along one axis of every slab
  StepOp op{};
  Layout lay{};
  LevelDesc *desc = nullptr;    // tables in float64
  LevelDesc *desc32 = nullptr;  // tables in float32 (mixed precision)
};

struct Level2 {
  int64_t nt = 0;
  int m = 0;    // to the next level, 0 on the coarsest
  Line1D x, y;  // levels >= 1
};

// The arrays of one precision: per level the C-points (two copies, N_c + 1
// slabs each) and the C-point residual (N_c slabs); the step and transpose
// work buffers (cap slabs each) and one zero slab.
template <class T>
struct Set2 {
  std::vector<T *> c0, c1, r;
  T *w[2] = {nullptr, nullptr}, *t1 = nullptr, *t2 = nullptr, *zero = nullptr;
};

}  // namespace

struct mgrit2d_handle {
  mgrit2d_problem prob{};
  mgrit_options opt{};
  hipStream_t stream = nullptr;
  std::vector<Level2> lv;
  Step2dArgs fine{};  // fine-step constants (pointers set per launch)
  int64_t cap = 0;    // slabs each work buffer holds
  Set2<double> d64;
  Set2<float> d32;    // mixed precision only
  // mixed precision: the inner right-hand side and solution (float32), the
  // outer residual and, without u_out, the outer iterate (float64)
  float *g32 = nullptr, *e32 = nullptr;
  double *r64 = nullptr, *u64 = nullptr;
  double *normpart = nullptr, *normsum = nullptr, *normsum_host = nullptr;
  int64_t normpart_len = 0;
  char *arena = nullptr;
  std::string err;
};

namespace {

constexpr int RESID_BLOCKS = 64;  // partial sums per slab of the C-point residual

mgrit_status fail2(mgrit2d_handle *h, mgrit_status s, const std::string &msg) {
  h->err = msg;
  return s;
}

#define HIPCHK2(h, expr)                                                                   \
  do {                                                                                     \
    const hipError_t e2_ = (expr);                                                         \
    if (e2_ != hipSuccess) return fail2((h), MGRIT_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e2_)); \
  } while (0)

int64_t slab(const mgrit2d_handle *h) { return h->prob.nx * h->prob.ny; }

template <class T>
Set2<T> &set_of(mgrit2d_handle *h);
template <>
Set2<double> &set_of<double>(mgrit2d_handle *h) { return h->d64; }
template <>
Set2<float> &set_of<float>(mgrit2d_handle *h) { return h->d32; }

hipError_t line_apply(const Line1D &ln, const double *src, double *dst, int64_t count, hipStream_t stream) {
  PassArgs pa{};
  pa.mode = MODE_APPLY;
  pa.m = 1;
  pa.nint = count;
  pa.cin = src;
  pa.cout = dst;
  return launch_pass(ln.desc, ln.op, ln.lay, pa, stream);
}

hipError_t line_apply(const Line1D &ln, const float *src, float *dst, int64_t count, hipStream_t stream) {
  PassArgs32 pa{};
  pa.mode = MODE_APPLY;
  pa.m = 1;
  pa.nint = count;
  pa.cin = src;
  pa.cout = dst;
  return launch_pass32(ln.desc32, ln.op, ln.lay, pa, stream);
}

// dst = Phi_l(src) + g_scale g on nb slabs (src and dst with slab strides;
// levels >= 1 need contiguous src and dst)
template <class T>
hipError_t apply2d(mgrit2d_handle *h, int l, const T *src, int64_t src_stride, T *dst, int64_t dst_stride, int64_t nb,
                   const T *g, int64_t g_stride, double g_scale = 1.0) {
  const int nx = (int)h->prob.nx, ny = (int)h->prob.ny;
  const int64_t S = slab(h);
  if (l == 0) {
    const Step2dArgs &f = h->fine;
    Step2dArgsT<T> a{};
    a.src = src;
    a.src_stride = src_stride;
    a.dst = dst;
    a.dst_stride = dst_stride;
    a.g = g;
    a.g_stride = g_stride;
    a.g_scale = g_scale;
    a.nb = nb;
    a.nx = f.nx;
    a.ny = f.ny;
    a.ncoef = f.ncoef;
    for (int i = 0; i < MAXCOEF; ++i) a.coef[i] = f.coef[i];
    a.sl = f.sl;
    a.sr = f.sr;
    for (int i = 0; i < MAXTAPS; ++i) {
      a.tx[i] = f.tx[i];
      a.ty[i] = f.ty[i];
    }
    a.use_reg = f.use_reg;
    return launch_step2d<T>(a, h->stream);
  }
  const Level2 &L = h->lv[l];
  Set2<T> &B = set_of<T>(h);
  // along x: every row of every slab is one 1D vector
  if (hipError_t e = line_apply(L.x, src, B.t1, nb * ny, h->stream)) return e;
  if (hipError_t e = launch_transpose<T>(B.t1, S, B.t2, S, (const T *)nullptr, 0, nb, ny, nx, h->stream)) return e;
  // along y: the rows of the transposed slabs, in place
  if (hipError_t e = line_apply(L.y, B.t2, B.t2, nb * nx, h->stream)) return e;
  return launch_transpose<T>(B.t2, S, dst, S, g, g_stride, nb, nx, ny, h->stream);
}

// One relaxation pass (PassMode) of level l over all its CF-intervals at
// once: the intervals' vectors advance together, one step per launch group.
// g: right-hand side rows g[n-1] for level point n (NULL = 0).
template <class T>
mgrit_status relax2d(mgrit2d_handle *h, int l, int mode, const T *cin, T *cout, const T *g, T *r, T *parent,
                     T *out) {
  const Level2 &L = h->lv[l];
  Set2<T> &B = set_of<T>(h);
  const int64_t S = slab(h);
  const int m = L.m;
  const int64_t nc = L.nt / m;
  const int nsteps = (mode == MODE_POST_F || mode == MODE_FINAL_F) ? m - 1 : m;
  if (mode == MODE_POST_F) HIPCHK2(h, launch_slab_axpy<T>(parent, m * S, cin, S, nc, S, true, h->stream));
  if (mode == MODE_FINAL_F) HIPCHK2(h, launch_slab_axpy<T>(out, m * S, cin, S, nc, S, false, h->stream));
  const T *src = cin;
  for (int j = 1; j <= nsteps; ++j) {
    T *dst = B.w[j & 1];
    HIPCHK2(h, apply2d<T>(h, l, src, S, dst, S, nc, g ? g + (j - 1) * S : nullptr, m * S));
    if (mode == MODE_POST_F) HIPCHK2(h, launch_slab_axpy<T>(parent + j * S, m * S, dst, S, nc, S, true, h->stream));
    if (mode == MODE_FINAL_F) HIPCHK2(h, launch_slab_axpy<T>(out + j * S, m * S, dst, S, nc, S, false, h->stream));
    src = dst;
  }
  if (mode == MODE_PASS_A) {
    if (cout != cin) HIPCHK2(h, launch_slab_axpy<T>(cout, S, cin, S, 1, S, false, h->stream));
    HIPCHK2(h, launch_slab_axpy<T>(cout + S, S, src, S, nc, S, false, h->stream));
  } else if (mode == MODE_PASS_B) {
    HIPCHK2(h, launch_slab_resid<T>(src, cin + S, r, nc, S, RESID_BLOCKS, h->normpart, h->stream));
  } else if (mode == MODE_POST_F) {
    HIPCHK2(h, launch_slab_axpy<T>(parent + nc * m * S, S, cin + nc * S, S, 1, S, true, h->stream));
  } else if (mode == MODE_FINAL_F) {
    HIPCHK2(h, launch_slab_axpy<T>(out + nc * m * S, S, cin + nc * S, S, 1, S, false, h->stream));
  }
  return MGRIT_OK;
}

// Coarse-grid correction below level l-1 (Sec. 2.2, V-cycle): relax level l
// from zero with right-hand side g, recurse on its residual, post-relax into
// the parent's C-points; the last level is solved by sequential stepping.
template <class T>
mgrit_status vcycle2d(mgrit2d_handle *h, int l, const T *g, T *parent) {
  Level2 &L = h->lv[l];
  Set2<T> &B = set_of<T>(h);
  const int64_t S = slab(h);
  const int nlev = (int)h->lv.size();
  if (l == nlev - 1) {
    const T *src = B.zero;
    for (int64_t j = 1; j <= L.nt; ++j) {
      T *dst = B.w[j & 1];
      HIPCHK2(h, apply2d<T>(h, l, src, S, dst, S, 1, g + (j - 1) * S, S));
      HIPCHK2(h, launch_slab_axpy<T>(parent + j * S, S, dst, S, 1, S, true, h->stream));
      src = dst;
    }
    return MGRIT_OK;
  }
  const int64_t nc = L.nt / L.m;
  T *c[2] = {B.c0[l], B.c1[l]};
  int cur = 0;
  HIPCHK2(h, launch_slab_axpy<T>(c[0], S, B.zero, 0, nc + 1, S, false, h->stream));  // zero C-points
  for (int s = 0; s < h->opt.nu; ++s) {
    const mgrit_status st = relax2d<T>(h, l, MODE_PASS_A, c[cur], c[1 - cur], g, nullptr, nullptr, nullptr);
    if (st != MGRIT_OK) return st;
    cur = 1 - cur;
  }
  mgrit_status st = relax2d<T>(h, l, MODE_PASS_B, c[cur], nullptr, g, B.r[l], nullptr, nullptr);
  if (st != MGRIT_OK) return st;
  st = vcycle2d<T>(h, l + 1, B.r[l], c[cur]);
  if (st != MGRIT_OK) return st;
  return relax2d<T>(h, l, MODE_POST_F, c[cur], nullptr, g, nullptr, parent, nullptr);
}

double norm2d(mgrit2d_handle *h, int64_t parts, hipError_t &e) {
  e = launch_reduce(h->normpart, parts, h->normsum, h->stream);
  if (!e) e = hipMemcpyAsync(h->normsum_host, h->normsum, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (!e) e = hipStreamSynchronize(h->stream);
  return e ? NAN : std::sqrt(*h->normsum_host);
}

// MGRIT at level 0 with right-hand side g (NULL: the homogeneous system with
// u_0 = the C-point row 0 already in c0[0]), from the C-points in c0[0];
// stops as rule says; the final C-points are in *cfinal.  Float64 solves
// record the residual history.
template <class T>
mgrit_status mgrit2d_iterate(mgrit2d_handle *h, const T *g, const StopRule &rule, int *iters, int *stop, T **cfinal,
                             std::vector<double> *hist, double *res0_out, double *rho_out, double *prev_out) {
  Level2 &L0 = h->lv[0];
  Set2<T> &B = set_of<T>(h);
  const int m = L0.m;
  const int64_t nc = L0.nt / m;
  T *c[2] = {B.c0[0], B.c1[0]};
  int cur = 0, it = 0;
  double res0 = NAN, rho = NAN, prev = NAN;
  for (;;) {
    for (int s = 0; s < h->opt.nu; ++s) {
      const mgrit_status st = relax2d<T>(h, 0, MODE_PASS_A, c[cur], c[1 - cur], g, nullptr, nullptr, nullptr);
      if (st != MGRIT_OK) return st;
      cur = 1 - cur;
    }
    mgrit_status st = relax2d<T>(h, 0, MODE_PASS_B, c[cur], nullptr, g, B.r[0], nullptr, nullptr);
    if (st != MGRIT_OK) return st;
    hipError_t e;
    prev = rho;
    rho = norm2d(h, nc * RESID_BLOCKS, e);
    if (e) return fail2(h, MGRIT_EDEVICE, std::string("residual norm: ") + hipGetErrorString(e));
    if (hist) hist->push_back(rho);
    if (it == 0) res0 = rho;
    int code = STOP_NONE;
    if (!std::isfinite(rho))
      code = STOP_NONFINITE;
    else if (rho <= rule.rtol * res0)
      code = STOP_CONVERGED;
    else if (rule.stall > 0 && it >= 1 && rho > rule.stall * prev)
      code = STOP_STALLED;
    else if (it >= rule.max_iter)
      code = STOP_MAX_ITER;
    else if (rule.diverge_factor > 0 && rho > rule.diverge_factor * res0)
      code = STOP_DIVERGED;
    if (code != STOP_NONE) {
      *stop = code;
      break;
    }
    st = vcycle2d<T>(h, 1, B.r[0], c[cur]);
    if (st != MGRIT_OK) return st;
    ++it;
  }
  *iters = it;
  *cfinal = c[cur];
  if (res0_out) *res0_out = res0;
  if (rho_out) *rho_out = rho;
  if (prev_out) *prev_out = prev;
  return MGRIT_OK;
}

void fill_stats(mgrit_stats *stats, int it, int inner, double res0, double rho, double prev,
                const std::vector<double> &hist, std::chrono::steady_clock::time_point t0) {
  if (!stats) return;
  stats->iterations = it;
  stats->inner_iterations = inner;
  stats->res0 = res0;
  stats->res_final = rho;
  stats->conv_factor = prev > 0 ? rho / prev : NAN;
  const int len = (int)hist.size();
  if (stats->res_history)
    for (int i = 0; i < std::min(len, stats->res_history_cap); ++i) stats->res_history[i] = hist[i];
  stats->res_history_len = std::min(len, std::max(stats->res_history_cap, 0));
  stats->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Mixed precision in 2D: as mp_solve in 1D (float64 space-time residual,
// test and update; float32 MGRIT on the correction equation).
mgrit_status mp2d_solve(mgrit2d_handle *h, const double *u0, const double *v_init, double *u_out, double *u_final,
                        mgrit_stats *stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t S = slab(h);
  const int64_t nt = h->prob.nt;
  const int64_t pts = nt * S;
  double *U = u_out ? u_out : h->u64;
  if (v_init && v_init != U) {
    HIPCHK2(h, hipMemcpyAsync(U, v_init, (pts + S) * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  } else if (!v_init) {
    HIPCHK2(h, launch_fill(U, pts + S, 0.0, h->stream));
  }
  HIPCHK2(h, hipMemcpyAsync(U, u0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  const StopRule inner{h->opt.inner_rtol, h->opt.diverge_factor, h->opt.inner_max_iter, 0.5};
  std::vector<double> hist;
  double res0 = NAN, rho = NAN, prev = NAN;
  int outer = 0, inner_total = 0;
  mgrit_status status = MGRIT_OK;
  const int64_t chunk = h->cap;
  for (;;) {
    // float64: r_n = Phi u_{n-1} - u_n, n = 1..nt, in chunks of cap slabs
    for (int64_t n0 = 0; n0 < nt; n0 += chunk) {
      const int64_t nb = std::min(chunk, nt - n0);
      HIPCHK2(h, apply2d<double>(h, 0, U + n0 * S, S, h->r64 + n0 * S, S, nb, U + (n0 + 1) * S, S, -1.0));
    }
    double acc = 0.0;  // chunk by chunk, in a fixed order
    for (int64_t n0 = 0; n0 < nt; n0 += chunk) {
      const int64_t nb = std::min(chunk, nt - n0);
      HIPCHK2(h, launch_slab_norm(h->r64 + n0 * S, nb, S, RESID_BLOCKS, h->normpart, h->stream));
      hipError_t e;
      const double part = norm2d(h, nb * RESID_BLOCKS, e);
      if (e) return fail2(h, MGRIT_EDEVICE, "outer residual norm");
      acc += part * part;
    }
    prev = rho;
    rho = std::sqrt(acc);
    hist.push_back(rho);
    if (outer == 0) res0 = rho;
    if (!std::isfinite(rho)) {
      status = fail2(h, MGRIT_EDIVERGED, "non-finite residual");
      break;
    }
    if (rho <= h->opt.rtol * res0) break;
    if (outer >= h->opt.max_iter) {
      status = MGRIT_ENOTCONVERGED;
      h->err = "max_iter reached";
      break;
    }
    if (h->opt.diverge_factor > 0 && rho > h->opt.diverge_factor * res0) {
      status = fail2(h, MGRIT_EDIVERGED, "residual grew past diverge_factor * res0");
      break;
    }
    // float32: A e = r from zero, then u += e in float64
    HIPCHK2(h, launch_round32(h->r64, h->g32, pts, h->stream));
    const int64_t nc = h->lv[0].nt / h->lv[0].m;
    HIPCHK2(h, launch_slab_axpy<float>(h->d32.c0[0], S, h->d32.zero, 0, nc + 1, S, false, h->stream));
    int iters = 0, stop = 0;
    float *cfin = nullptr;
    const mgrit_status st =
        mgrit2d_iterate<float>(h, h->g32, inner, &iters, &stop, &cfin, nullptr, nullptr, nullptr, nullptr);
    if (st != MGRIT_OK) return st;
    inner_total += iters;
    if (stop == STOP_NONFINITE || stop == STOP_DIVERGED) {
      status = fail2(h, MGRIT_EDIVERGED, "the float32 inner solve diverged");
      break;
    }
    const mgrit_status fs = relax2d<float>(h, 0, MODE_FINAL_F, cfin, nullptr, h->g32, nullptr, nullptr, h->e32);
    if (fs != MGRIT_OK) return fs;
    HIPCHK2(h, launch_add32(U, h->e32, pts + S, h->stream));
    ++outer;
  }
  if (u_final) HIPCHK2(h, hipMemcpyAsync(u_final, U + pts, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  HIPCHK2(h, hipStreamSynchronize(h->stream));
  fill_stats(stats, outer, inner_total, res0, rho, prev, hist, t0);
  return status;
}

}  // namespace

extern "C" {

mgrit_status mgrit2d_setup(const mgrit2d_problem *P, const mgrit_options *O, void *stream, mgrit2d_handle **out) {
  g_setup_error.clear();
  if (out) *out = nullptr;
  auto bad = [&](mgrit_status s, const std::string &m) {
    g_setup_error = m;
    return s;
  };
  if (!P || !O || !out) return bad(MGRIT_EINVAL, "null argument");
  if (!(P->velocity_x > 0) || !(P->velocity_y > 0) || !(P->x_hi > P->x_lo) || !(P->y_hi > P->y_lo) || !(P->dt > 0))
    return bad(MGRIT_EINVAL, "need a_x, a_y > 0, a non-empty rectangle and dt > 0");
  if (P->nx < 1 || P->nx > MGRIT_MAX_NX || P->ny < 1 || P->ny > MGRIT_MAX_NX)
    return bad(MGRIT_EINVAL, "nx and ny must be in 1..16384");
  if (P->nt < 1) return bad(MGRIT_EINVAL, "nt must be >= 1");
  if (P->upwind_order != 1 && P->upwind_order != 3 && P->upwind_order != 5)
    return bad(MGRIT_EINVAL, "the 2D coarse step needs odd upwind order 1, 3 or 5");
  if (O->max_levels < 2 || O->max_levels > MGRIT_MAX_LEVELS) return bad(MGRIT_EINVAL, "max_levels must be in 2..16");
  if (O->nu < 0 || O->nu > 8) return bad(MGRIT_EINVAL, "nu must be in 0..8");
  if (O->max_iter < 0 || !(O->rtol >= 0)) return bad(MGRIT_EINVAL, "need max_iter >= 0 and rtol >= 0");
  if (O->cg_kind != MGRIT_CG_SL_CORRECTED) return bad(MGRIT_EINVAL, "2D: corrected semi-Lagrangian coarse step only");
  if (O->coarse_solve != 0) return bad(MGRIT_EINVAL, "2D: the coarse solves are exact (coarse_solve = 0)");
  if (O->precision != MGRIT_PREC_FP64 && O->precision != MGRIT_PREC_MIXED) return bad(MGRIT_EINVAL, "unknown precision");
  const bool mixed = O->precision == MGRIT_PREC_MIXED;
  if (mixed && !(O->inner_rtol > 0 && O->inner_rtol < 1))
    return bad(MGRIT_EINVAL, "mixed precision needs 0 < inner_rtol < 1");
  if (mixed && O->inner_max_iter < 1) return bad(MGRIT_EINVAL, "mixed precision needs inner_max_iter >= 1");
  mgrit_problem p1{};
  p1.velocity = 1;
  p1.x_lo = 0;
  p1.x_hi = 1;
  p1.nx = P->nx;
  p1.nt = P->nt;
  p1.cfl = 1;
  p1.upwind_order = P->upwind_order;
  p1.rk_kind = MGRIT_ERK;
  p1.rk_order = P->rk_order;
  FineInfo fi;
  std::string err;
  mgrit_status st = fine_info(p1, fi, err);
  if (st != MGRIT_OK) return bad(st, err);
  std::vector<int64_t> nts;
  std::vector<int> ms;
  if (!level_hierarchy(p1, *O, nts, ms, err)) return bad(MGRIT_EINVAL, err);
  const int nlev = (int)nts.size();
  const int p = P->upwind_order, q = P->rk_order;
  const double cx = P->velocity_x * P->dt / ((P->x_hi - P->x_lo) / (double)P->nx);
  const double cy = P->velocity_y * P->dt / ((P->y_hi - P->y_lo) / (double)P->ny);
  // stability of the fine step: |R(-(c_x Lhat(w_x) + c_y Lhat(w_y)))| <= 1
  {
    const int N = 256;
    const std::vector<ld> beta = rk_series(fi.tab, fi.tab.s);
    std::vector<std::complex<double>> lx(N), ly(N);
    for (int k = 0; k < N; ++k) {
      const double om = -M_PI + 2 * M_PI * k / N;
      lx[k] = cx * upwind_symbol(fi, om);
      ly[k] = cy * upwind_symbol(fi, om);
    }
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) {
        const std::complex<double> z = -(lx[i] + ly[k]);
        std::complex<double> acc = (double)beta[fi.tab.s];
        for (int j = fi.tab.s - 1; j >= 0; --j) acc = acc * z + (double)beta[j];
        if (std::abs(acc) > 1 + 1e-10) return bad(MGRIT_EUNSTABLE, "2D explicit step above its stability limit");
      }
  }
  std::vector<SlLevel> chx, chy;
  const std::vector<int> mc(ms.begin(), ms.begin() + (nlev - 1));
  if (!sl_chain(fi, p, q, cx, mc, (int)P->nx, 16, false, chx, err) ||
      !sl_chain(fi, p, q, cy, mc, (int)P->ny, 16, false, chy, err))
    return bad(MGRIT_EINVAL, err);

  auto *h = new mgrit2d_handle();
  h->prob = *P;
  h->opt = *O;
  h->stream = (hipStream_t)stream;
  h->lv.resize(nlev);
  for (int l = 0; l < nlev; ++l) {
    h->lv[l].nt = nts[l];
    h->lv[l].m = l < nlev - 1 ? ms[l] : 0;
  }
  // fine step constants: Horner coefficients of R and the two stencils
  Step2dArgs &f = h->fine;
  f.nx = (int)P->nx;
  f.ny = (int)P->ny;
  f.ncoef = fi.tab.s + 1;
  for (int i = 0; i <= fi.tab.s; ++i) f.coef[i] = (double)fi.beta[i];
  f.sl = fi.l;
  f.sr = fi.r;
  f.use_reg = env_int("MGRIT_2D_LDS", 0) == 0;
  for (int j = 0; j <= fi.l + fi.r; ++j) {
    f.tx[j] = -cx * fi.w[j];
    f.ty[j] = -cy * fi.w[j];
  }
  if (step2d_lds_bytes(f.ncoef, f.sl, f.sr) > LDS_LIMIT) {
    mgrit2d_destroy(h);
    return bad(MGRIT_EINVAL, "2D fine step: halo too wide for LDS");
  }
  if (configure_once() != hipSuccess) {
    mgrit2d_destroy(h);
    return bad(MGRIT_EDEVICE, "configure");
  }
  // ---- device memory: one allocation.  Head (uploaded): the line tables in
  // float64 (and float32), the line descriptors; then the arrays.
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const int64_t S = P->nx * P->ny;
  const int64_t nc0 = nts[0] / ms[0];
  h->cap = std::max<int64_t>(nc0, 1);
  std::vector<size_t> tab_off(2 * nlev, 0), tab_len(2 * nlev, 0);
  std::vector<double> tabs;
  for (int l = 1; l < nlev; ++l)
    for (int ax = 0; ax < 2; ++ax) {
      const SlLevel &SL = ax == 0 ? chx[l - 1] : chy[l - 1];
      tab_off[2 * l + ax] = tabs.size();
      tab_len[2 * l + ax] = SL.tabs.size();
      tabs.insert(tabs.end(), SL.tabs.begin(), SL.tabs.end());
    }
  size_t off = 0;
  const size_t o_tabs = off;
  off += al(std::max<size_t>(tabs.size(), 1) * sizeof(double));
  const size_t o_tabs32 = off;
  if (mixed) off += al(std::max<size_t>(tabs.size(), 1) * sizeof(float));
  const size_t o_desc = off;
  off += al(4 * nlev * sizeof(LevelDesc));
  const size_t head = off;
  auto arrays = [&](size_t w, std::vector<size_t> &oc0, std::vector<size_t> &oc1, std::vector<size_t> &orr,
                    size_t (&ow)[5]) {
    oc0.assign(nlev, 0);
    oc1.assign(nlev, 0);
    orr.assign(nlev, 0);
    for (int l = 0; l + 1 < nlev; ++l) {
      const int64_t nc = nts[l] / ms[l];
      oc0[l] = off, off += al((nc + 1) * S * w);
      oc1[l] = off, off += al((nc + 1) * S * w);
      orr[l] = off, off += al(nc * S * w);
    }
    for (int i = 0; i < 4; ++i) ow[i] = off, off += al(h->cap * S * w);
    ow[4] = off, off += al(S * w);  // zero slab
  };
  std::vector<size_t> a0, a1, ar, b0, b1, br;
  size_t wa[5], wb[5];
  arrays(sizeof(double), a0, a1, ar, wa);
  size_t o_g32 = 0, o_e32 = 0, o_r64 = 0, o_u64 = 0;
  if (mixed) {
    arrays(sizeof(float), b0, b1, br, wb);
    o_g32 = off, off += al((size_t)(nts[0] * S) * sizeof(float));
    o_e32 = off, off += al(((size_t)(nts[0] * S) + S) * sizeof(float));
    o_r64 = off, off += al((size_t)(nts[0] * S) * sizeof(double));
    o_u64 = off, off += al(((size_t)(nts[0] * S) + S) * sizeof(double));
  }
  h->normpart_len = h->cap * RESID_BLOCKS;
  const size_t o_np = off;
  off += al(h->normpart_len * sizeof(double));
  const size_t o_ns = off;
  off += al(sizeof(double));
  if (hipMalloc((void **)&h->arena, off) != hipSuccess) {
    mgrit2d_destroy(h);
    return bad(MGRIT_ENOMEM, "device workspace");
  }
  char *base = h->arena;
  std::vector<char> up(head, 0);
  std::memcpy(up.data() + o_tabs, tabs.data(), tabs.size() * sizeof(double));
  if (mixed) {
    float *t32 = (float *)(up.data() + o_tabs32);
    for (size_t i = 0; i < tabs.size(); ++i) t32[i] = (float)tabs[i];
  }
  int di = 0;
  for (int l = 1; l < nlev; ++l)
    for (int ax = 0; ax < 2; ++ax) {
      const SlLevel &SL = ax == 0 ? chx[l - 1] : chy[l - 1];
      Line1D &ln = ax == 0 ? h->lv[l].x : h->lv[l].y;
      ln.op = SL.op;
      ln.lay = SL.lay;
      for (int prec = 0; prec < (mixed ? 2 : 1); ++prec) {
        LevelDesc hd{ln.op, ln.lay};
        const size_t tb = tab_off[2 * l + ax];
        // the level's tables: scan tables, then (when present) the windowed plan's
        auto tab_at = [&](size_t i) -> const void * {
          if (i >= SL.offs.size() || SL.offs[i] == (size_t)-1) return nullptr;
          if (prec == 0) return (const double *)(base + o_tabs) + tb + SL.offs[i];
          return (const float *)(base + o_tabs32) + tb + SL.offs[i];
        };
        hd.op.fw.tab = tab_at(0);
        hd.op.bw.tab = tab_at(1);
        hd.op.fw.wtab = tab_at(2);
        hd.op.bw.wtab = tab_at(3);
        LevelDesc *dd = (LevelDesc *)(base + o_desc) + di++;
        (prec == 0 ? ln.desc : ln.desc32) = dd;
        std::memcpy(up.data() + ((char *)dd - base), &hd, sizeof(LevelDesc));
      }
    }
  auto place = [&](auto &B, const std::vector<size_t> &o0, const std::vector<size_t> &o1,
                   const std::vector<size_t> &orr, const size_t (&ow)[5]) {
    using P_ = std::remove_reference_t<decltype(*B.w[0])>;
    B.c0.assign(nlev, nullptr);
    B.c1.assign(nlev, nullptr);
    B.r.assign(nlev, nullptr);
    for (int l = 0; l + 1 < nlev; ++l) {
      B.c0[l] = (P_ *)(base + o0[l]);
      B.c1[l] = (P_ *)(base + o1[l]);
      B.r[l] = (P_ *)(base + orr[l]);
    }
    B.w[0] = (P_ *)(base + ow[0]);
    B.w[1] = (P_ *)(base + ow[1]);
    B.t1 = (P_ *)(base + ow[2]);
    B.t2 = (P_ *)(base + ow[3]);
    B.zero = (P_ *)(base + ow[4]);
  };
  place(h->d64, a0, a1, ar, wa);
  if (mixed) {
    place(h->d32, b0, b1, br, wb);
    h->g32 = (float *)(base + o_g32);
    h->e32 = (float *)(base + o_e32);
    h->r64 = (double *)(base + o_r64);
    h->u64 = (double *)(base + o_u64);
  }
  h->normpart = (double *)(base + o_np);
  h->normsum = (double *)(base + o_ns);
  if (hipMemcpyAsync(base, up.data(), head, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      launch_fill(h->d64.zero, S, 0.0, h->stream) != hipSuccess ||
      (mixed && launch_fill32(h->d32.zero, S, h->stream) != hipSuccess) ||
      hipHostMalloc((void **)&h->normsum_host, sizeof(double)) != hipSuccess) {
    mgrit2d_destroy(h);
    return bad(MGRIT_EDEVICE, "upload");
  }
  *out = h;
  return MGRIT_OK;
}

mgrit_status mgrit2d_solve(mgrit2d_handle *h, const double *u0, const double *v_init, double *u_out, double *u_final,
                           mgrit_stats *stats) {
  if (!h) return MGRIT_EINVAL;
  if (!u0) return fail2(h, MGRIT_EINVAL, "u0 is required");
  if (h->opt.precision == MGRIT_PREC_MIXED) return mp2d_solve(h, u0, v_init, u_out, u_final, stats);
  const auto t0 = std::chrono::steady_clock::now();
  Level2 &L0 = h->lv[0];
  const int64_t S = slab(h);
  const int m = L0.m;
  const int64_t nc = L0.nt / m;
  double *c0 = h->d64.c0[0];
  if (v_init) {
    HIPCHK2(h, launch_slab_axpy<double>(c0, S, v_init, m * S, nc + 1, S, false, h->stream));
  } else {
    HIPCHK2(h, launch_fill(c0, (nc + 1) * S, 0.0, h->stream));
  }
  HIPCHK2(h, hipMemcpyAsync(c0, u0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  const StopRule rule{h->opt.rtol, h->opt.diverge_factor, h->opt.max_iter, 0.0};
  std::vector<double> hist;
  double res0 = NAN, rho = NAN, prev = NAN;
  int it = 0, stop = 0;
  double *cfin = nullptr;
  const mgrit_status st = mgrit2d_iterate<double>(h, (const double *)nullptr, rule, &it, &stop, &cfin, &hist, &res0,
                                                  &rho, &prev);
  if (st != MGRIT_OK) return st;
  mgrit_status status = MGRIT_OK;
  if (stop == STOP_NONFINITE) {
    status = fail2(h, MGRIT_EDIVERGED, "non-finite residual");
  } else if (stop == STOP_MAX_ITER) {
    status = MGRIT_ENOTCONVERGED;
    h->err = "max_iter reached";
  } else if (stop == STOP_DIVERGED) {
    status = fail2(h, MGRIT_EDIVERGED, "residual grew past diverge_factor * res0");
  }
  if (status == MGRIT_OK || status == MGRIT_ENOTCONVERGED) {
    if (u_out) {
      const mgrit_status fs = relax2d<double>(h, 0, MODE_FINAL_F, cfin, nullptr, nullptr, nullptr, nullptr, u_out);
      if (fs != MGRIT_OK) return fs;
    }
    if (u_final)
      HIPCHK2(h, hipMemcpyAsync(u_final, cfin + nc * S, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  }
  HIPCHK2(h, hipStreamSynchronize(h->stream));
  fill_stats(stats, it, 0, res0, rho, prev, hist, t0);
  return status;
}

mgrit_status mgrit2d_sequential(mgrit2d_handle *h, const double *u0, double *u_out) {
  if (!h || !u0 || !u_out) return MGRIT_EINVAL;
  const int64_t S = slab(h);
  HIPCHK2(h, hipMemcpyAsync(u_out, u0, S * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  for (int64_t n = 1; n <= h->prob.nt; ++n)
    HIPCHK2(h, apply2d<double>(h, 0, u_out + (n - 1) * S, S, u_out + n * S, S, 1, nullptr, 0));
  HIPCHK2(h, hipStreamSynchronize(h->stream));
  return MGRIT_OK;
}

mgrit_status mgrit2d_apply_step(mgrit2d_handle *h, int32_t level, const double *v_in, double *v_out, int64_t count) {
  if (!h || !v_in || !v_out || level < 0 || level >= (int32_t)h->lv.size() || count < 0) return MGRIT_EINVAL;
  const int64_t S = slab(h);
  for (int64_t b = 0; b < count; b += h->cap) {
    const int64_t nb = std::min<int64_t>(h->cap, count - b);
    HIPCHK2(h, apply2d<double>(h, level, v_in + b * S, S, v_out + b * S, S, nb, nullptr, 0));
  }
  HIPCHK2(h, hipStreamSynchronize(h->stream));
  return MGRIT_OK;
}

int32_t mgrit2d_num_levels(const mgrit2d_handle *h) { return h ? (int32_t)h->lv.size() : 0; }

const char *mgrit2d_last_error(const mgrit2d_handle *h) { return h ? h->err.c_str() : g_setup_error.c_str(); }

void mgrit2d_destroy(mgrit2d_handle *h) {
  if (!h) return;
  if (h->arena) (void)hipStreamSynchronize(h->stream);
  if (h->arena) (void)hipFree(h->arena);
  if (h->normsum_host) (void)hipHostFree(h->normsum_host);
  delete h;
}

}  // extern "C"

namespace mgrit {

// The allocation-free solve behind mgrit_solve_noalloc (mgrit_noalloc.hip):
// set up a float64 handle inside the device workspace ws (no device, pinned
// or event allocations), solve with the host waiting for each stopping
// decision, and release the host-side handle.  Messages go to the
// thread's setup-error string (mgrit_last_error(NULL)).
mgrit_status noalloc_solve(const mgrit_problem *P, const mgrit_options *O, void *stream, void *ws,
                           uint64_t ws_bytes, const double *u0, const double *v_init, double *u_out,
                           double *u_final, mgrit_stats *stats) {
  if (!P || !O) {
    g_setup_error = "null argument";
    return MGRIT_EINVAL;
  }
  if (O->precision != MGRIT_PREC_FP64) {
    g_setup_error = "the allocation-free solve runs float64 problems only";
    return MGRIT_EINVAL;
  }
  if (O->tile_tune) {
    g_setup_error = "the allocation-free solve takes no tile tuning (it times launches with events)";
    return MGRIT_EINVAL;
  }
  if (!u0) {
    g_setup_error = "u0 is required";
    return MGRIT_EINVAL;
  }
  uint64_t need = 0;
  mgrit_status st = mgrit_workspace_bytes(P, O, &need);
  if (st != MGRIT_OK) {
    g_setup_error = "invalid problem or options";
    return st;
  }
  if (need > ws_bytes) {
    g_setup_error = "the problem needs " + std::to_string(need) + " bytes of workspace; the allocation-free solve has " +
                    std::to_string(ws_bytes);
    return MGRIT_EINVAL;
  }
  mgrit_handle *h = nullptr;
  st = setup_impl(P, O, stream, ws, ws_bytes, &h, true);
  if (st != MGRIT_OK) return st;
  auto &ss = h->ss;
  st = mgrit_solve_start(h, u0, v_init, u_out, u_final);
  while (st == MGRIT_OK && !ss.finished) {
    // the iteration's state reached ctl_local by a copy queued before its
    // coarse-grid correction; the next iteration is queued after the decision
    if (hipError_t e = hipStreamSynchronize(h->stream)) {
      st = hipfail(h, e, "stream");
      break;
    }
    st = take_decision(h);
    if (st == MGRIT_OK && !ss.finished) st = queue_iteration(h);
  }
  if (st == MGRIT_OK) {
    st = mgrit_solve_finish(h, stats);
  } else {
    (void)hipStreamSynchronize(h->stream);
  }
  g_setup_error = (st == MGRIT_OK) ? std::string() : h->err;
  mgrit_destroy(h);
  return st;
}

}  // namespace mgrit

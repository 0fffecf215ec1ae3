// Reference quadrature and interpolation data, built on the host in long
// double when a plan is created.
//
// Gauss rules come from the three-term recurrence of their orthogonal
// polynomials: the nodes are the eigenvalues of the symmetric tridiagonal
// Jacobi matrix, isolated one at a time by bisection on Sturm-sequence sign
// counts; the weights are the Christoffel numbers 1 / sum_k p_k(x)^2 of the
// orthonormal polynomials.  Rules used by the method:
//   * Gauss-Legendre on [0,1]            arc-length panels (Sec. 3.4), the
//                                        smooth part of the radial rule
//   * Gauss-Jacobi (1,0) x Gauss-Legendre the q x q collapsed rule on the
//                                        simplex (far and near rules, Sec. 3.2/3.3)
//   * Gauss for the weight -log(r)       the r log r part of the radial rule
//                                        (Sec. 3.4), recurrence from modified
//                                        moments against shifted Legendre
//                                        polynomials (modified Chebyshev algorithm)
//   * Gauss-Lobatto-Legendre points      interpolation nodes (Blyth-Pozrikidis)
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>

#include "vp_internal.h"

namespace vp {
namespace {

typedef long double ld;

// Number of eigenvalues of the Jacobi matrix (diag a, off-diag sqrt(b[k]),
// k >= 1) below x.
int sturm_count(const std::vector<ld>& a, const std::vector<ld>& b, ld x) {
  int neg = 0;
  ld d = 1.0L;
  for (size_t k = 0; k < a.size(); ++k) {
    ld v = (a[k] - x) - (k ? b[k] / d : 0.0L);
    if (v == 0.0L) v = -1e-300L;
    if (v < 0.0L) ++neg;
    d = v;
  }
  return neg;
}

// Gauss rule from monic recurrence coefficients a[0..n-1], b[0..n-1]
// (b[0] = total mass of the measure).
Rule1D gauss_from_recurrence(const std::vector<ld>& a, const std::vector<ld>& b) {
  const int n = (int)a.size();
  // Gershgorin interval
  ld lo = 1e300L, hi = -1e300L;
  for (int k = 0; k < n; ++k) {
    ld r = (k > 0 ? sqrtl(b[k]) : 0.0L) + (k + 1 < n ? sqrtl(b[k + 1]) : 0.0L);
    lo = std::min(lo, a[k] - r);
    hi = std::max(hi, a[k] + r);
  }
  Rule1D out;
  out.x.resize(n);
  out.w.resize(n);
  for (int i = 0; i < n; ++i) {
    ld l = lo, h = hi;
    for (int it = 0; it < 200 && h - l > 0.0L; ++it) {
      ld mid = 0.5L * (l + h);
      if (mid == l || mid == h) break;
      if (sturm_count(a, b, mid) > i)
        h = mid;
      else
        l = mid;
    }
    const ld x = 0.5L * (l + h);
    // Christoffel number from orthonormal polynomials
    ld pm1 = 0.0L, p0 = 1.0L / sqrtl(b[0]);
    ld sum = p0 * p0;
    for (int k = 0; k + 1 < n; ++k) {
      ld p1 = ((x - a[k]) * p0 - (k > 0 ? sqrtl(b[k]) : 0.0L) * pm1) / sqrtl(b[k + 1]);
      pm1 = p0;
      p0 = p1;
      sum += p0 * p0;
    }
    out.x[i] = (double)x;
    out.w[i] = (double)(1.0L / sum);
  }
  return out;
}

// Monic Jacobi (alpha, beta) recurrence on [-1, 1].
void jacobi_recurrence(int n, ld al, ld be, std::vector<ld>& a, std::vector<ld>& b) {
  a.assign(n, 0.0L);
  b.assign(n, 0.0L);
  for (int k = 0; k < n; ++k) {
    ld s = 2.0L * k + al + be;
    if (k == 0)
      a[k] = (be - al) / (al + be + 2.0L);
    else
      a[k] = (be * be - al * al) / (s * (s + 2.0L));
  }
  b[0] = powl(2.0L, al + be + 1.0L) * tgammal(al + 1.0L) * tgammal(be + 1.0L) / tgammal(al + be + 2.0L);
  for (int k = 1; k < n; ++k) {
    ld s = 2.0L * k + al + be;
    ld num = 4.0L * k * (k + al) * (k + be) * (k + al + be);
    ld den = s * s * (s + 1.0L) * (s - 1.0L);
    b[k] = num / den;
  }
}

// Map a monic Jacobi (al, be) recurrence on [-1,1] to [0,1] (s = 2x - 1):
// the weight (1-s)^al (1+s)^be becomes 2^(al+be) (1-x)^al x^be, so the mass
// is divided by 2^(al+be+1) to get the rule for (1-x)^al x^be on [0,1].
void to_unit_interval(std::vector<ld>& a, std::vector<ld>& b, ld al_plus_be) {
  for (size_t k = 0; k < a.size(); ++k) {
    a[k] = 0.5L * (a[k] + 1.0L);
    b[k] = (k == 0) ? b[k] / powl(2.0L, al_plus_be + 1.0L) : 0.25L * b[k];
  }
}

}  // namespace

static Rule1D gauss_legendre01_compute(int n) {
  std::vector<ld> a, b;
  jacobi_recurrence(n, 0.0L, 0.0L, a, b);
  to_unit_interval(a, b, 0.0L);
  return gauss_from_recurrence(a, b);
}

static Rule1D gauss_log01_compute(int n) {
  // Modified moments nu_l = int_0^1 -log(r) pi_l(r) dr against the monic
  // shifted Legendre polynomials pi_l (recurrence a_l = 1/2,
  // b_l = l^2 / (4 (4 l^2 - 1))).  With P*_l(r) = P_l(2r - 1):
  //   int_0^1 -log(r) P*_l(r) dr = 1 (l = 0), (-1)^l / (l (l+1)) (l >= 1),
  // and pi_l = P*_l (l!)^2 / (2l)!.
  const int m = 2 * n;
  std::vector<ld> nu(m), am(m, 0.5L), bm(m, 0.0L);
  for (int l = 0; l < m; ++l) {
    ld lead = 1.0L;  // (2l)! / (l!)^2
    for (int i = 1; i <= l; ++i) lead = lead * (ld)(l + i) / (ld)i;
    ld mom = (l == 0) ? 1.0L : ((l % 2 == 0) ? 1.0L : -1.0L) / ((ld)l * (l + 1));
    nu[l] = mom / lead;
    if (l >= 1) bm[l] = (ld)l * l / (4.0L * (4.0L * l * l - 1.0L));
  }
  // modified Chebyshev algorithm
  std::vector<ld> alpha(n), beta(n);
  std::vector<ld> sig_prev(m + 1, 0.0L), sig(m + 1, 0.0L), sig_new(m + 1, 0.0L);
  for (int l = 0; l < m; ++l) sig[l] = nu[l];
  alpha[0] = am[0] + nu[1] / nu[0];
  beta[0] = nu[0];
  for (int k = 1; k < n; ++k) {
    std::fill(sig_new.begin(), sig_new.end(), 0.0L);
    for (int l = k; l < m - k; ++l) {
      sig_new[l] = sig[l + 1] - (alpha[k - 1] - am[l]) * sig[l] - beta[k - 1] * sig_prev[l] +
                   bm[l] * sig[l - 1];
    }
    alpha[k] = am[k] + sig_new[k + 1] / sig_new[k] - sig[k] / sig[k - 1];
    beta[k] = sig_new[k] / sig[k - 1];
    sig_prev.swap(sig);
    sig.swap(sig_new);
  }
  return gauss_from_recurrence(alpha, beta);
}

static Rule2D collapsed_gauss_compute(int q) {
  // int_T g = int_0^1 int_0^1 g(u, (1-u) v) (1-u) dv du: Gauss-Jacobi for the
  // weight (1-u) in u, Gauss-Legendre in v.
  std::vector<ld> a, b;
  jacobi_recurrence(q, 1.0L, 0.0L, a, b);
  to_unit_interval(a, b, 1.0L);
  Rule1D ru = gauss_from_recurrence(a, b);
  Rule1D rv = gauss_legendre01(q);
  Rule2D r;
  r.x.resize(q * q);
  r.y.resize(q * q);
  r.w.resize(q * q);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      r.x[i * q + j] = ru.x[i];
      r.y[i * q + j] = (double)((1.0L - (ld)ru.x[i]) * (ld)rv.x[j]);
      r.w[i * q + j] = (double)((ld)ru.w[i] * (ld)rv.w[j]);
    }
  return r;
}

void edge_weights(const Rule2D& r, int q, double out[3]) {
  // Per edge of the simplex (AB: y = 0, BC: x + y = 1, CA: x = 0): the
  // largest weight among the q nodes nearest the edge (Sec. 4.1, the weight
  // w of eq. rho0).
  const size_t n = r.w.size();
  for (int e = 0; e < 3; ++e) {
    std::vector<double> d(n);
    for (size_t i = 0; i < n; ++i) {
      d[i] = (e == 0) ? r.y[i] : (e == 1) ? (1.0 - r.x[i] - r.y[i]) * 0.70710678118654752440 : r.x[i];
    }
    std::vector<size_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return d[a] < d[b]; });
    double w = 0.0;
    for (int i = 0; i < q; ++i) w = std::max(w, r.w[idx[i]]);
    out[e] = w;
  }
}

static Rule2D interp_nodes_compute(int p) {
  // Gauss-Lobatto-Legendre points of order M = p + 3 on [0,1]: 0, 1 and the
  // roots of P_M', i.e. the Gauss-Jacobi (1,1) nodes of degree M - 1.
  const int M = p + 3;
  std::vector<ld> a, b;
  jacobi_recurrence(M - 1, 1.0L, 1.0L, a, b);
  to_unit_interval(a, b, 2.0L);
  Rule1D inner = gauss_from_recurrence(a, b);
  std::vector<double> v(M + 1);
  v[0] = 0.0;
  v[M] = 1.0;
  for (int i = 1; i < M; ++i) v[i] = inner.x[i - 1];
  // Blyth-Pozrikidis: i + j + k = M, all >= 1
  Rule2D r;
  for (int i = 1; i < M; ++i)
    for (int j = 1; j < M - i; ++j) {
      int k = M - i - j;
      ld vi = v[i], vj = v[j], vk = v[k];
      r.x.push_back((double)((1.0L + 2.0L * vi - vj - vk) / 3.0L));
      r.y.push_back((double)((1.0L + 2.0L * vj - vi - vk) / 3.0L));
      r.w.push_back(0.0);
    }
  return r;
}

void log_table(double2* out, int n) {
  // centres c_i = 1/2 + (i + 1/2)/(2n) of the n sub-intervals of [1/2, 1);
  // inv_c_i = nearest double to 1/c_i, paired with -log(inv_c_i) (long
  // double, then rounded); the last entry splits ln 2 into a 32-bit head
  // and its remainder.
  const ld ln2 = logl(2.0L);
  const double hi = (double)(ldexpl(floorl(ldexpl(ln2, 32)), -32));
  for (int i = 0; i < n; ++i) {
    const ld c = 0.5L + ((ld)i + 0.5L) / (2.0L * n);
    const double inv = (double)(1.0L / c);
    out[i] = make_double2(inv, (double)(-logl((ld)inv)));
  }
  out[n] = make_double2(hi, (double)(ln2 - (ld)hi));
}

int radial_half(int p) { return std::max(4, (p + 3) / 2); }

void radial_rule(int p, std::vector<double>& r, std::vector<double>& alpha, std::vector<double>& beta) {
  // int_0^1 r log(r0 r) phi(r) dr = log r0 int r phi + int r log(r) phi:
  // Gauss-Legendre for the first, Gauss for the weight -log(r) for the
  // second; exact for phi of degree <= p.
  const int n = radial_half(p);
  Rule1D g = gauss_legendre01(n);
  Rule1D l = gauss_log01(n);
  r.clear();
  alpha.clear();
  beta.clear();
  for (int i = 0; i < n; ++i) {
    r.push_back(g.x[i]);
    alpha.push_back(g.w[i] * g.x[i]);
    beta.push_back(0.0);
  }
  for (int i = 0; i < n; ++i) {
    r.push_back(l.x[i]);
    alpha.push_back(0.0);
    beta.push_back(-l.w[i] * l.x[i]);
  }
}

void radial_rule_folded(int p, std::vector<double>& r, std::vector<double>& alpha, std::vector<double>& beta) {
  // Along a ray of a straight self piece the basis is a polynomial of degree
  // <= p in r, so the radial rule's sum sum_i (alpha_i log r0 + beta_i)
  // phi(r_i) equals sum_j (A_j log r0 + B_j) phi(rho_j) over any p + 1
  // nodes rho_j, with A_j = sum_i alpha_i l_j(r_i), B_j = sum_i beta_i
  // l_j(r_i) (l_j the Lagrange polynomials of the rho_j): the same integrals
  // int_0^1 r l_j(r) dr and int_0^1 r log(r) l_j(r) dr, with p + 1 basis
  // evaluations per ray instead of 2 radial_half(p).  rho_0 = 0, the ray's
  // apex (the target itself, the same point on every ray of a piece, so
  // its basis values are needed once per pair), then the p-point
  // Gauss-Legendre nodes on [0, 1] (small Lagrange polynomials on [0, 1]).
  std::vector<double> ri, ai, bi;
  radial_rule(p, ri, ai, bi);
  const Rule1D g = gauss_legendre01(p);
  r.assign(1, 0.0);
  r.insert(r.end(), g.x.begin(), g.x.end());
  alpha.assign(p + 1, 0.0);
  beta.assign(p + 1, 0.0);
  for (int j = 0; j <= p; ++j) {
    ld A = 0.0L, B = 0.0L;
    for (size_t i = 0; i < ri.size(); ++i) {
      ld l = 1.0L;
      for (int k = 0; k <= p; ++k)
        if (k != j) l *= ((ld)ri[i] - (ld)r[k]) / ((ld)r[j] - (ld)r[k]);
      A += (ld)ai[i] * l;
      B += (ld)bi[i] * l;
    }
    alpha[j] = (double)A;
    beta[j] = (double)B;
  }
}

std::vector<double> basis_connection(int p) {
  const int np = (p + 1) * (p + 2) / 2;
  std::vector<double> g((size_t)np * (p + 1), 0.0);
  // P^{(a,0)}_k(z) for a = 2m + 1 in monomials (the three-term recurrence
  // of the device basis), then in the monic Legendre polynomials Pm_j
  // (highest degree first: Pm_j is monic), times c_mn and the leading
  // coefficient (2m)! / (2^m m!^2) of the Legendre polynomial in Q_m
  std::vector<std::vector<ld>> pm(p + 1);
  pm[0] = {1.0L};
  if (p >= 1) pm[1] = {0.0L, 1.0L};
  for (int j = 1; j < p; ++j) {
    std::vector<ld> nx(j + 2, 0.0L);
    for (int i = 0; i <= j; ++i) nx[i + 1] += pm[j][i];
    const ld e = (ld)(j * j) / (ld)(4 * j * j - 1);
    for (int i = 0; i < j; ++i) nx[i] -= e * pm[j - 1][i];
    pm[j + 1] = nx;
  }
  ld lead = 1.0L;  // (2m)! / (2^m m!^2)
  for (int m = 0; m <= p; ++m) {
    if (m > 0) lead *= (ld)(2 * m - 1) / (ld)m;
    const int K = p - m;
    const ld a = 2.0L * m + 1.0L;
    std::vector<std::vector<ld>> jac(K + 1);
    jac[0] = {1.0L};
    if (K >= 1) jac[1] = {0.5L * a, 0.5L * (a + 2.0L)};
    for (int k = 2; k <= K; ++k) {
      const ld c1 = 2.0L * k + a - 1.0L, c2 = (2.0L * k + a) * (2.0L * k + a - 2.0L);
      const ld c3 = 2.0L * (k + a - 1.0L) * (k - 1.0L) * (2.0L * k + a);
      const ld inv = 1.0L / (2.0L * k * (k + a) * (2.0L * k + a - 2.0L));
      std::vector<ld> nx(k + 1, 0.0L);
      for (int i = 0; i < k; ++i) {
        nx[i + 1] += c1 * c2 * jac[k - 1][i] * inv;
        nx[i] += c1 * a * a * jac[k - 1][i] * inv;
      }
      for (int i = 0; i < k - 1; ++i) nx[i] -= c3 * jac[k - 2][i] * inv;
      jac[k] = nx;
    }
    for (int k = 0; k <= K; ++k) {
      const ld c = std::sqrt((ld)(2 * (2 * m + 1) * (m + k + 1))) * lead;
      std::vector<ld> rem = jac[k];
      for (int j = k; j >= 0; --j) {
        const ld cj = rem[j];
        for (int i = 0; i <= j; ++i) rem[i] -= cj * pm[j][i];
        const int n = m + k;
        g[(size_t)(n * (n + 1) / 2 + m) * (p + 1) + j] = (double)(c * cj);
      }
    }
  }
  return g;
}

// The rules depend on their order alone and every plan asks for several of
// them (0.4 ms of host time for the 16 x 16 collapsed rule): each is computed
// once per process and copied out afterwards.
namespace {
// one table (and lock) per rule function
template <class R, R (*Make)(int)>
R memo(int n) {
  static std::mutex mu;
  static std::map<int, R> done;
  std::lock_guard<std::mutex> lock(mu);
  auto it = done.find(n);
  if (it == done.end()) it = done.emplace(n, Make(n)).first;
  return it->second;
}
}  // namespace

Rule1D gauss_legendre01(int n) { return memo<Rule1D, gauss_legendre01_compute>(n); }
Rule1D gauss_log01(int n) { return memo<Rule1D, gauss_log01_compute>(n); }
Rule2D collapsed_gauss(int q) { return memo<Rule2D, collapsed_gauss_compute>(q); }
Rule2D interp_nodes(int p) { return memo<Rule2D, interp_nodes_compute>(p); }

}  // namespace vp

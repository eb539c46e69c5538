// CMA-ES search of Robin transmission coefficients (Sec. 4) on the Fourier
// convergence factor of the two-subdomain Schwarz iteration (Sec. 3).
//
// Cost: rho_max = max over k in [kmin, kmax] (n_k uniform samples) of
//   |(k - L1)(k - L2)| / ((k + L1)(k + L2)),  L_s = p_s + q_s k^2.
// Search space: the logarithms of the free coefficients (they must stay
// positive). The evolution strategy follows the standard (mu/mu_w, lambda)
// CMA-ES: a multivariate normal search distribution N(m, sigma^2 C);
// lambda samples per generation; the mu best recombined with log-decreasing
// weights into the new mean; cumulative step-size adaptation of sigma from
// the conjugate evolution path; covariance adaptation from the evolution path
// (information of previous generations: rank-one update) and from the current
// generation (rank-mu update). Host code only, deterministic for a seed.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/sos.h"

namespace {

struct Rng {  // splitmix64 + Box-Muller
  uint64_t s;
  double spare = 0.0;
  bool has = false;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    if (has) {
      has = false;
      return spare;
    }
    const double u = uniform(), v = uniform();
    const double r = std::sqrt(-2.0 * std::log(u));
    spare = r * std::sin(2.0 * M_PI * v);
    has = true;
    return r * std::cos(2.0 * M_PI * v);
  }
};

// Symmetric eigen-decomposition (cyclic Jacobi) of an n x n matrix, n <= 4.
void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = std::max(A[i * n + i], 1e-300);
}

// Coefficients (p1, q1, p2, q2) of a search point for the given kind.
void unpack(int kind, const double* y, double* pq) {
  switch (kind) {
    case 0: pq[0] = pq[2] = std::exp(y[0]); pq[1] = pq[3] = 0.0; break;
    case 1: pq[0] = std::exp(y[0]); pq[2] = std::exp(y[1]); pq[1] = pq[3] = 0.0; break;
    case 2: pq[0] = pq[2] = std::exp(y[0]); pq[1] = pq[3] = std::exp(y[1]); break;
    default: pq[0] = std::exp(y[0]); pq[1] = std::exp(y[1]); pq[2] = std::exp(y[2]); pq[3] = std::exp(y[3]); break;
  }
}

double rho_max(const double* pq, const std::vector<double>& ks) {
  double m = 0.0;
  for (double k : ks) {
    const double l1 = pq[0] + pq[1] * k * k, l2 = pq[2] + pq[3] * k * k;
    const double r = std::fabs((k - l1) * (k - l2)) / ((k + l1) * (k + l2));
    m = std::max(m, r);
  }
  return m;
}

}  // namespace

extern "C" int sos_optimize_robin(int32_t kind, double kmin, double kmax, int32_t n_k, int32_t popsize,
                                  int32_t max_iter, double tol, uint64_t seed, double* pq_out, double* rho_out,
                                  int32_t* iters_out) {
  if (kind < 0 || kind > 3 || !(kmin > 0.0) || !(kmax > kmin) || n_k < 2 || popsize < 4 || max_iter < 1 ||
      !(tol > 0.0) || !pq_out || !rho_out)
    return SOS_EINVAL;
  const int N = kind == 0 ? 1 : (kind == 3 ? 4 : 2);
  std::vector<double> ks(n_k);
  for (int i = 0; i < n_k; ++i) ks[i] = kmin + (kmax - kmin) * i / (n_k - 1);
  // initial distribution: p around sqrt(kmin kmax) (the zeroth-order optimum),
  // q around 1/sqrt(kmin kmax); sigma of one decade in log space
  const double p0 = std::log(std::sqrt(kmin * kmax)), q0 = -p0;
  std::vector<double> m(N);
  if (kind == 0) m = {p0};
  else if (kind == 1) m = {p0, p0};
  else if (kind == 2) m = {p0, q0};
  else m = {p0, q0, p0, q0};
  double sigma = std::log(10.0);
  const int lam = popsize, mu = lam / 2;
  std::vector<double> wts(mu);
  for (int i = 0; i < mu; ++i) wts[i] = std::log(mu + 0.5) - std::log(i + 1.0);
  const double wsum = std::accumulate(wts.begin(), wts.end(), 0.0);
  double w2 = 0.0;
  for (auto& v : wts) {
    v /= wsum;
    w2 += v * v;
  }
  const double mueff = 1.0 / w2;
  const double cc = (4.0 + mueff / N) / (N + 4.0 + 2.0 * mueff / N);
  const double cs = (mueff + 2.0) / (N + mueff + 5.0);
  const double c1 = 2.0 / ((N + 1.3) * (N + 1.3) + mueff);
  const double cmu = std::min(1.0 - c1, 2.0 * (mueff - 2.0 + 1.0 / mueff) / ((N + 2.0) * (N + 2.0) + mueff));
  const double damps = 1.0 + 2.0 * std::max(0.0, std::sqrt((mueff - 1.0) / (N + 1.0)) - 1.0) + cs;
  const double chiN = std::sqrt((double)N) * (1.0 - 1.0 / (4.0 * N) + 1.0 / (21.0 * N * N));
  std::vector<double> pc(N, 0.0), ps(N, 0.0), C(N * N, 0.0), B, D, BD(N * N);
  for (int i = 0; i < N; ++i) C[i * N + i] = 1.0;
  Rng rng{seed ? seed : 1};
  std::vector<double> z(lam * N), y(lam * N), x(lam * N), f(lam);
  std::vector<int> idx(lam);
  double best = INFINITY, best_prev = INFINITY;
  std::vector<double> best_x(m);
  int it = 0, stall = 0;
  for (it = 1; it <= max_iter; ++it) {
    jacobi_eigen(N, C, D, B);
    for (int i = 0; i < N; ++i) D[i] = std::sqrt(D[i]);
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < N; ++c) BD[r * N + c] = B[r * N + c] * D[c];
    for (int k = 0; k < lam; ++k) {
      for (int i = 0; i < N; ++i) z[k * N + i] = rng.normal();
      for (int r = 0; r < N; ++r) {
        double s = 0.0;
        for (int c = 0; c < N; ++c) s += BD[r * N + c] * z[k * N + c];
        y[k * N + r] = s;
        x[k * N + r] = m[r] + sigma * s;
      }
      double pq[4];
      unpack(kind, &x[k * N], pq);
      f[k] = rho_max(pq, ks);
    }
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return f[a] < f[b]; });
    if (f[idx[0]] < best) {
      best = f[idx[0]];
      best_x.assign(&x[idx[0] * N], &x[idx[0] * N] + N);
    }
    // recombination
    std::vector<double> yw(N, 0.0), zw(N, 0.0);
    for (int i = 0; i < mu; ++i)
      for (int d = 0; d < N; ++d) {
        yw[d] += wts[i] * y[idx[i] * N + d];
        zw[d] += wts[i] * z[idx[i] * N + d];
      }
    for (int d = 0; d < N; ++d) m[d] += sigma * yw[d];
    // conjugate evolution path: C^-1/2 yw = B zw
    double psn = 0.0;
    for (int r = 0; r < N; ++r) {
        double s = 0.0;
        for (int c = 0; c < N; ++c) s += B[r * N + c] * zw[c];
        ps[r] = (1.0 - cs) * ps[r] + std::sqrt(cs * (2.0 - cs) * mueff) * s;
        psn += ps[r] * ps[r];
    }
    psn = std::sqrt(psn);
    const double hs = psn / std::sqrt(1.0 - std::pow(1.0 - cs, 2.0 * it)) < (1.4 + 2.0 / (N + 1.0)) * chiN ? 1.0 : 0.0;
    for (int d = 0; d < N; ++d) pc[d] = (1.0 - cc) * pc[d] + hs * std::sqrt(cc * (2.0 - cc) * mueff) * yw[d];
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < N; ++c) {
        double rank_mu = 0.0;
        for (int i = 0; i < mu; ++i) rank_mu += wts[i] * y[idx[i] * N + r] * y[idx[i] * N + c];
        C[r * N + c] = (1.0 - c1 - cmu) * C[r * N + c] + c1 * (pc[r] * pc[c] + (1.0 - hs) * cc * (2.0 - cc) * C[r * N + c]) +
                       cmu * rank_mu;
      }
    sigma *= std::exp((cs / damps) * (psn / chiN - 1.0));
    // stop: the distribution has collapsed, or the best cost stopped moving
    double spread = 0.0;
    for (int d = 0; d < N; ++d) spread = std::max(spread, sigma * std::sqrt(C[d * N + d]));
    stall = (best_prev - best < tol) ? stall + 1 : 0;
    best_prev = best;
    if (spread < tol || stall > 10 * (N + 1)) break;
  }
  unpack(kind, best_x.data(), pq_out);
  *rho_out = best;
  if (iters_out) *iters_out = std::min(it, max_iter);
  return SOS_OK;
}

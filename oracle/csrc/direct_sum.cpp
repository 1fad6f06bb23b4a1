// Direct-summation FP64 fields of point charges and point dipoles on all host cores.
//
// TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Only tests, the smoke check and the benchmark's
// CPU-baseline leg load it (through oracle/native.py).  It shares no code, header or table with the
// HIP library.
//
// What it computes is the plain definition of Sec. II.A, summed over every source j != i:
//   potential        phi_i  = sum_j q_j / r  +  mu_j . r / r^3              (r = x_i - x_j)
//   static field     E^q_i  = sum_j q_j r / r^3
//   dipole field     E^mu_i = sum_j H(r) mu_j, H the Hessian of the interaction kernel g(r):
//                    g = 1/r for the undamped field (what acts on charges), and for the field
//                    acting on dipoles the Thole linear (cone) smearing of radius
//                    s_ij = a (alpha_i alpha_j)^(1/6): g = (2 - 2v^2 + v^3)/s for v = r/s < 1
//   field gradient   G_i[a][b] = d_a E_b: -q_j H_ab(r) for charges, sum_c T3_abc mu_j,c for dipoles
//                    (damped), T3 the third derivatives of g.
// With u = r/|r| and the radial derivatives g', g'', g''' of g:
//   H_ab    = (g'' - g'/r) u_a u_b + (g'/r) delta_ab
//   T3_abc  = (g''' - 3 g''/r + 3 g'/r^2) u_a u_b u_c + (g''/r - g'/r^2)(delta_ab u_c + delta_ac u_b + delta_bc u_a)
//
// Summation: each target is summed over blocks of sources; the plain partial sum of a block is added
// to the target's total with Neumaier's compensated summation, so the rounding of a total grows
// with the number of blocks only through the compensated error term.  Targets are spread over the
// OpenMP threads in chunks; each chunk walks the sources block by block so that a block stays in
// cache while the chunk's targets use it.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

constexpr int64_t SRC_BLOCK = 512;  // sources per block
constexpr int64_t TGT_CHUNK = 32;   // targets per chunk

// Neumaier's variant of Kahan summation.
struct Compensated {
  double s = 0.0, c = 0.0;
  void add(double x) {
    const double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// Radial derivatives g', g'', g''' of the interaction kernel at distance r (1/r, or the Thole cone
// potential when r < s).
inline void radial(double r, double rinv, double s, double& g1, double& g2, double& g3) {
  if (s > 0.0 && r < s) {
    const double v = r / s, is = 1.0 / s, is2 = is * is;
    g1 = (-4.0 * v + 3.0 * v * v) * is2;
    g2 = (-4.0 + 6.0 * v) * is2 * is;
    g3 = 6.0 * is2 * is2;
  } else {
    const double ri2 = rinv * rinv;
    g1 = -ri2;
    g2 = 2.0 * ri2 * rinv;
    g3 = -6.0 * ri2 * ri2;
  }
}

struct Sources {
  std::vector<double> x, y, z, q, mx, my, mz, tau;
  bool has_q = false, has_mu = false;
  Sources(int64_t n, const double* X, const double* qq, const double* mu, const double* alpha) {
    x.resize(n); y.resize(n); z.resize(n); tau.resize(n);
    for (int64_t j = 0; j < n; ++j) {
      x[j] = X[3 * j]; y[j] = X[3 * j + 1]; z[j] = X[3 * j + 2];
      tau[j] = alpha ? std::cbrt(std::sqrt(alpha[j])) : 0.0;  // alpha^(1/6)
    }
    if (qq) {
      has_q = true;
      q.assign(qq, qq + n);
    }
    if (mu) {
      has_mu = true;
      mx.resize(n); my.resize(n); mz.resize(n);
      for (int64_t j = 0; j < n; ++j) { mx[j] = mu[3 * j]; my[j] = mu[3 * j + 1]; mz[j] = mu[3 * j + 2]; }
    }
  }
};

// Outputs of one target: phi, Eu[3], Ed[3], G[9].
constexpr int NOUT = 16;

// Adds the plain sum over sources [j0, j1) at target i to acc[0..NOUT).
void block_full(const Sources& S, double thole_a, int64_t i, int64_t j0, int64_t j1, double* acc, int* coincident) {
  const double xi = S.x[i], yi = S.y[i], zi = S.z[i], ti = S.tau[i];
  for (int64_t j = j0; j < j1; ++j) {
    if (j == i) continue;
    const double rx = xi - S.x[j], ry = yi - S.y[j], rz = zi - S.z[j];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) {
      *coincident = 1;
      continue;
    }
    const double rinv = 1.0 / std::sqrt(r2), r = r2 * rinv;
    const double u[3] = {rx * rinv, ry * rinv, rz * rinv};
    // undamped kernel 1/r
    double g1, g2, g3;
    radial(r, rinv, 0.0, g1, g2, g3);
    const double Huu = g2 - g1 * rinv, HI = g1 * rinv;
    if (S.has_q) {
      const double qj = S.q[j];
      acc[0] += qj * rinv;
      for (int a = 0; a < 3; ++a) {
        const double e = -qj * g1 * u[a];  // E = -q grad g
        acc[1 + a] += e;
        acc[4 + a] += e;
      }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[7 + 3 * a + b] -= qj * (Huu * u[a] * u[b] + (a == b ? HI : 0.0));
    }
    if (S.has_mu) {
      const double m[3] = {S.mx[j], S.my[j], S.mz[j]};
      const double um = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
      acc[0] -= g1 * um;  // -mu . grad g
      for (int a = 0; a < 3; ++a) acc[1 + a] += Huu * u[a] * um + HI * m[a];
      // damped kernel for the field on dipoles and its gradient
      const double s = thole_a * ti * S.tau[j];
      double d1, d2, d3;
      radial(r, rinv, s, d1, d2, d3);
      const double Duu = d2 - d1 * rinv, DI = d1 * rinv;
      for (int a = 0; a < 3; ++a) acc[4 + a] += Duu * u[a] * um + DI * m[a];
      const double A = d3 - 3.0 * d2 * rinv + 3.0 * d1 * rinv * rinv;
      const double B = d2 * rinv - d1 * rinv * rinv;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          acc[7 + 3 * a + b] += A * u[a] * u[b] * um + B * ((a == b ? um : 0.0) + u[a] * m[b] + u[b] * m[a]);
    }
  }
}

// Damped dipole field only (the matrix-vector product of the dipole solve).
void block_dipole(const Sources& S, double thole_a, int64_t i, int64_t j0, int64_t j1, double* acc) {
  const double xi = S.x[i], yi = S.y[i], zi = S.z[i], ti = S.tau[i];
  double ex = 0.0, ey = 0.0, ez = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    if (j == i) continue;
    const double rx = xi - S.x[j], ry = yi - S.y[j], rz = zi - S.z[j];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) continue;  // coincident pair: orc_fields reports it
    const double rinv = 1.0 / std::sqrt(r2), r = r2 * rinv;
    const double ux = rx * rinv, uy = ry * rinv, uz = rz * rinv;
    const double s = thole_a * ti * S.tau[j];
    double d1, d2, d3;
    radial(r, rinv, s, d1, d2, d3);
    const double Duu = d2 - d1 * rinv, DI = d1 * rinv;
    const double um = ux * S.mx[j] + uy * S.my[j] + uz * S.mz[j];
    ex += Duu * ux * um + DI * S.mx[j];
    ey += Duu * uy * um + DI * S.my[j];
    ez += Duu * uz * um + DI * S.mz[j];
  }
  acc[0] += ex;
  acc[1] += ey;
  acc[2] += ez;
}

}  // namespace

extern "C" {

// Number of OpenMP threads the sums run on.
int orc_threads(void) { return omp_get_max_threads(); }

// Fields of the sources (charges q and/or point dipoles mu; either may be NULL) at m targets
// (targets = NULL: every particle, m = n).  X is n x 3; alpha (n, or NULL = no damping) sets the
// Thole radii.  Outputs per target: phi (m), Eu (m x 3; dipole part undamped), Ed (m x 3; dipole
// part damped), G (m x 9, row-major d_a (Ed)_b).  Returns 0, 1 (bad argument) or 3 (two particles
// at the same position).
int orc_fields(int64_t n, const double* X, const double* q, const double* mu, const double* alpha, double thole_a,
               int64_t m, const int64_t* targets, double* phi, double* Eu, double* Ed, double* G) {
  if (n < 0 || m < 0 || !X || !phi || !Eu || !Ed || !G) return 1;
  if (!targets && m != n) return 1;
  for (int64_t k = 0; k < m && targets; ++k)
    if (targets[k] < 0 || targets[k] >= n) return 1;
  const Sources S(n, X, q, mu, alpha);
  int coincident = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : coincident)
  for (int64_t c0 = 0; c0 < m; c0 += TGT_CHUNK) {
    const int64_t c1 = std::min(m, c0 + TGT_CHUNK);
    std::vector<Compensated> tot((size_t)(c1 - c0) * NOUT);
    for (int64_t j0 = 0; j0 < n; j0 += SRC_BLOCK) {
      const int64_t j1 = std::min(n, j0 + SRC_BLOCK);
      for (int64_t k = c0; k < c1; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double acc[NOUT] = {};
        block_full(S, thole_a, i, j0, j1, acc, &coincident);
        for (int o = 0; o < NOUT; ++o) tot[(size_t)(k - c0) * NOUT + o].add(acc[o]);
      }
    }
    for (int64_t k = c0; k < c1; ++k) {
      const Compensated* t = &tot[(size_t)(k - c0) * NOUT];
      phi[k] = t[0].value();
      for (int a = 0; a < 3; ++a) {
        Eu[3 * k + a] = t[1 + a].value();
        Ed[3 * k + a] = t[4 + a].value();
      }
      for (int a = 0; a < 9; ++a) G[9 * k + a] = t[7 + a].value();
    }
  }
  return coincident ? 3 : 0;
}

// Damped field of the point dipoles mu (n x 3) at m targets (targets = NULL: every particle, m = n):
// Ed = T~ mu, the product the dipole solve iterates on.  Returns 0 or 1 (bad argument).
int orc_dipole_field(int64_t n, const double* X, const double* alpha, double thole_a, const double* mu, int64_t m,
                     const int64_t* targets, double* Ed) {
  if (n < 0 || m < 0 || !X || !mu || !Ed) return 1;
  if (!targets && m != n) return 1;
  for (int64_t k = 0; k < m && targets; ++k)
    if (targets[k] < 0 || targets[k] >= n) return 1;
  const Sources S(n, X, nullptr, mu, alpha);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c0 = 0; c0 < m; c0 += TGT_CHUNK) {
    const int64_t c1 = std::min(m, c0 + TGT_CHUNK);
    std::vector<Compensated> tot((size_t)(c1 - c0) * 3);
    for (int64_t j0 = 0; j0 < n; j0 += SRC_BLOCK) {
      const int64_t j1 = std::min(n, j0 + SRC_BLOCK);
      for (int64_t k = c0; k < c1; ++k) {
        double acc[3] = {};
        block_dipole(S, thole_a, targets ? targets[k] : k, j0, j1, acc);
        for (int o = 0; o < 3; ++o) tot[(size_t)(k - c0) * 3 + o].add(acc[o]);
      }
    }
    for (int64_t k = c0; k < c1; ++k)
      for (int o = 0; o < 3; ++o) Ed[3 * k + o] = tot[(size_t)(k - c0) * 3 + o].value();
  }
  return 0;
}

}  // extern "C"

// Induced-dipole solve, energy/force assembly and the adjoint backward (Sec. II.A and Sec. III).
//
// The dipole equation mu = alpha (E^q + T~ mu) is solved in the symmetric scaled form
//   (I - S T~ S) y = S E^q,   mu = S y,   S = diag(sqrt(alpha)),
// by conjugate gradients (the paper iterates the dipoles but gives the scheme elsewhere; plain
// fixed-point iteration diverges at protein densities).  Vectors are float64 in Morton order; dot
// products are two-stage block reductions in a fixed order, so results are deterministic.  All
// scalars live on the device (CGState); every kernel of an iteration returns at once when the
// `done` flag is set, so iterations can be enqueued ahead of the convergence test.
#include "kernels.hpp"

namespace pfmm {

namespace {

constexpr int TPB = 256;

template <int K>
__device__ inline void block_sum(double (&v)[K], double* part) {
  __shared__ double red[K][TPB];
  for (int k = 0; k < K; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < K) part[blockIdx.x * K + threadIdx.x] = red[threadIdx.x][0];
}

template <int K>
__device__ inline void finish_sum(const double* part, int nblk, double (&out)[K]) {
  __shared__ double red[K][TPB];
  double v[K];
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB)
    for (int k = 0; k < K; ++k) v[k] += part[b * K + k];
  for (int k = 0; k < K; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  for (int k = 0; k < K; ++k) out[k] = red[k][0];
}

#define GRID_STRIDE(i, n) \
  for (int i = blockIdx.x * TPB + threadIdx.x; i < (n); i += gridDim.x * TPB)

// y0 = S E^q (or the warm start mu0 / S), dipoles for the first matvec, ||alpha E^q||^2.
// mu_warm may alias mu4 (each thread reads its own entry before writing it).
__global__ __launch_bounds__(TPB) void k_cg_init(Particles pa, const double* __restrict__ Eq,
                                                 const double4* mu_warm, int warm,
                                                 double* __restrict__ y, double* __restrict__ pv,
                                                 double4* mu4, double* __restrict__ part) {
  double v[1] = {0.0};
  GRID_STRIDE(i, pa.n) {
    const double s = pa.sqa[i], a = pa.alpha[i];
    double yi[3];
    for (int c = 0; c < 3; ++c) {
      const double e = Eq[3 * i + c];
      v[0] += a * a * e * e;
      if (warm) {
        const double m = c == 0 ? mu_warm[i].x : (c == 1 ? mu_warm[i].y : mu_warm[i].z);
        yi[c] = s > 0.0 ? m / s : 0.0;
      } else {
        yi[c] = s * e;
      }
      y[3 * i + c] = yi[c];
      pv[3 * i + c] = yi[c];
    }
    mu4[i] = make_double4(s * yi[0], s * yi[1], s * yi[2], pa.tau[i]);
  }
  block_sum<1>(v, part);
}

__global__ __launch_bounds__(TPB) void k_cg_init_finish(const double* part, int nblk, CGState* st) {
  double o[1];
  finish_sum<1>(part, nblk, o);
  if (threadIdx.x == 0) {
    st->bnorm2 = o[0];
    st->done = 0; st->iters = 0; st->notspd = 0; st->maxed = 0;
    st->rr = st->pAp = st->a = st->b = 0.0;
    st->res = 0.0;
  }
}

// Cold start of the preconditioned solve: y0 = 0, r0 = S E^q (no field evaluation needed),
// ||alpha E^q||^2, r.r; the residual is 1 (or the solve is done when E^q = 0).
__global__ __launch_bounds__(TPB) void k_cg_init_zero(Particles pa, const double* __restrict__ Eq,
                                                      double* __restrict__ y, double* __restrict__ r,
                                                      double* __restrict__ part) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, pa.n) {
    const double s = pa.sqa[i], a = pa.alpha[i];
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      const double e = Eq[k];
      y[k] = 0.0;
      r[k] = s * e;
      v[0] += a * a * e * e;
      v[1] += a * e * e;
    }
  }
  block_sum<2>(v, part);
}
__global__ __launch_bounds__(TPB) void k_cg_init_zero_finish(const double* part, int nblk, CGState* st,
                                                             double tol) {
  double o[2];
  finish_sum<2>(part, nblk, o);
  if (threadIdx.x == 0) {
    st->bnorm2 = o[0];
    st->done = 0; st->iters = 0; st->notspd = 0; st->maxed = 0;
    st->rr = o[1];
    st->pAp = st->a = st->b = 0.0;
    st->res = o[0] > 0.0 ? 1.0 : 0.0;
    if (o[0] == 0.0 || st->res <= tol) st->done = 1;
  }
}

// r0 = S E^q - (y0 - S E(S y0)); p0 = r0; rr = r.r; residual in dipole units.
__global__ __launch_bounds__(TPB) void k_cg_res0(Particles pa, const double* __restrict__ Eq,
                                                 const double* __restrict__ E, double* __restrict__ y,
                                                 double* __restrict__ r, double* __restrict__ pv,
                                                 double* __restrict__ part) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, pa.n) {
    const double s = pa.sqa[i], a = pa.alpha[i];
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      const double rk = s * Eq[k] - (y[k] - s * E[k]);
      r[k] = rk;
      pv[k] = rk;
      v[0] += rk * rk;
      v[1] += a * rk * rk;
    }
  }
  block_sum<2>(v, part);
}

__global__ __launch_bounds__(TPB) void k_cg_res0_finish(const double* part, int nblk, CGState* st,
                                                        double tol) {
  double o[2];
  finish_sum<2>(part, nblk, o);
  if (threadIdx.x == 0) {
    st->rr = o[0];
    st->res = st->bnorm2 > 0.0 ? sqrt(o[1] / st->bnorm2) : 0.0;
    if (st->bnorm2 == 0.0 || st->res <= tol) st->done = 1;
  }
}

__global__ __launch_bounds__(TPB) void k_make_dipoles(Particles pa, const double* __restrict__ v,
                                                      double4* __restrict__ mu4, const int* done) {
  if (done && *done) return;
  GRID_STRIDE(i, pa.n) {
    const double s = pa.sqa[i];
    mu4[i] = make_double4(s * v[3 * i], s * v[3 * i + 1], s * v[3 * i + 2], pa.tau[i]);
  }
}

// Ap = p - S E(S p); partial p.Ap
__global__ __launch_bounds__(TPB) void k_cg_ap(Particles pa, const double* __restrict__ pv,
                                               const double* __restrict__ E, double* __restrict__ Ap,
                                               double* __restrict__ part, const CGState* st) {
  if (st->done) return;
  double v[1] = {0.0};
  GRID_STRIDE(i, pa.n) {
    const double s = pa.sqa[i];
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      const double a = pv[k] - s * E[k];
      Ap[k] = a;
      v[0] += pv[k] * a;
    }
  }
  block_sum<1>(v, part);
}

__global__ __launch_bounds__(TPB) void k_cg_ap_finish(const double* part, int nblk, CGState* st) {
  if (st->done) return;
  double o[1];
  finish_sum<1>(part, nblk, o);
  if (threadIdx.x == 0) {
    st->pAp = o[0];
    if (!(o[0] > 0.0)) {
      st->notspd = 1;
      st->done = 1;
    } else {
      st->a = st->rr / o[0];
    }
  }
}

// y += a p; r -= a Ap; partial r.r and sum alpha |r|^2
__global__ __launch_bounds__(TPB) void k_cg_update(Particles pa, double* __restrict__ y,
                                                   double* __restrict__ r,
                                                   const double* __restrict__ pv,
                                                   const double* __restrict__ Ap,
                                                   double* __restrict__ part, const CGState* st) {
  if (st->done) return;
  const double a = st->a;
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, pa.n) {
    const double al = pa.alpha[i];
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      y[k] += a * pv[k];
      const double rk = r[k] - a * Ap[k];
      r[k] = rk;
      v[0] += rk * rk;
      v[1] += al * rk * rk;
    }
  }
  block_sum<2>(v, part);
}

__global__ __launch_bounds__(TPB) void k_cg_update_finish(const double* part, int nblk, CGState* st,
                                                          double tol, int max_iter, RelaxParams rp) {
  if (st->done) return;
  double o[2];
  finish_sum<2>(part, nblk, o);
  if (threadIdx.x == 0) {
    st->b = o[0] / st->rr;
    st->rr = o[0];
    st->iters += 1;
    st->res = st->bnorm2 > 0.0 ? sqrt(o[1] / st->bnorm2) : 0.0;
    if (rp.track) {
      // the evaluation of this iteration used st->qcap; choose the cap of the next one
      const int used = st->qcap;
      if (used >= 0 && used < 16) st->ncap[used] += 1;
      int q = rp.p;
      if (rp.start > 0.0 && st->res < rp.start) {
        const double lower = st->res > 0.0 ? floor(log(rp.start / st->res) / rp.lrho) : (double)rp.p;
        q = lower >= (double)(rp.p - rp.qmin) ? rp.qmin : rp.p - (int)lower;
      }
      st->qcap = q;
    }
    if (st->res <= tol) st->done = 1;
    else if (st->iters >= max_iter) { st->maxed = 1; st->done = 1; }
  }
}

__global__ __launch_bounds__(TPB) void k_cg_dir(int n3, const double* __restrict__ r,
                                                double* __restrict__ pv, const CGState* st) {
  if (st->done) return;
  const double b = st->b;
  // b = 0 starts a direction afresh (p may be unset then, e.g. on the cold-started solve)
  if (b == 0.0) {
    GRID_STRIDE(k, n3) pv[k] = r[k];
  } else {
    GRID_STRIDE(k, n3) pv[k] = r[k] + b * pv[k];
  }
}

// ---- preconditioned (flexible) conjugate gradients.  The preconditioner is a few inner CG
// iterations on (I - S T~_near S) z = r, T~_near the damped dipole tensor of the pairs closer than
// a cutoff; since the inner solve is not a fixed linear map, the outer iteration is the flexible
// variant with one-step orthogonalisation: a = p.r / p.q, b = -z.q / p.q, p <- z + b p (q = A p).

// q = p - S E(S p); partials p.q and p.r
__global__ __launch_bounds__(TPB) void k_pcg_ap(Particles pa, const double* __restrict__ pv,
                                                const double* __restrict__ E, const double* __restrict__ r,
                                                double* __restrict__ Ap, double* __restrict__ part,
                                                const CGState* st) {
  if (st->done) return;
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, pa.n) {
    const double s = pa.sqa[i];
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      const double a = pv[k] - s * E[k];
      Ap[k] = a;
      v[0] += pv[k] * a;
      v[1] += pv[k] * r[k];
    }
  }
  block_sum<2>(v, part);
}
__global__ __launch_bounds__(TPB) void k_pcg_ap_finish(const double* part, int nblk, CGState* st) {
  if (st->done) return;
  double o[2];
  finish_sum<2>(part, nblk, o);
  if (threadIdx.x == 0) {
    st->pAp = o[0];
    if (!(o[0] > 0.0)) {
      st->notspd = 1;
      st->done = 1;
    } else {
      st->a = o[1] / o[0];
    }
  }
}
// b = -z.q / p.q
__global__ __launch_bounds__(TPB) void k_pcg_zq(int n3, const double* __restrict__ z,
                                                const double* __restrict__ Ap, double* __restrict__ part,
                                                const CGState* st) {
  if (st->done) return;
  double v[1] = {0.0};
  GRID_STRIDE(k, n3) v[0] += z[k] * Ap[k];
  block_sum<1>(v, part);
}
__global__ __launch_bounds__(TPB) void k_pcg_zq_finish(const double* part, int nblk, CGState* st) {
  if (st->done) return;
  double o[1];
  finish_sum<1>(part, nblk, o);
  if (threadIdx.x == 0) st->b = -o[0] / st->pAp;
}
// inner solve start: z = 0, r_in = r, p_in = r, rr_in = r.r; the inner state is done at once
// when the outer one is
__global__ __launch_bounds__(TPB) void k_pc_init(int n3, const double* __restrict__ r,
                                                 double* __restrict__ z, double* __restrict__ ri,
                                                 double* __restrict__ pi, double* __restrict__ part,
                                                 const CGState* outer) {
  if (outer->done) return;
  double v[1] = {0.0};
  GRID_STRIDE(k, n3) {
    const double x = r[k];
    z[k] = 0.0;
    ri[k] = x;
    pi[k] = x;
    v[0] += x * x;
  }
  block_sum<1>(v, part);
}
__global__ __launch_bounds__(TPB) void k_pc_init_finish(const double* part, int nblk, CGState* inner,
                                                        const CGState* outer) {
  const int od = outer->done;  // not written by this kernel: the same value in every thread
  double o[1] = {0.0};
  if (!od) finish_sum<1>(part, nblk, o);
  if (threadIdx.x == 0) {
    inner->done = od;
    inner->rr = o[0];
    inner->bnorm2 = 1.0;
    inner->iters = 0; inner->notspd = 0; inner->maxed = 0;
    inner->pAp = inner->a = inner->b = inner->res = 0.0;
    if (!(o[0] > 0.0)) inner->done = 1;
  }
}

__device__ inline double m3(const double4& u, int c) { return c == 0 ? u.x : (c == 1 ? u.y : u.z); }

// Energies, forces, potentials; outputs un-permuted to the caller's order.
// Energies, forces and potentials at the converged dipoles (Sec. II.A), with the static field
// E^{qE} of the charges q^E that polarise the dipoles (Sec. III; fc.qE == nullptr: q^E = q and
// fc.E, fc.G are the Coulomb charges' own field):
//   U^qq = 1/2 sum q phi^q,  U^pol = sum |mu|^2/(2 alpha) - sum mu.E^{qE} - 1/2 sum mu.E^mu_d,
//   F_i = q_i E^q_i + qE_i E^mu_u,i + (mu_i.grad)(E^{qE} + E^mu_d)_i,
//   dU/dq_i = phi^q_i (+ phi^mu_i when q^E = q),  dU/dqE_i = phi^mu_i.
__global__ __launch_bounds__(TPB) void k_assemble(
    Particles pa, const int* __restrict__ perm, const double4* __restrict__ mu4,
    const double* __restrict__ phiq, const double* __restrict__ Eq, FieldCharges fc,
    const double* __restrict__ phim, const double* __restrict__ Eum, const double* __restrict__ Edm,
    const double* __restrict__ Gm, double k_e, double* __restrict__ mu_out, double* __restrict__ F_out,
    double* __restrict__ phi_out, double* __restrict__ phiE_out, double* __restrict__ F_s,
    double* __restrict__ phi_s, double* __restrict__ phiE_s, double* __restrict__ Etot_s,
    double* __restrict__ part) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  double vmax = 0.0;
  const bool sep = fc.qE != nullptr;
  GRID_STRIDE(i, pa.n) {
    const int o = perm[i];
    const double q = pa.P[i].w, a = pa.alpha[i];
    const double qe = sep ? fc.qE[i] : q;
    const double4 u = mu4[i];
    const double mu[3] = {u.x, u.y, u.z};
    v[0] += 0.5 * q * phiq[i];
    double mm = mu[0] * mu[0] + mu[1] * mu[1] + mu[2] * mu[2];
    if (a > 0.0) v[1] += 0.5 * mm / a;
    double G[6];
    for (int k = 0; k < 6; ++k) G[k] = fc.G[6 * i + k] + Gm[6 * i + k];
    // G as xx, yy, zz, xy, xz, yz; (mu.grad) E_b = sum_a mu_a d_a E_b
    const double gm[3] = {mu[0] * G[0] + mu[1] * G[3] + mu[2] * G[4],
                          mu[0] * G[3] + mu[1] * G[1] + mu[2] * G[5],
                          mu[0] * G[4] + mu[1] * G[5] + mu[2] * G[2]};
    double rl2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double eq = Eq[3 * i + c], ee = fc.E[3 * i + c], ed = Edm[3 * i + c], eu = Eum[3 * i + c];
      v[2] += mu[c] * ee;
      v[3] += mu[c] * ed;
      const double et = ee + ed;
      const double rc = a * et - mu[c];
      rl2 += rc * rc;
      v[5] += a * a * ee * ee;
      const double f = k_e * ((sep ? q * eq + qe * eu : q * (eq + eu)) + gm[c]);
      if (F_out) F_out[3 * o + c] = f;
      F_s[3 * i + c] = f;
      Etot_s[3 * i + c] = et;
      mu_out[3 * o + c] = mu[c];
    }
    v[4] += rl2;
    vmax = fmax(vmax, sqrt(rl2));
    const double ph = k_e * (sep ? phiq[i] : phiq[i] + phim[i]);
    phi_s[i] = ph;
    if (phi_out) phi_out[o] = ph;
    const double pe = k_e * phim[i];
    phiE_s[i] = pe;
    if (phiE_out) phiE_out[o] = pe;
  }
  block_sum<6>(v, part);
  __shared__ double mx[TPB];
  mx[threadIdx.x] = vmax;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[gridDim.x * 6 + blockIdx.x] = mx[0];
}

__global__ __launch_bounds__(TPB) void k_assemble_finish(const double* part, int nblk, EnergyParts* ep) {
  double o[6];
  finish_sum<6>(part, nblk, o);
  __shared__ double mx[TPB];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) m = fmax(m, part[nblk * 6 + b]);
  mx[threadIdx.x] = m;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ep->Uqq = o[0]; ep->Amu = o[1]; ep->muEq = o[2]; ep->muEd = o[3]; ep->res2 = o[4];
    ep->bn2 = o[5]; ep->resmax = mx[0];
  }
}

__global__ __launch_bounds__(TPB) void k_backward(Particles pa, const int* __restrict__ perm,
                                                  const double4* __restrict__ mu4,
                                                  const double* __restrict__ F_s,
                                                  const double* __restrict__ phi_s,
                                                  const double* __restrict__ Etot_s,
                                                  const double* __restrict__ phiE_s,
                                                  const double* __restrict__ dal, double k_e, double g,
                                                  double* __restrict__ gpos, double* __restrict__ gq,
                                                  double* __restrict__ gqE, double* __restrict__ ga) {
  GRID_STRIDE(i, pa.n) {
    const int o = perm[i];
    if (gpos)
      for (int c = 0; c < 3; ++c) gpos[3 * o + c] = -g * F_s[3 * i + c];
    if (gq) gq[o] = g * phi_s[i];
    if (gqE) gqE[o] = g * phiE_s[i];
    if (ga) {
      const double a = pa.alpha[i];
      const double4 u = mu4[i];
      double d;
      if (a > 0.0) {
        d = -(u.x * u.x + u.y * u.y + u.z * u.z) / (2.0 * a * a) + (dal ? dal[i] : 0.0);
      } else {
        const double ex = Etot_s[3 * i], ey = Etot_s[3 * i + 1], ez = Etot_s[3 * i + 2];
        d = -0.5 * (ex * ex + ey * ey + ez * ez);
      }
      ga[o] = g * k_e * d;
    }
  }
}

// Gradients of a loss L(mu) through the dipoles (the adjoint of the dipole equations, from the
// stationary problem of Sec. II.A): with lambda = A^-1 dL/dmu (A = diag(1/alpha) - T~),
//   dL/dx_i     = qE_i E^lambda_u,i + (lambda_i . grad)(E^qE + E^mu_d)_i + (mu_i . grad) E^lambda_d,i
//   dL/dqE_i    = -phi^lambda_i
//   dL/dalpha_i = (G_i + E^lambda_d,i) . E_i + b_i,   E = E^qE + E^mu_d,
// b_i the Thole term sum_j [lambda_i . dT~/ds mu_j + mu_i . dT~/ds lambda_j] ds_ij/dalpha_i, obtained
// from the Thole term of dU/dalpha (P2P mode 2, dal(m) = -sum_j m_i . dT~/ds m_j ds/dalpha_i) by
// polarisation: b = (dal(mu - c lambda) - dal(mu + c lambda)) / (2 c).  Gradients are written in the
// caller's particle order; G6 arrays are symmetric gradients (xx, yy, zz, xy, xz, yz).
__global__ __launch_bounds__(TPB) void k_backward_mu(
    Particles pa, const int* __restrict__ perm, const double4* __restrict__ mu4, const double4* __restrict__ lam4,
    const double* __restrict__ phil, const double* __restrict__ Eul, const double* __restrict__ Edl,
    const double* __restrict__ Gl, const double* __restrict__ Ge, const double* __restrict__ Gm,
    const double* __restrict__ Etot, const double* __restrict__ Gs, const double* __restrict__ qEs,
    const double* __restrict__ dalp, const double* __restrict__ dalm, double inv2c, double* __restrict__ gpos,
    double* __restrict__ gq, double* __restrict__ gqE, double* __restrict__ ga) {
  GRID_STRIDE(i, pa.n) {
    const int o = perm[i];
    const double qe = qEs ? qEs[i] : pa.P[i].w;
    if (gpos) {
      const double4 l = lam4[i], m = mu4[i];
      double A[6], B[6];
      for (int k = 0; k < 6; ++k) {
        A[k] = Ge[6 * i + k] + Gm[6 * i + k];
        B[k] = Gl[6 * i + k];
      }
      const double la[3] = {l.x * A[0] + l.y * A[3] + l.z * A[4], l.x * A[3] + l.y * A[1] + l.z * A[5],
                            l.x * A[4] + l.y * A[5] + l.z * A[2]};
      const double mb[3] = {m.x * B[0] + m.y * B[3] + m.z * B[4], m.x * B[3] + m.y * B[1] + m.z * B[5],
                            m.x * B[4] + m.y * B[5] + m.z * B[2]};
      for (int c = 0; c < 3; ++c) gpos[3 * o + c] = qe * Eul[3 * i + c] + la[c] + mb[c];
    }
    if (gq) gq[o] = qEs ? 0.0 : -phil[i];
    if (gqE) gqE[o] = -phil[i];
    if (ga) {
      double d = 0.0;
      for (int c = 0; c < 3; ++c) d += (Gs[3 * i + c] + Edl[3 * i + c]) * Etot[3 * i + c];
      if (dalp) d += (dalm[i] - dalp[i]) * inv2c;
      ga[o] = d;
    }
  }
}

// out = a[perm] as a sorted 3-vector per particle (caller order in, sorted order out)
__global__ __launch_bounds__(TPB) void k_permute_vec3(const int* __restrict__ perm, int n, const double* __restrict__ in,
                                                      double* __restrict__ out) {
  GRID_STRIDE(i, n) {
    const int o = perm[i];
    for (int c = 0; c < 3; ++c) out[3 * i + c] = in[3 * o + c];
  }
}

// plus/minus = (a.xyz +/- c b.xyz, a.w): the two dipole sets of the polarisation identity
__global__ __launch_bounds__(TPB) void k_dipole_pm(int n, const double4* __restrict__ a, const double4* __restrict__ b,
                                                   double c, double4* __restrict__ plus, double4* __restrict__ minus) {
  GRID_STRIDE(i, n) {
    const double4 u = a[i], v = b[i];
    plus[i] = make_double4(u.x + c * v.x, u.y + c * v.y, u.z + c * v.z, u.w);
    minus[i] = make_double4(u.x - c * v.x, u.y - c * v.y, u.z - c * v.z, u.w);
  }
}

// The tree of the polarisable sites (T^mu of Sec. III): the sites with alpha > 0 in the caller's
// order, compacted through an inclusive prefix sum of their flags, with zero charges (the dipole solve
// uses dipole sources only).
__global__ __launch_bounds__(TPB) void k_flag_polarisable(const double* __restrict__ alpha, int n, int* __restrict__ f) {
  GRID_STRIDE(i, n) { f[i] = alpha[i] > 0.0 ? 1 : 0; }
}
__global__ __launch_bounds__(TPB) void k_compact_sites(const int* __restrict__ scan, const double* __restrict__ pos,
                                                       const double* __restrict__ alpha, int n, int* __restrict__ idx,
                                                       double* __restrict__ spos, double* __restrict__ salpha,
                                                       double* __restrict__ sq) {
  GRID_STRIDE(i, n) {
    if (alpha[i] > 0.0) {
      const int k = scan[i] - 1;
      idx[k] = i;
      for (int c = 0; c < 3; ++c) spos[3 * k + c] = pos[3 * i + c];
      salpha[k] = alpha[i];
      sq[k] = 0.0;
    }
  }
}
// For the j-th particle of the site tree (sorted): its caller index comp[j] and its index in the
// sorted order of the full tree map[j] (inv = inverse permutation of the full tree).
__global__ __launch_bounds__(TPB) void k_site_maps(const int* __restrict__ perm_mu, const int* __restrict__ idx,
                                                   const int* __restrict__ inv, int m, int* __restrict__ comp,
                                                   int* __restrict__ map) {
  GRID_STRIDE(j, m) {
    const int o = idx[perm_mu[j]];
    comp[j] = o;
    map[j] = inv[o];
  }
}
// dst = (0, 0, 0, tau) everywhere, then the site tree's dipoles at their places in the full tree
__global__ __launch_bounds__(TPB) void k_zero_dipoles(int n, const double* __restrict__ tau, double4* __restrict__ dst) {
  GRID_STRIDE(i, n) { dst[i] = make_double4(0.0, 0.0, 0.0, tau[i]); }
}
__global__ __launch_bounds__(TPB) void k_scatter_dipoles(const int* __restrict__ map, int m, const double4* __restrict__ src,
                                                         double4* __restrict__ dst) {
  GRID_STRIDE(j, m) {
    const double4 u = src[j];
    const int i = map[j];
    dst[i] = make_double4(u.x, u.y, u.z, dst[i].w);
  }
}

__global__ __launch_bounds__(TPB) void k_unpermute_field(const int* __restrict__ perm, int n,
                                                         FieldOut src, double* __restrict__ phi,
                                                         double* __restrict__ E,
                                                         double* __restrict__ Ed,
                                                         double* __restrict__ G9) {
  GRID_STRIDE(i, n) {
    const int o = perm[i];
    if (phi) phi[o] = src.phi[i];
    for (int c = 0; c < 3; ++c) {
      if (E) E[3 * o + c] = src.Eu[3 * i + c];
      if (Ed) Ed[3 * o + c] = src.Ed[3 * i + c];
    }
    if (G9) {
      const double* g = src.G + 6 * (int64_t)i;
      const double full[9] = {g[0], g[3], g[4], g[3], g[1], g[5], g[4], g[5], g[2]};
      for (int k = 0; k < 9; ++k) G9[9 * (int64_t)o + k] = full[k];
    }
  }
}

__global__ __launch_bounds__(TPB) void k_permute_dipoles(const int* __restrict__ perm, int n,
                                                         const double* __restrict__ mu,
                                                         const double* __restrict__ tau,
                                                         double4* __restrict__ mu4) {
  GRID_STRIDE(i, n) {
    const int o = perm[i];
    mu4[i] = make_double4(mu[3 * o], mu[3 * o + 1], mu[3 * o + 2], tau[i]);
  }
}

// sorted copy of the field charges: PE = (x, y, z, qE) of each sorted particle, qEs = qE sorted
__global__ __launch_bounds__(TPB) void k_field_charges(const int* __restrict__ perm, int n,
                                                       const double4* __restrict__ P,
                                                       const double* __restrict__ qE,
                                                       double4* __restrict__ PE, double* __restrict__ qEs) {
  GRID_STRIDE(i, n) {
    const double e = qE[perm[i]];
    const double4 p = P[i];
    PE[i] = make_double4(p.x, p.y, p.z, e);
    qEs[i] = e;
  }
}

__global__ __launch_bounds__(TPB) void k_check_finite(const double* __restrict__ v, int64_t count,
                                                      int* flags) {
  int f = 0;
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < count; i += (int64_t)gridDim.x * TPB)
    if (!isfinite(v[i])) f = 1;
  if (f) atomicOr(flags, 1);
}

inline int grid(int64_t n) {
  int64_t g = (n + TPB - 1) / TPB;
  if (g < 1) g = 1;
  if (g > RED_BLOCKS) g = RED_BLOCKS;
  return (int)g;
}

}  // namespace

void launch_cg_init(const Particles& pa, const double* Eq, const double4* mu_warm, bool warm,
                    double* y, double* pvec, double4* mu4, double* part, CGState* st, hipStream_t s) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_cg_init, dim3(g), dim3(TPB), 0, s, pa, Eq, mu_warm, warm ? 1 : 0, y, pvec, mu4,
                     part);
  hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(TPB), 0, s, part, g, st);
  PFMM_LAUNCH_CHECK();
}

void launch_cg_residual0(const Particles& pa, const double* Eq, const double* E, double* y, double* r,
                         double* pvec, double* part, CGState* st, double tol, hipStream_t s) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_cg_res0, dim3(g), dim3(TPB), 0, s, pa, Eq, E, y, r, pvec, part);
  hipLaunchKernelGGL(k_cg_res0_finish, dim3(1), dim3(TPB), 0, s, part, g, st, tol);
  PFMM_LAUNCH_CHECK();
}

void launch_make_dipoles(const Particles& pa, const double* v, double4* mu4, const int* done,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_make_dipoles, dim3(grid(pa.n)), dim3(TPB), 0, s, pa, v, mu4, done);
  PFMM_LAUNCH_CHECK();
}

void launch_cg_ap(const Particles& pa, const double* pvec, const double* E, double* Ap, double* part,
                  CGState* st, hipStream_t s) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_cg_ap, dim3(g), dim3(TPB), 0, s, pa, pvec, E, Ap, part, st);
  hipLaunchKernelGGL(k_cg_ap_finish, dim3(1), dim3(TPB), 0, s, part, g, st);
  PFMM_LAUNCH_CHECK();
}

void launch_cg_update(const Particles& pa, double* y, double* r, const double* pvec, const double* Ap,
                      double* part, CGState* st, double tol, int max_iter, hipStream_t s,
                      const RelaxParams& rp) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(TPB), 0, s, pa, y, r, pvec, Ap, part, st);
  hipLaunchKernelGGL(k_cg_update_finish, dim3(1), dim3(TPB), 0, s, part, g, st, tol, max_iter, rp);
  PFMM_LAUNCH_CHECK();
}

void launch_cg_init_zero(const Particles& pa, const double* Eq, double* y, double* r, double* part,
                         CGState* st, double tol, hipStream_t s) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_cg_init_zero, dim3(g), dim3(TPB), 0, s, pa, Eq, y, r, part);
  hipLaunchKernelGGL(k_cg_init_zero_finish, dim3(1), dim3(TPB), 0, s, part, g, st, tol);
  PFMM_LAUNCH_CHECK();
}

void launch_pcg_ap(const Particles& pa, const double* pvec, const double* E, const double* r, double* Ap,
                   double* part, CGState* st, hipStream_t s) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_pcg_ap, dim3(g), dim3(TPB), 0, s, pa, pvec, E, r, Ap, part, st);
  hipLaunchKernelGGL(k_pcg_ap_finish, dim3(1), dim3(TPB), 0, s, part, g, st);
  PFMM_LAUNCH_CHECK();
}

void launch_pcg_zq(int n3, const double* z, const double* Ap, double* part, CGState* st, hipStream_t s) {
  const int g = grid(n3);
  hipLaunchKernelGGL(k_pcg_zq, dim3(g), dim3(TPB), 0, s, n3, z, Ap, part, st);
  hipLaunchKernelGGL(k_pcg_zq_finish, dim3(1), dim3(TPB), 0, s, part, g, st);
  PFMM_LAUNCH_CHECK();
}

void launch_pc_init(int n3, const double* r, double* z, double* ri, double* pi, double* part,
                    CGState* inner, const CGState* outer, hipStream_t s) {
  const int g = grid(n3);
  hipLaunchKernelGGL(k_pc_init, dim3(g), dim3(TPB), 0, s, n3, r, z, ri, pi, part, outer);
  hipLaunchKernelGGL(k_pc_init_finish, dim3(1), dim3(TPB), 0, s, part, g, inner, outer);
  PFMM_LAUNCH_CHECK();
}

void launch_cg_direction(int n3, const double* r, double* pvec, const CGState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir, dim3(grid(n3)), dim3(TPB), 0, s, n3, r, pvec, st);
  PFMM_LAUNCH_CHECK();
}

void launch_assemble(const Particles& pa, const int* perm, const double4* mu4, const double* phiq,
                     const double* Eq, const FieldCharges& fc, const double* phim, const double* Eum,
                     const double* Edm, const double* Gm, double k_e, double* mu_out, double* F_out,
                     double* phi_out, double* phiE_out, double* F_s, double* phi_s, double* phiE_s,
                     double* Etot_s, double* part, EnergyParts* ep, hipStream_t s) {
  const int g = grid(pa.n);
  hipLaunchKernelGGL(k_assemble, dim3(g), dim3(TPB), 0, s, pa, perm, mu4, phiq, Eq, fc, phim, Eum, Edm,
                     Gm, k_e, mu_out, F_out, phi_out, phiE_out, F_s, phi_s, phiE_s, Etot_s, part);
  hipLaunchKernelGGL(k_assemble_finish, dim3(1), dim3(TPB), 0, s, part, g, ep);
  PFMM_LAUNCH_CHECK();
}

void launch_backward(const Particles& pa, const int* perm, const double4* mu4, const double* F_s,
                     const double* phi_s, const double* Etot_s, const double* phiE_s, const double* dal_thole,
                     double k_e, double g, double* gpos, double* gq, double* gqE, double* galpha,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_backward, dim3(grid(pa.n)), dim3(TPB), 0, s, pa, perm, mu4, F_s, phi_s, Etot_s,
                     phiE_s, dal_thole, k_e, g, gpos, gq, gqE, galpha);
  PFMM_LAUNCH_CHECK();
}

void launch_backward_mu(const Particles& pa, const int* perm, const double4* mu4, const double4* lam4,
                        const FieldOut& lam, const double* Ge, const double* Gm, const double* Etot, const double* Gs,
                        const double* qEs, const double* dalp, const double* dalm, double inv2c, double* gpos,
                        double* gq, double* gqE, double* ga, hipStream_t s) {
  if (pa.n <= 0) return;
  hipLaunchKernelGGL(k_backward_mu, dim3(grid(pa.n)), dim3(TPB), 0, s, pa, perm, mu4, lam4, lam.phi, lam.Eu, lam.Ed,
                     lam.G, Ge, Gm, Etot, Gs, qEs, dalp, dalm, inv2c, gpos, gq, gqE, ga);
  PFMM_LAUNCH_CHECK();
}

void launch_permute_vec3(const int* perm, int n, const double* in, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute_vec3, dim3(grid(n)), dim3(TPB), 0, s, perm, n, in, out);
  PFMM_LAUNCH_CHECK();
}

void launch_dipole_pm(int n, const double4* a, const double4* b, double c, double4* plus, double4* minus,
                      hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_dipole_pm, dim3(grid(n)), dim3(TPB), 0, s, n, a, b, c, plus, minus);
  PFMM_LAUNCH_CHECK();
}

void launch_flag_polarisable(const double* alpha, int n, int* flags, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_flag_polarisable, dim3(grid(n)), dim3(TPB), 0, s, alpha, n, flags);
  PFMM_LAUNCH_CHECK();
}
void launch_compact_sites(const int* scan, const double* pos, const double* alpha, int n, int* idx, double* spos,
                          double* salpha, double* sq, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_compact_sites, dim3(grid(n)), dim3(TPB), 0, s, scan, pos, alpha, n, idx, spos, salpha, sq);
  PFMM_LAUNCH_CHECK();
}
void launch_site_maps(const int* perm_mu, const int* idx, const int* inv, int m, int* comp, int* map, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_site_maps, dim3(grid(m)), dim3(TPB), 0, s, perm_mu, idx, inv, m, comp, map);
  PFMM_LAUNCH_CHECK();
}
void launch_place_site_dipoles(const int* map, int m, const double4* src, int n, const double* tau, double4* dst,
                               hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_dipoles, dim3(grid(n)), dim3(TPB), 0, s, n, tau, dst);
  PFMM_LAUNCH_CHECK();
  if (m <= 0) return;
  hipLaunchKernelGGL(k_scatter_dipoles, dim3(grid(m)), dim3(TPB), 0, s, map, m, src, dst);
  PFMM_LAUNCH_CHECK();
}

void launch_field_charges(const int* perm, int n, const double4* P, const double* qE, double4* PE,
                          double* qEs, hipStream_t s) {
  hipLaunchKernelGGL(k_field_charges, dim3(grid(n)), dim3(TPB), 0, s, perm, n, P, qE, PE, qEs);
  PFMM_LAUNCH_CHECK();
}

void launch_unpermute_field(const int* perm, int n, const FieldOut& src, double* phi, double* E,
                            double* Ed, double* G9, hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute_field, dim3(grid(n)), dim3(TPB), 0, s, perm, n, src, phi, E, Ed, G9);
  PFMM_LAUNCH_CHECK();
}

void launch_permute_dipoles(const int* perm, int n, const double* mu_in, const double* tau,
                            double4* mu4, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_dipoles, dim3(grid(n)), dim3(TPB), 0, s, perm, n, mu_in, tau, mu4);
  PFMM_LAUNCH_CHECK();
}

void launch_check_finite(const double* v, int64_t count, int* flags, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_check_finite, dim3(grid(count)), dim3(TPB), 0, s, v, count, flags);
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

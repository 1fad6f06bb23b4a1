// Upward and downward passes of the Cartesian FMM (Sec. II.B-II.C) on level-scaled expansions:
//   P2M  M~_n = (-1)^|n|/n! sum_a [ q_a rho_a^n + (mu_a / w) . grad(rho^n)(rho_a) ],  rho = (x - z)/w
//        (point dipoles enter through the delta-l -> 0 limit of the +/- q^mu pair of Sec. II.C, or,
//        on request, as the pair itself: charges +/- |mu_a| / (2 dl) at rho_a +/- (dl / w) mu_a/|mu_a|)
//   M2M  M~_n(parent) = sum_{k <= n} xt^k/k! 2^-(|n|-|k|) M~_{n-k}(child)
//   L2L  F~_n(child) += sum_{|k| <= p-|n|} xt'^k/k! 2^-(|n|+1) F~_{n+k}(parent)
//   L2P  phi = (1/w) sum rho^n/n! F~_n,  E_c = -(1/w^2) sum rho^n/n! F~_{n+e_c},
//        d_a E_b = -(1/w^3) sum rho^n/n! F~_{n+e_a+e_b}
// with M~_n = M_n / w^|n| and F~_n = F_n w^(|n|+1) for the cell edge w of the level.
// All four are memory-bound; they run in float64 on both precision paths.
#include <utility>

#include "kernels.hpp"
#include "morton.hpp"
#include "schedule.hpp"

namespace pfmm {

namespace {

__device__ inline void cell_centre(const TreeView& t, int g, int level, double c[3], double& w) {
  const uint64_t k = t.key[g];
  w = ldexp(t.w, t.L - level);
  c[0] = t.origin[0] + ((double)compact3(k >> 2) + 0.5) * w;
  c[1] = t.origin[1] + ((double)compact3(k >> 1) + 0.5) * w;
  c[2] = t.origin[2] + ((double)compact3(k) + 0.5) * w;
}

constexpr int P2M_TPB = 128;
constexpr int P2M_CHUNK = 64;

// One block per leaf; particles staged in LDS with the powers of their scaled offsets, one thread
// per coefficient.  PAIR: each dipole enters as its pair of Sec. II.C, the charges +/- |mu| / (2 dl)
// at rho +/- (dl / w) mu/|mu|, staged as two more point charges after the particle's own charge (a
// zero dipole stages two zero charges); otherwise through the point-dipole term above.
template <bool PAIR, int PM>
__global__ __launch_bounds__(P2M_TPB) void k_p2m(TreeView t, OpTables op, Particles pa,
                                                 const double4* __restrict__ mu4, int sources, double pair_dl,
                                                 double* __restrict__ M, const int* done) {
  if (done && *done) return;
  __shared__ double pw[P2M_CHUNK][3][PM + 1];
  __shared__ double sq[P2M_CHUNK], sm[P2M_CHUNK][3];
  const int g = t.off[t.L] + blockIdx.x;
  const int first = t.first[g], cnt = t.count[g];
  double c[3], w;
  cell_centre(t, g, t.L, c, w);
  const double iw = 1.0 / w;
  const int p = op.p, nc = op.nc;
  constexpr int KPT = (mi_count(PM) + P2M_TPB - 1) / P2M_TPB;  // coefficients per thread at order PM
  double acc[KPT];
  int ex[KPT][3];
  for (int r = 0; r < KPT; ++r) {
    acc[r] = 0.0;
    const int k = threadIdx.x + r * P2M_TPB;
    for (int a = 0; a < 3; ++a) ex[r][a] = k < nc ? op.mi[3 * k + a] : 0;
  }
  auto stage = [&](int v, const double* rho) {
    for (int a = 0; a < 3; ++a) {
      double x = 1.0;
      pw[v][a][0] = 1.0;
      for (int e = 1; e <= p; ++e) { x *= rho[a]; pw[v][a][e] = x; }
    }
  };
  // staged points per particle and particles per chunk (PAIR requires dipole sources)
  const int per = PAIR ? ((sources & 1) ? 3 : 2) : 1;
  const int rc = P2M_CHUNK / per;
  for (int s0 = 0; s0 < cnt; s0 += rc) {
    const int m = min(rc, cnt - s0);
    if (threadIdx.x < m) {
      const int j = threadIdx.x;
      const double4 P = pa.P[first + s0 + j];
      const double rho[3] = {(P.x - c[0]) * iw, (P.y - c[1]) * iw, (P.z - c[2]) * iw};
      if (!PAIR) {
        stage(j, rho);
        sq[j] = (sources & 1) ? P.w : 0.0;
        if (sources & 2) {
          const double4 u = mu4[first + s0 + j];
          sm[j][0] = u.x * iw; sm[j][1] = u.y * iw; sm[j][2] = u.z * iw;
        } else {
          sm[j][0] = sm[j][1] = sm[j][2] = 0.0;
        }
      } else {
        int v = per * j;
        if (sources & 1) {
          stage(v, rho);
          sq[v++] = P.w;
        }
        const double4 u = mu4[first + s0 + j];
        const double nrm = sqrt(u.x * u.x + u.y * u.y + u.z * u.z);
        const double qm = nrm > 0.0 ? nrm / (2.0 * pair_dl) : 0.0;
        const double f = nrm > 0.0 ? pair_dl * iw / nrm : 0.0;
        const double rp[3] = {rho[0] + u.x * f, rho[1] + u.y * f, rho[2] + u.z * f};
        const double rm[3] = {rho[0] - u.x * f, rho[1] - u.y * f, rho[2] - u.z * f};
        stage(v, rp);
        sq[v] = qm;
        stage(v + 1, rm);
        sq[v + 1] = -qm;
      }
    }
    __syncthreads();
    const int mv = per * m;
    for (int r = 0; r < KPT; ++r) {
      const int k = threadIdx.x + r * P2M_TPB;
      if (k >= nc) break;
      const int nx = ex[r][0], ny = ex[r][1], nz = ex[r][2];
      double a = 0.0;
      for (int j = 0; j < mv; ++j) {
        const double X = pw[j][0][nx], Y = pw[j][1][ny], Z = pw[j][2][nz];
        double v = sq[j] * X * Y * Z;
        if (!PAIR) {
          if (nx) v += sm[j][0] * nx * pw[j][0][nx - 1] * Y * Z;
          if (ny) v += sm[j][1] * ny * X * pw[j][1][ny - 1] * Z;
          if (nz) v += sm[j][2] * nz * X * Y * pw[j][2][nz - 1];
        }
        a += v;
      }
      acc[r] += a;
    }
    __syncthreads();
  }
  for (int r = 0; r < KPT; ++r) {
    const int k = threadIdx.x + r * P2M_TPB;
    if (k < nc) M[(int64_t)g * op.stride + k] = op.p2m_coef[k] * acc[r];
    else if (k < op.stride) M[(int64_t)g * op.stride + k] = 0.0;
  }
}

constexpr int SH_TPB = 256;


// (h/4)^e / e! and (-h/4)^e / e! for e = 0..p: per-axis factors of the shift coefficients x^k / k!
// for a child centre offset of a quarter of the parent edge, times 2^e when h = 2
__device__ inline void shift_powers(double* plus, double* minus, int p, double h) {
  double v = 1.0;
  for (int e = 0; e <= p; ++e) {
    plus[e] = v;
    minus[e] = (e & 1) ? -v : v;
    v *= 0.25 * h / (double)(e + 1);
  }
}

// One block per parent cell:
//   M~_n(parent) = 2^-|n| sum_children sum_{k <= n} prod_a (2 xt_a)^{k_a} / k_a! M~_{n-k}(child),
// xt_a = +1/4 for octant bit 0 and -1/4 for bit 1 (parent centre minus child centre, in parent
// edges).  The shift coefficient factorises over the axes, and children that differ only in their
// z bit (then y, then x) share the x and y factors, so the sum runs as three passes over LDS rows:
// z (8 rows -> 4), y (4 -> 2), x (2 -> 1), each term one multiply-add.
template <int PM>
__global__ __launch_bounds__(SH_TPB) void k_m2m(TreeView t, OpTables op, int lp,
                                                double* __restrict__ M, const int* done) {
  if (done && *done) return;
  constexpr int MAX_STRIDE = sched_stride(PM);  // row stride of an expansion at order PM
  __shared__ double sA[8][MAX_STRIDE];
  __shared__ double sB[4][MAX_STRIDE];
  __shared__ double hp[2][PM + 1];
  __shared__ int ch[8];
  const int g = t.off[lp] + blockIdx.x;
  const int nc = op.nc, p = op.p;
  if (threadIdx.x < 8) ch[threadIdx.x] = t.child8[8 * g + threadIdx.x];
  if (threadIdx.x == 8) shift_powers(hp[0], hp[1], p, 2.0);
  __syncthreads();
  for (int e = threadIdx.x; e < 8 * nc; e += SH_TPB) {
    const int o = e / nc, k = e - o * nc;
    const int c = ch[o];
    sA[o][k] = c >= 0 ? M[(int64_t)c * op.stride + k] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 4 * nc; e += SH_TPB) {  // z: pair (bx, by) of children
    const int pr = e / nc, k = e - pr * nc;
    const int nx = op.mi[3 * k], ny = op.mi[3 * k + 1], nz = op.mi[3 * k + 2];
    double v = 0.0;
    for (int bz = 0; bz < 2; ++bz) {
      if (ch[2 * pr + bz] < 0) continue;
      const double* row = sA[2 * pr + bz];
      for (int kz = 0; kz <= nz; ++kz) v += hp[bz][kz] * row[mi_index(nx, ny, nz - kz)];
    }
    sB[pr][k] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * nc; e += SH_TPB) {  // y: children rows are no longer needed
    const int bx = e / nc, k = e - bx * nc;
    const int nx = op.mi[3 * k], ny = op.mi[3 * k + 1], nz = op.mi[3 * k + 2];
    double v = 0.0;
    for (int by = 0; by < 2; ++by)
      for (int ky = 0; ky <= ny; ++ky) v += hp[by][ky] * sB[2 * bx + by][mi_index(nx, ny - ky, nz)];
    sA[bx][k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < op.stride; k += SH_TPB) {
    double v = 0.0;
    if (k < nc) {
      const int nx = op.mi[3 * k], ny = op.mi[3 * k + 1], nz = op.mi[3 * k + 2];
      for (int bx = 0; bx < 2; ++bx)
        for (int kx = 0; kx <= nx; ++kx) v += hp[bx][kx] * sA[bx][mi_index(nx - kx, ny, nz)];
      v = ldexp(v, -(nx + ny + nz));
    }
    M[(int64_t)g * op.stride + k] = v;
  }
}

// One block per parent cell, for its children at level lc: F~(child) += partial M2L sums of the
// other offset splits, then, from level 3 on,
//   F~_n(child) += 2^-(|n|+1) sum_{|k| <= p-|n|} prod_a xl_a^{k_a} / k_a! F~_{n+k}(parent),
// xl_a = +1/4 for octant bit 1 and -1/4 for bit 0 (the parent row is complete because levels run
// top-down).  As in M2M the sum factorises: z (1 row -> 2), y (2 -> 4), x (4 -> 8 children).
// The truncation |k| <= p - |n| is kept exactly: each pass only reaches indices of degree <= p.
template <int PM>
__global__ __launch_bounds__(SH_TPB) void k_l2l(TreeView t, OpTables op, int lc, double* F,
                                                int nsplit, int64_t split_stride, const int* done) {
  if (done && *done) return;
  constexpr int MAX_STRIDE = sched_stride(PM);  // row stride of an expansion at order PM
  __shared__ double sP[MAX_STRIDE];
  __shared__ double sU1[2][MAX_STRIDE];
  __shared__ double sU2[4][MAX_STRIDE];
  __shared__ double qp[2][PM + 1];  // [bit]: bit 1 -> +1/4, bit 0 -> -1/4
  __shared__ int ch[8];
  const int g = t.off[lc - 1] + blockIdx.x;
  const int nc = op.nc, p = op.p;
  const bool shift = lc >= 3;
  if (threadIdx.x < 8) ch[threadIdx.x] = t.child8[8 * g + threadIdx.x];
  if (shift) {
    if (threadIdx.x == 8) shift_powers(qp[1], qp[0], p, 1.0);
    for (int k = threadIdx.x; k < nc; k += SH_TPB) sP[k] = F[(int64_t)g * op.stride + k];
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * nc; e += SH_TPB) {
      const int bz = e / nc, k = e - bz * nc;
      const int nx = op.mi[3 * k], ny = op.mi[3 * k + 1], nz = op.mi[3 * k + 2];
      const int rem = p - nx - ny - nz;
      double v = 0.0;
      for (int kz = 0; kz <= rem; ++kz) v += qp[bz][kz] * sP[mi_index(nx, ny, nz + kz)];
      sU1[bz][k] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * nc; e += SH_TPB) {
      const int yz = e / nc, k = e - yz * nc;
      const int by = yz >> 1, bz = yz & 1;
      const int nx = op.mi[3 * k], ny = op.mi[3 * k + 1], nz = op.mi[3 * k + 2];
      const int rem = p - nx - ny - nz;
      double v = 0.0;
      for (int ky = 0; ky <= rem; ++ky) v += qp[by][ky] * sU1[bz][mi_index(nx, ny + ky, nz)];
      sU2[yz][k] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 8 * nc; e += SH_TPB) {
    const int o = e / nc, k = e - o * nc;
    const int c = ch[o];
    if (c < 0) continue;
    double acc = 0.0;
    for (int sp = 1; sp < nsplit; ++sp) acc += F[sp * split_stride + (int64_t)c * op.stride + k];
    if (shift) {
      const int nx = op.mi[3 * k], ny = op.mi[3 * k + 1], nz = op.mi[3 * k + 2];
      const int dn = nx + ny + nz;
      const int bx = (o >> 2) & 1;
      const double* u = sU2[o & 3];
      double v = 0.0;
      for (int kx = 0; kx <= p - dn; ++kx) v += qp[bx][kx] * u[mi_index(nx + kx, ny, nz)];
      acc += ldexp(v, -(dn + 1));
    }
    F[(int64_t)c * op.stride + k] += acc;
  }
}

constexpr int L2P_TPB = 64;

// Orders above MAX_P_MFMA (k_l2p_fixed below serves the others).
// One wavefront per leaf.  A leaf holds few particles at protein density, so each particle is
// served by G = 64 / T lanes (T = the leaf occupancy rounded up to a power of two), each lane taking
// every G-th coefficient; the partial sums are combined by a fixed butterfly of cross-lane
// exchanges.  The leaf's F~ is staged in LDS, each particle's powers of its scaled offset sit in its
// own LDS column, and the coefficient table (exponents, degree, indices of n + e_c and n + e_a + e_b)
// is read through the scalar cache.
// MODE 0 (dipole-solve evaluations): E only, so the coefficients of degree p, which feed only the
// potential, are skipped; MODE 1: potential, field and field gradient.
template <int MODE, int PM>
__global__ __launch_bounds__(L2P_TPB) void k_l2p(TreeView t, OpTables op, Particles pa,
                                                 const double* __restrict__ F, FieldOut out,
                                                 const int* done) {
  constexpr int mode = MODE;
  if (done && *done) return;
  constexpr int MAX_NC = mi_count(PM);  // multi-indices of degree <= PM
  __shared__ double sF[MAX_NC];
  __shared__ double pw[3][PM + 1][L2P_TPB];
  // the per-coefficient table, packed, and 1/k!: read from LDS (a broadcast per slice) rather
  // than from global memory in the inner loop
  __shared__ int4 sT[MAX_NC];    // nx | ny << 8 | nz << 16 | deg << 24, e_x | e_y << 16, e_z | ee_xx << 16, ee_yy | ee_zz << 16
  __shared__ int2 sU[MAX_NC];    // ee_xy | ee_xz << 16, ee_yz
  __shared__ double sIF[MAX_NC];
  const int g = t.off[t.L] + blockIdx.x;
  const int first = t.first[g], cnt = t.count[g];
  const int p = op.p, nc = op.nc;
  for (int k = threadIdx.x; k < nc; k += L2P_TPB) {
    sF[k] = F[(int64_t)g * op.stride + k];
    const int* tk = op.l2p_tab + 16 * k;
    sT[k] = make_int4(tk[0] | (tk[1] << 8) | (tk[2] << 16) | (tk[3] << 24), tk[4] | (tk[5] << 16),
                      tk[6] | (tk[7] << 16), tk[8] | (tk[9] << 16));
    sU[k] = make_int2(tk[10] | (tk[11] << 16), tk[12]);
    sIF[k] = op.inv_fact[k];
  }
  double c[3], w;
  cell_centre(t, g, t.L, c, w);
  const double iw = 1.0 / w;
  const int lane = threadIdx.x;
  const int T_ = cnt >= L2P_TPB ? L2P_TPB : (cnt <= 1 ? 1 : (1 << (32 - __clz(cnt - 1))));
  const int G = L2P_TPB / T_;
  const int slot = lane & (T_ - 1), slice = lane / T_;
  for (int i0 = 0; i0 < cnt; i0 += L2P_TPB) {
    const int li = i0 + slot;
    const bool active = li < cnt;
    const int i = first + (active ? li : 0);
    __syncthreads();  // sF staged; previous chunk done with pw
    if (slice == 0) {
      const double4 Pi = pa.P[i];
      const double rho[3] = {(Pi.x - c[0]) * iw, (Pi.y - c[1]) * iw, (Pi.z - c[2]) * iw};
      for (int a = 0; a < 3; ++a) {
        double v = 1.0;
        pw[a][0][slot] = 1.0;
        for (int e = 1; e <= p; ++e) { v *= rho[a]; pw[a][e][slot] = v; }
      }
    }
    __syncthreads();
    double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    double gxx = 0.0, gyy = 0.0, gzz = 0.0, gxy = 0.0, gxz = 0.0, gyz = 0.0;
    // degree-ordered coefficients: those of degree <= p - 1 are the first ncE
    const int ncE = mode == 1 ? nc : (p * (p + 1) * (p + 2)) / 6;
    for (int k = slice; k < ncE; k += G) {
      const int4 tk = sT[k];
      const int deg = (tk.x >> 24) & 0xff;
      const double m = pw[0][tk.x & 0xff][slot] * pw[1][(tk.x >> 8) & 0xff][slot] *
                       pw[2][(tk.x >> 16) & 0xff][slot] * sIF[k];
      if (mode == 1) phi += m * sF[k];
      if (deg <= p - 1) {
        ex -= m * sF[tk.y & 0xffff];
        ey -= m * sF[tk.y >> 16];
        ez -= m * sF[tk.z & 0xffff];
        if (mode == 1 && deg <= p - 2) {
          const int2 tu = sU[k];
          gxx -= m * sF[tk.z >> 16];
          gyy -= m * sF[tk.w & 0xffff];
          gzz -= m * sF[tk.w >> 16];
          gxy -= m * sF[tu.x & 0xffff];
          gxz -= m * sF[tu.x >> 16];
          gyz -= m * sF[tu.y];
        }
      }
    }
    for (int msk = T_; msk < L2P_TPB; msk <<= 1) {
      ex += __shfl_xor(ex, msk); ey += __shfl_xor(ey, msk); ez += __shfl_xor(ez, msk);
      if (mode == 1) {
        phi += __shfl_xor(phi, msk);
        gxx += __shfl_xor(gxx, msk); gyy += __shfl_xor(gyy, msk); gzz += __shfl_xor(gzz, msk);
        gxy += __shfl_xor(gxy, msk); gxz += __shfl_xor(gxz, msk); gyz += __shfl_xor(gyz, msk);
      }
    }
    if (!active || slice != 0) continue;
    const double iw2 = iw * iw, iw3 = iw2 * iw;
    ex *= iw2; ey *= iw2; ez *= iw2;
    out.Ed[3 * i] = ex; out.Ed[3 * i + 1] = ey; out.Ed[3 * i + 2] = ez;
    if (mode == 1) {
      out.phi[i] = phi * iw;
      out.Eu[3 * i] = ex; out.Eu[3 * i + 1] = ey; out.Eu[3 * i + 2] = ez;
      double* G6 = out.G + 6 * (int64_t)i;
      G6[0] = gxx * iw3; G6[1] = gyy * iw3; G6[2] = gzz * iw3;
      G6[3] = gxy * iw3; G6[4] = gxz * iw3; G6[5] = gyz * iw3;
    }
  }
}

// L2P at a compile-time order (orders up to MAX_P_MFMA).  The coefficient loop unrolls into
// straight-line code whose exponents and F~ indices are constants, so neither the per-coefficient
// table nor the powers need LDS.  The coefficients are visited x-major (n_x, then n_y, then n_z
// ascending), so each rho^n / n! follows from the previous one by one factor rho_a / n_a, and only
// three running products stay live.  Half a wavefront serves one leaf, 32 particles at a time; a
// workgroup serves 8 consecutive leaves, whose F~ rows it stages in LDS (18 KB at p = 10).  The sums,
// and MODE, are those of k_l2p.
constexpr int L2PF_TPB = 256, L2PF_LANES = 32, L2PF_LEAVES = L2PF_TPB / L2PF_LANES;
constexpr int L2PF_MIN_WAVES = 4;  // waves per SIMD the register budget must allow

// the multi-indices of degree <= D in x-major order
template <int D>
struct MiXMajor {
  int x[mi_count(D)], y[mi_count(D)], z[mi_count(D)];
  constexpr MiXMajor() : x(), y(), z() {
    int k = 0;
    for (int nx = 0; nx <= D; ++nx)
      for (int ny = 0; ny <= D - nx; ++ny)
        for (int nz = 0; nz <= D - nx - ny; ++nz) {
          x[k] = nx;
          y[k] = ny;
          z[k] = nz;
          ++k;
        }
  }
};

template <int MODE, int P>
__global__ __launch_bounds__(L2PF_TPB, L2PF_MIN_WAVES) void k_l2p_fixed(TreeView t, int stride, Particles pa,
                                                                        const double* __restrict__ F,
                                                                        FieldOut out, const int* done) {
  if (done && *done) return;
  constexpr int NC = mi_count(P);
  constexpr int D = MODE == 1 ? P : P - 1;  // MODE 0 skips the degree-P coefficients
  __shared__ double sF[L2PF_LEAVES][NC];
  const int g0 = t.off[t.L] + blockIdx.x * L2PF_LEAVES;
  const int nl = min(L2PF_LEAVES, t.off[t.L + 1] - g0);
  for (int e = threadIdx.x; e < nl * NC; e += L2PF_TPB) {
    const int l = e / NC, k = e - l * NC;
    sF[l][k] = F[(int64_t)(g0 + l) * stride + k];
  }
  __syncthreads();
  const int l = threadIdx.x / L2PF_LANES, slot = threadIdx.x % L2PF_LANES;
  if (l >= nl) return;
  const int g = g0 + l;
  const int first = t.first[g], cnt = t.count[g];
  double c[3], w;
  cell_centre(t, g, t.L, c, w);
  const double iw = 1.0 / w;
  const double* Fl = sF[l];
  constexpr MiXMajor<D> mx{};
#pragma unroll 1
  for (int li = slot; li < cnt; li += L2PF_LANES) {
    const int i = first + li;
    const double4 Pi = pa.P[i];
    const double rx = (Pi.x - c[0]) * iw, ry = (Pi.y - c[1]) * iw, rz = (Pi.z - c[2]) * iw;
    double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    double gxx = 0.0, gyy = 0.0, gzz = 0.0, gxy = 0.0, gxz = 0.0, gyz = 0.0;
    double a = 1.0, b = 1.0, m = 1.0;  // rho_x^nx/nx!, times rho_y^ny/ny!, times rho_z^nz/nz!
#pragma unroll
    for (int k = 0; k < mi_count(D); ++k) {
      const int x = mx.x[k], y = mx.y[k], z = mx.z[k];
      // a compiler-only fence at the start of each run of n_z: the LDS reads of one run are not
      // merged with, or hoisted into, another's, which would keep them live across the body
      if (z == 0) __asm__ volatile("" ::: "memory");
      if (z > 0) {
        m = m * (rz * (1.0 / z));
      } else if (y > 0) {
        b = b * (ry * (1.0 / y));
        m = b;
      } else if (x > 0) {
        a = a * (rx * (1.0 / x));
        b = a;
        m = a;
      }
      if (MODE == 1) phi += m * Fl[mi_index(x, y, z)];
      if (x + y + z <= P - 1) {
        ex -= m * Fl[mi_index(x + 1, y, z)];
        ey -= m * Fl[mi_index(x, y + 1, z)];
        ez -= m * Fl[mi_index(x, y, z + 1)];
        if (MODE == 1 && x + y + z <= P - 2) {
          gxx -= m * Fl[mi_index(x + 2, y, z)];
          gyy -= m * Fl[mi_index(x, y + 2, z)];
          gzz -= m * Fl[mi_index(x, y, z + 2)];
          gxy -= m * Fl[mi_index(x + 1, y + 1, z)];
          gxz -= m * Fl[mi_index(x + 1, y, z + 1)];
          gyz -= m * Fl[mi_index(x, y + 1, z + 1)];
        }
      }
    }
    const double iw2 = iw * iw, iw3 = iw2 * iw;
    ex *= iw2; ey *= iw2; ez *= iw2;
    out.Ed[3 * i] = ex; out.Ed[3 * i + 1] = ey; out.Ed[3 * i + 2] = ez;
    if (MODE == 1) {
      out.phi[i] = phi * iw;
      out.Eu[3 * i] = ex; out.Eu[3 * i + 1] = ey; out.Eu[3 * i + 2] = ez;
      double* G6 = out.G + 6 * (int64_t)i;
      G6[0] = gxx * iw3; G6[1] = gyy * iw3; G6[2] = gzz * iw3;
      G6[3] = gxy * iw3; G6[4] = gxz * iw3; G6[5] = gyz * iw3;
    }
  }
}

typedef void (*L2PFixedKernel)(TreeView, int, Particles, const double*, FieldOut, const int*);

template <int MODE, int... Ps>
L2PFixedKernel l2p_fixed_kernel(int p, std::integer_sequence<int, Ps...>) {
  L2PFixedKernel k = nullptr;
  ((p == Ps + 1 ? (void)(k = &k_l2p_fixed<MODE, Ps + 1>) : (void)0), ...);
  return k;
}

}  // namespace

// The kernels' LDS and registers are sized for an order class: orders up to MAX_P_MFMA, the
// benchmark's, keep the smaller footprint; the orders above take the larger one.
constexpr int PM_LO = MAX_P_MFMA, PM_HI = MAX_P;

void launch_p2m(const TreeView& t, const OpTables& op, const Particles& pa, const double4* mu4,
                int sources, double pair_dl, double* M, const int* done, hipStream_t s) {
  const int nleaf = t.off[t.L + 1] - t.off[t.L];
  if (nleaf <= 0) return;
  if (op.p > PM_HI) throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  const bool pair = pair_dl > 0.0 && (sources & 2), lo = op.p <= PM_LO;
  auto k = pair ? (lo ? k_p2m<true, PM_LO> : k_p2m<true, PM_HI>) : (lo ? k_p2m<false, PM_LO> : k_p2m<false, PM_HI>);
  hipLaunchKernelGGL(k, dim3(nleaf), dim3(P2M_TPB), 0, s, t, op, pa, mu4, sources, pair_dl, M, done);
  PFMM_LAUNCH_CHECK();
}

void launch_m2m(const TreeView& t, const OpTables& op, int parent_level, double* M, const int* done,
                hipStream_t s) {
  const int nc = t.off[parent_level + 1] - t.off[parent_level];
  if (nc <= 0) return;
  if (op.p > PM_HI) throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  hipLaunchKernelGGL(op.p <= PM_LO ? k_m2m<PM_LO> : k_m2m<PM_HI>, dim3(nc), dim3(SH_TPB), 0, s, t, op, parent_level,
                     M, done);
  PFMM_LAUNCH_CHECK();
}

void launch_l2l(const TreeView& t, const OpTables& op, int child_level, double* F, int nsplit,
                int64_t split_stride, const int* done, hipStream_t s) {
  if (child_level < 2) return;
  const int np = t.off[child_level] - t.off[child_level - 1];
  if (np <= 0 || (child_level < 3 && nsplit <= 1)) return;
  if (op.p > PM_HI) throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  hipLaunchKernelGGL(op.p <= PM_LO ? k_l2l<PM_LO> : k_l2l<PM_HI>, dim3(np), dim3(SH_TPB), 0, s, t, op, child_level,
                     F, nsplit, split_stride, done);
  PFMM_LAUNCH_CHECK();
}

void launch_l2p(const TreeView& t, const OpTables& op, const Particles& pa, const double* F, int mode,
                FieldOut out, const int* done, hipStream_t s) {
  const int nleaf = t.off[t.L + 1] - t.off[t.L];
  if (nleaf <= 0) return;
  if (op.p < 1 || op.p > PM_HI || op.nc != mi_count(op.p)) throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  if (op.p <= PM_LO) {
    const L2PFixedKernel k = mode == 1 ? l2p_fixed_kernel<1>(op.p, std::make_integer_sequence<int, PM_LO>{})
                                       : l2p_fixed_kernel<0>(op.p, std::make_integer_sequence<int, PM_LO>{});
    if (!k) throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
    hipLaunchKernelGGL(k, dim3((nleaf + L2PF_LEAVES - 1) / L2PF_LEAVES), dim3(L2PF_TPB), 0, s, t, op.stride, pa, F,
                       out, done);
  } else {
    auto k = mode == 1 ? k_l2p<1, PM_HI> : k_l2p<0, PM_HI>;
    hipLaunchKernelGGL(k, dim3(nleaf), dim3(L2P_TPB), 0, s, t, op, pa, F, out, done);
  }
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

// Upward and downward passes of the Cartesian FMM (Sec. II.B-II.C) on level-scaled expansions:
//   P2M  M~_n = (-1)^|n|/n! sum_a [ q_a rho_a^n + (mu_a / w) . grad(rho^n)(rho_a) ],  rho = (x - z)/w
//        (point dipoles enter through the delta-l -> 0 limit of the +/- q^mu pair of Sec. II.C)
//   M2M  M~_n(parent) = sum_{k <= n} xt^k/k! 2^-(|n|-|k|) M~_{n-k}(child)
//   L2L  F~_n(child) += sum_{|k| <= p-|n|} xt'^k/k! 2^-(|n|+1) F~_{n+k}(parent)
//   L2P  phi = (1/w) sum rho^n/n! F~_n,  E_c = -(1/w^2) sum rho^n/n! F~_{n+e_c},
//        d_a E_b = -(1/w^3) sum rho^n/n! F~_{n+e_a+e_b}
// with M~_n = M_n / w^|n| and F~_n = F_n w^(|n|+1) for the cell edge w of the level.
// All four are memory-bound; they run in float64 on both precision paths.
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
// per coefficient.
__global__ __launch_bounds__(P2M_TPB) void k_p2m(TreeView t, OpTables op, Particles pa,
                                                 const double4* __restrict__ mu4, int sources,
                                                 double* __restrict__ M, const int* done) {
  if (done && *done) return;
  __shared__ double pw[P2M_CHUNK][3][MAX_P + 1];
  __shared__ double sq[P2M_CHUNK], sm[P2M_CHUNK][3];
  const int g = t.off[t.L] + blockIdx.x;
  const int first = t.first[g], cnt = t.count[g];
  double c[3], w;
  cell_centre(t, g, t.L, c, w);
  const double iw = 1.0 / w;
  const int p = op.p, nc = op.nc;
  constexpr int KPT = (286 + P2M_TPB - 1) / P2M_TPB;  // coefficients per thread at p = 10
  double acc[KPT];
  int ex[KPT][3];
  for (int r = 0; r < KPT; ++r) {
    acc[r] = 0.0;
    const int k = threadIdx.x + r * P2M_TPB;
    for (int a = 0; a < 3; ++a) ex[r][a] = k < nc ? op.mi[3 * k + a] : 0;
  }
  for (int s0 = 0; s0 < cnt; s0 += P2M_CHUNK) {
    const int m = min(P2M_CHUNK, cnt - s0);
    if (threadIdx.x < m) {
      const int j = threadIdx.x;
      const double4 P = pa.P[first + s0 + j];
      const double rho[3] = {(P.x - c[0]) * iw, (P.y - c[1]) * iw, (P.z - c[2]) * iw};
      for (int a = 0; a < 3; ++a) {
        double v = 1.0;
        pw[j][a][0] = 1.0;
        for (int e = 1; e <= p; ++e) { v *= rho[a]; pw[j][a][e] = v; }
      }
      sq[j] = (sources & 1) ? P.w : 0.0;
      if (sources & 2) {
        const double4 u = mu4[first + s0 + j];
        sm[j][0] = u.x * iw; sm[j][1] = u.y * iw; sm[j][2] = u.z * iw;
      } else {
        sm[j][0] = sm[j][1] = sm[j][2] = 0.0;
      }
    }
    __syncthreads();
    for (int r = 0; r < KPT; ++r) {
      const int k = threadIdx.x + r * P2M_TPB;
      if (k >= nc) break;
      const int nx = ex[r][0], ny = ex[r][1], nz = ex[r][2];
      double a = 0.0;
      for (int j = 0; j < m; ++j) {
        const double X = pw[j][0][nx], Y = pw[j][1][ny], Z = pw[j][2][nz];
        double v = sq[j] * X * Y * Z;
        if (nx) v += sm[j][0] * nx * pw[j][0][nx - 1] * Y * Z;
        if (ny) v += sm[j][1] * ny * X * pw[j][1][ny - 1] * Z;
        if (nz) v += sm[j][2] * nz * X * Y * pw[j][2][nz - 1];
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

constexpr int SH_TPB = 128;

// One block per parent cell: M~(parent) = sum over children of the octant's shift matrix.
__global__ __launch_bounds__(SH_TPB) void k_m2m(TreeView t, OpTables op, int lp,
                                                double* __restrict__ M, const int* done) {
  if (done && *done) return;
  const int g = t.off[lp] + blockIdx.x;
  int ch[8];
  for (int o = 0; o < 8; ++o) ch[o] = t.child8[8 * g + o];
  for (int k = threadIdx.x; k < op.stride; k += SH_TPB) {
    double acc = 0.0;
    if (k < op.nc) {
      for (int o = 0; o < 8; ++o) {
        if (ch[o] < 0) continue;
        const double* Mc = M + (int64_t)ch[o] * op.stride;
        const int b = op.m2m_ptr[o * (op.nc + 1) + k], e = op.m2m_ptr[o * (op.nc + 1) + k + 1];
        for (int j = b; j < e; ++j) acc += op.m2m_val[j] * Mc[op.m2m_col[j]];
      }
    }
    M[(int64_t)g * op.stride + k] = acc;
  }
}

// One block per child cell: F~(child) += partial M2L sums of the other offset splits, then the
// shift of F~(parent) (levels >= 3; the parent row is complete because levels run top-down).
__global__ __launch_bounds__(SH_TPB) void k_l2l(TreeView t, OpTables op, int lc, double* F,
                                                int nsplit, int64_t split_stride, const int* done) {
  if (done && *done) return;
  const int g = t.off[lc] + blockIdx.x;
  const int par = t.parent[g];
  const int o = (int)(t.key[g] & 7);
  const double* Fp = F + (int64_t)par * op.stride;
  for (int k = threadIdx.x; k < op.nc; k += SH_TPB) {
    double acc = 0.0;
    for (int sp = 1; sp < nsplit; ++sp) acc += F[sp * split_stride + (int64_t)g * op.stride + k];
    if (lc >= 3) {
      const int b = op.l2l_ptr[o * (op.nc + 1) + k], e = op.l2l_ptr[o * (op.nc + 1) + k + 1];
      for (int j = b; j < e; ++j) acc += op.l2l_val[j] * Fp[op.l2l_col[j]];
    }
    F[(int64_t)g * op.stride + k] += acc;
  }
}

constexpr int L2P_TPB = 64;
constexpr int MAX_NC = 286;  // multi-indices of degree <= 10

// One wavefront per leaf; one particle per lane.  The leaf's F~ is staged in LDS, each lane keeps
// the powers of its scaled offset in its own LDS column, and the coefficient loop walks a table
// (exponents, degree, indices of n + e_c and n + e_a + e_b) whose entries are uniform across
// the wave, so table reads are scalar and F~ reads are LDS broadcasts.
__global__ __launch_bounds__(L2P_TPB) void k_l2p(TreeView t, OpTables op, Particles pa,
                                                 const double* __restrict__ F, int mode, FieldOut out,
                                                 const int* done) {
  if (done && *done) return;
  __shared__ double sF[MAX_NC];
  __shared__ double pw[3][MAX_P + 1][L2P_TPB];
  const int g = t.off[t.L] + blockIdx.x;
  const int first = t.first[g], cnt = t.count[g];
  const int p = op.p, nc = op.nc;
  for (int k = threadIdx.x; k < nc; k += L2P_TPB) sF[k] = F[(int64_t)g * op.stride + k];
  __syncthreads();
  double c[3], w;
  cell_centre(t, g, t.L, c, w);
  const double iw = 1.0 / w;
  const int tid = threadIdx.x;
  for (int i0 = 0; i0 < cnt; i0 += L2P_TPB) {
    const int li = i0 + tid;
    if (li >= cnt) break;
    const int i = first + li;
    const double4 Pi = pa.P[i];
    const double rho[3] = {(Pi.x - c[0]) * iw, (Pi.y - c[1]) * iw, (Pi.z - c[2]) * iw};
    for (int a = 0; a < 3; ++a) {
      double v = 1.0;
      pw[a][0][tid] = 1.0;
      for (int e = 1; e <= p; ++e) { v *= rho[a]; pw[a][e][tid] = v; }
    }
    double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    double gxx = 0.0, gyy = 0.0, gzz = 0.0, gxy = 0.0, gxz = 0.0, gyz = 0.0;
    for (int k = 0; k < nc; ++k) {
      const int* tk = op.l2p_tab + 16 * k;
      const int deg = tk[3];
      const double m = pw[0][tk[0]][tid] * pw[1][tk[1]][tid] * pw[2][tk[2]][tid] * op.inv_fact[k];
      phi += m * sF[k];
      if (deg <= p - 1) {
        ex -= m * sF[tk[4]];
        ey -= m * sF[tk[5]];
        ez -= m * sF[tk[6]];
        if (mode == 1 && deg <= p - 2) {
          gxx -= m * sF[tk[7]];
          gyy -= m * sF[tk[8]];
          gzz -= m * sF[tk[9]];
          gxy -= m * sF[tk[10]];
          gxz -= m * sF[tk[11]];
          gyz -= m * sF[tk[12]];
        }
      }
    }
    const double iw2 = iw * iw, iw3 = iw2 * iw;
    ex *= iw2; ey *= iw2; ez *= iw2;
    out.Ed[3 * i] = ex; out.Ed[3 * i + 1] = ey; out.Ed[3 * i + 2] = ez;
    if (mode == 1) {
      out.phi[i] = phi * iw;
      out.Eu[3 * i] = ex; out.Eu[3 * i + 1] = ey; out.Eu[3 * i + 2] = ez;
      double* G = out.G + 6 * (int64_t)i;
      G[0] = gxx * iw3; G[1] = gyy * iw3; G[2] = gzz * iw3;
      G[3] = gxy * iw3; G[4] = gxz * iw3; G[5] = gyz * iw3;
    }
  }
}

}  // namespace

void launch_p2m(const TreeView& t, const OpTables& op, const Particles& pa, const double4* mu4,
                int sources, double* M, const int* done, hipStream_t s) {
  const int nleaf = t.off[t.L + 1] - t.off[t.L];
  if (nleaf <= 0) return;
  hipLaunchKernelGGL(k_p2m, dim3(nleaf), dim3(P2M_TPB), 0, s, t, op, pa, mu4, sources, M, done);
  PFMM_LAUNCH_CHECK();
}

void launch_m2m(const TreeView& t, const OpTables& op, int parent_level, double* M, const int* done,
                hipStream_t s) {
  const int nc = t.off[parent_level + 1] - t.off[parent_level];
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_m2m, dim3(nc), dim3(SH_TPB), 0, s, t, op, parent_level, M, done);
  PFMM_LAUNCH_CHECK();
}

void launch_l2l(const TreeView& t, const OpTables& op, int child_level, double* F, int nsplit,
                int64_t split_stride, const int* done, hipStream_t s) {
  const int nc = t.off[child_level + 1] - t.off[child_level];
  if (nc <= 0 || (child_level < 3 && nsplit <= 1)) return;
  hipLaunchKernelGGL(k_l2l, dim3(nc), dim3(SH_TPB), 0, s, t, op, child_level, F, nsplit, split_stride,
                     done);
  PFMM_LAUNCH_CHECK();
}

void launch_l2p(const TreeView& t, const OpTables& op, const Particles& pa, const double* F, int mode,
                FieldOut out, const int* done, hipStream_t s) {
  const int nleaf = t.off[t.L + 1] - t.off[t.L];
  if (nleaf <= 0) return;
  if (op.nc > MAX_NC) throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  hipLaunchKernelGGL(k_l2p, dim3(nleaf), dim3(L2P_TPB), 0, s, t, op, pa, F, mode, out, done);
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

// Near field by direct summation over neighbouring leaves (the direct component of Sec. III),
// with true point dipoles and Thole damping of dipole-dipole pairs.
//
// One wavefront per target leaf.  The sources of all colleague leaves (Chebyshev distance <= ws),
// or of the leaf's row of the near list of the acceptance-criterion walk (mac.hip, LIST), are walked
// as one concatenated sequence and staged in LDS 64 at a time, densely, whatever the
// leaf occupancy.  A leaf holds only a few particles at protein density, so each of its T targets
// is served by G = floor(64 / T) lanes (lanes t, t + T, t + 2T, ...); every lane sweeps a 1/G slice
// of each staged chunk, and the G partial sums of a target are combined at the end through LDS in
// a fixed order (deterministic).  Results are added to the far-field values already written by L2P.
//
// Pair kernels, with r = x_i - x_j, u = r/|r|:
//   charge  q_j:  phi += q/r,  E += q r/r^3,  d_a E_b += q (delta_ab/r^3 - 3 r_a r_b/r^5)
//   dipole mu_j:  phi += mu.r/r^3 (undamped),  E_u += (3 u (u.mu) - mu)/r^3 (undamped),
//                 E_d += (3 f_t u (u.mu) - f_e mu)/r^3,
//                 d_a (E_d)_b += A u_a u_b (u.mu)/r^4 + B (delta_ab (u.mu) + u_a mu_b + u_b mu_a)/r^4
// where, for the Thole linear model with v = min(r/s, 1), s = a (alpha_i alpha_j)^(1/6):
//   f_t = v^4, f_e = 4 v^3 - 3 v^4, A = -3 v^4 (v < 1) or -15 (v >= 1), B = 3 v^4.
// Float32 variant (mixed path): offsets relative to the target leaf centre, float32 arithmetic
// and accumulation, results added to the float64 fields.
// Mode 3 is the operator of the dipole-solve preconditioner: the damped dipole field from the
// sources within a cutoff radius rc (rc <= leaf edge, so the 27 adjacent leaves hold them all),
// written rather than added.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "kernels.hpp"
#include "morton.hpp"

namespace pfmm {

namespace {

constexpr int TPB = 64;
constexpr int CHUNK = 2 * TPB;  // source leaves per prefix pass (the 125 colleagues at ws = 2 in one)

// 1/sqrt(x) for a finite x > 0, which is all that reaches it here (the r^2 of two distinct
// particles, or 1 in place of a masked pair): the hardware estimate y, refined by one step of the
// series (1 - e)^(-1/2) = 1 + e/2 + 3 e^2/8 + ..., e = 1 - x y^2, which triples its correct bits.
// The library function adds a guard for 0, infinities and denormals that these arguments never need.
__device__ inline double rsqrt_t(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}
// float32: the hardware estimate alone (the library function's result for every normal x; it adds a
// rescaling of denormal arguments, which an r^2 here never is).
__device__ inline float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }

template <typename T, int MODE, int SRC, bool LIST>
__global__ __launch_bounds__(TPB) void k_p2p(TreeView t, Particles pa, const double4* __restrict__ mu4,
                                             FieldOut out, double* __restrict__ dal,
                                             int* __restrict__ err, const int* done, T rc2) {
  if (done && *done) return;
  constexpr bool HQ = (SRC & 1) != 0;
  constexpr bool HM = (SRC & 2) != 0;
  constexpr bool STAGE_MU = HM || MODE == 2;
  static_assert(!LIST || MODE != 3, "the preconditioner takes the colleagues");
  __shared__ int s_pref[CHUNK + 1], s_first[CHUNK];
  __shared__ T sx[TPB], sy[TPB], sz[TPB], sq[TPB], smx[TPB], smy[TPB], smz[TPB], sit[TPB];
  __shared__ int sidx[TPB];
  const int g = t.off[t.L] + blockIdx.x;
  const int first = t.first[g], cnt = t.count[g];
  const int lane = threadIdx.x;
  // the source leaves: the colleague row (nnear <= 125 entries in offset order, -1 where empty), or
  // the leaf's row of the near list, taken in chunks of CHUNK
  const int* ent = t.coll + (int64_t)g * t.nnear;
  int ne = t.nnear;
  if constexpr (LIST) {
    const int lg = g - t.off[t.L];
    ent = t.nidx + t.nptr[lg];
    ne = t.nptr[lg + 1] - t.nptr[lg];
  }

  // The colleagues are taken adjacent ones first (offsets with every component in [-1, 1]).  When the
  // damping radius is at most the leaf edge (t.damp_adjacent) only they can hold Thole-damped pairs,
  // so the staged chunks past their particles run the undamped pair kernel; mode 3 (the
  // preconditioner, cutoff below the leaf edge) takes the adjacent ones alone.  s_ord[k]: colleague
  // index of position k.
  __shared__ int s_ord[LIST ? 1 : CHUNK];
  if constexpr (!LIST) {
    const int side = 2 * t.ws + 1;
    auto is_adj = [&](int ci) {
      return abs(ci / (side * side) - t.ws) <= 1 && abs((ci / side) % side - t.ws) <= 1 && abs(ci % side - t.ws) <= 1;
    };
    const bool a0 = lane < ne && is_adj(lane), a1 = lane + TPB < ne && is_adj(lane + TPB);
    const unsigned long long b0 = __ballot(a0), b1 = __ballot(a1);
    const unsigned long long below = lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
    const int n0 = __popcll(b0), na = n0 + __popcll(b1);
    if (lane < ne) {
      const int ra = __popcll(b0 & below);
      s_ord[a0 ? ra : na + (lane - ra)] = lane;
    }
    if (lane + TPB < ne) {
      const int ra = n0 + __popcll(b1 & below), k = lane + TPB;
      s_ord[a1 ? ra : na + (k - ra)] = k;
    }
    if (MODE == 3) ne = na;
    __syncthreads();
  }
  const int nadj = [&] {
    if constexpr (LIST) return ne;
    const int side = 2 * t.ws + 1;
    return min(ne, side >= 3 ? 27 : ne);
  }();

  // exclusive prefix of the occupancies of the source leaves E0 .. E0 + nn - 1 (two per lane) into
  // s_pref[0 .. nn], their first particles into s_first; returns nn
  auto entry = [&](int k) {
    if constexpr (LIST) return ent[k];
    else return ent[s_ord[k]];
  };
  auto prefix = [&](int E0) {
    const int nn = min(CHUNK, ne - E0);
    int c0 = 0, c1 = 0, f0 = 0, f1 = 0;
    if (lane < nn) {
      const int A = entry(E0 + lane);
      if (A >= 0) { c0 = t.count[A]; f0 = t.first[A]; }
    }
    if (lane + TPB < nn) {
      const int A = entry(E0 + lane + TPB);
      if (A >= 0) { c1 = t.count[A]; f1 = t.first[A]; }
    }
    int i0 = c0, i1 = c1;
    for (int d = 1; d < TPB; d <<= 1) {
      const int u0 = __shfl_up(i0, d), u1 = __shfl_up(i1, d);
      if (lane >= d) { i0 += u0; i1 += u1; }
    }
    const int tot0 = __shfl(i0, TPB - 1);
    if (lane < nn) { s_pref[lane] = i0 - c0; s_first[lane] = f0; }
    if (lane + TPB < nn) { s_pref[lane + TPB] = tot0 + i1 - c1; s_first[lane + TPB] = f1; }
    const int tot = tot0 + __shfl(i1, TPB - 1);
    if (lane == 0) s_pref[nn] = tot;
    return nn;
  };
  int nn = 0;
  int adj_src = INT_MAX;  // staged sources below this index may form damped pairs
  if constexpr (!LIST) {
    nn = prefix(0);
    __syncthreads();
    if (t.damp_adjacent) adj_src = s_pref[min(nadj, nn)];
  }

  double cen[3];
  {
    const uint64_t k = t.key[g];
    cen[0] = t.origin[0] + ((double)compact3(k >> 2) + 0.5) * t.w;
    cen[1] = t.origin[1] + ((double)compact3(k >> 1) + 0.5) * t.w;
    cen[2] = t.origin[2] + ((double)compact3(k) + 0.5) * t.w;
  }
  // lanes per target: T targets per pass, G = floor(64 / T) lanes each; lanes from G T on idle
  const int T_ = cnt >= TPB ? TPB : (cnt < 1 ? 1 : cnt);
  const int G = TPB / T_;
  const int slot = lane % T_, slice = lane / T_;

  for (int t0 = 0; t0 < cnt; t0 += TPB) {
    const int li = t0 + slot;
    const bool active = slice < G && li < cnt;
    const int i = first + (active ? li : 0);
    const double4 Pi = pa.P[i];
    const T xi = (T)(Pi.x - cen[0]), yi = (T)(Pi.y - cen[1]), zi = (T)(Pi.z - cen[2]);
    const T iti = (T)pa.itau[i];
    double4 mui = make_double4(0, 0, 0, 0);
    if (MODE == 2) mui = mu4[i];
    T phi = 0, eux = 0, euy = 0, euz = 0, edx = 0, edy = 0, edz = 0;
    T gxx = 0, gyy = 0, gzz = 0, gxy = 0, gxz = 0, gyz = 0;
    double dsum = 0.0;
    int bad = 0;
    for (int E0 = 0; LIST ? E0 < ne : E0 == 0; E0 += CHUNK) {
      if constexpr (LIST) {
        __syncthreads();  // the previous chunk's prefix is no longer read
        nn = prefix(E0);
        __syncthreads();
      }
      const int total = s_pref[nn];
      for (int S0 = 0; S0 < total; S0 += TPB) {
        if (MODE == 2 && S0 >= adj_src) break;  // the Thole term needs damped pairs only
        const int m = min(TPB, total - S0);
        __syncthreads();
        if (lane < m) {
          const int idx = S0 + lane;
          int lo = 0, hi = nn - 1;  // last colleague k with s_pref[k] <= idx
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pref[mid] <= idx) lo = mid; else hi = mid - 1;
          }
          const int j = s_first[lo] + idx - s_pref[lo];
          const double4 Pj = pa.P[j];
          sx[lane] = (T)(Pj.x - cen[0]);
          sy[lane] = (T)(Pj.y - cen[1]);
          sz[lane] = (T)(Pj.z - cen[2]);
          sq[lane] = (T)Pj.w;
          if (STAGE_MU) {
            const double4 u = mu4[j];
            smx[lane] = (T)u.x; smy[lane] = (T)u.y; smz[lane] = (T)u.z;
          }
          sit[lane] = (T)pa.itau[j];
          sidx[lane] = j;
        }
        __syncthreads();
        if (!active) continue;
        // DAMP: the chunk may hold pairs inside a damping cone; otherwise v = 1 for every pair
        auto chunk = [&](auto dampc) {
          constexpr bool DAMP = decltype(dampc)::value;
          if constexpr (MODE == 3) {
            // The cutoff keeps about a tenth of the staged sources: mark the lane's sources inside it
            // (at most 64: m <= 64), then evaluate those alone, in the same order; the others would
            // add exact zeros.
            // Bit b of the mask is the lane's source jj = slice + b G.  The first nfull of them are
            // below m on every slice (a loop with a wave-uniform trip count), one more on some.
            const int Gu = __builtin_amdgcn_readfirstlane(G), mu = __builtin_amdgcn_readfirstlane(m);
            const int nfull = mu >= Gu ? (mu - Gu) / Gu + 1 : 0;
            auto inside = [&](int jj) {
              const T rx = xi - sx[jj], ry = yi - sy[jj], rz = zi - sz[jj];
              const T r2 = rx * rx + ry * ry + rz * rz;
              return r2 > T(0) && r2 < rc2;
            };
            unsigned lo = 0u, hi = 0u;
            const int n0 = min(nfull, 32);
  #pragma unroll 4
            for (int b = 0; b < n0; ++b) lo |= inside(slice + b * Gu) ? 1u << b : 0u;
  #pragma unroll 4
            for (int b = n0; b < nfull; ++b) hi |= inside(slice + b * Gu) ? 1u << (b - 32) : 0u;
            if (nfull < 64 && slice + nfull * Gu < mu && inside(slice + nfull * Gu)) {
              if (nfull < 32) lo |= 1u << nfull; else hi |= 1u << (nfull - 32);
            }
            unsigned long long in = ((unsigned long long)hi << 32) | lo;
            while (in) {
              const int jj = slice + __builtin_ctzll(in) * G;
              in &= in - 1ULL;
              const T rx = xi - sx[jj], ry = yi - sy[jj], rz = zi - sz[jj];
              const T r2 = rx * rx + ry * ry + rz * rz;
              const T rinv = rsqrt_t(r2), rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
              const T mx = smx[jj], my = smy[jj], mz = smz[jj];
              const T rmu = rx * mx + ry * my + rz * mz;
              T v = T(1), v4 = T(1);
              if constexpr (DAMP) {
                const T ii = iti * sit[jj];
                v = ii > T(0) ? fmin(r2 * rinv * ii, T(1)) : T(1);
                v4 = v * v * v * v;
              }
              const T fe = DAMP ? v * v * v * (T(4) - T(3) * v) : T(1);
              const T c3 = T(3) * v4 * rmu * rinv2;
              edx += (c3 * rx - fe * mx) * rinv3;
              edy += (c3 * ry - fe * my) * rinv3;
              edz += (c3 * rz - fe * mz) * rinv3;
            }
            return;
          }
  #pragma unroll 4
          for (int jj = slice; jj < m; jj += G) {
            const T rx = xi - sx[jj], ry = yi - sy[jj], rz = zi - sz[jj];
            const T r2 = rx * rx + ry * ry + rz * rz;
            // Undamped chunks hold sources of non-adjacent leaves only, a leaf edge or more away:
            // no self pair and no coincident pair can occur there, so the test is left out.
            const bool valid = !DAMP || (r2 > T(0) && (MODE != 3 || r2 < rc2));
            if (MODE == 1 && !valid && sidx[jj] != i) bad = 1;
            const T rinv = valid ? rsqrt_t(valid ? r2 : T(1)) : T(0);
            const T rinv2 = rinv * rinv;
            const T rinv3 = rinv * rinv2;
            if (MODE == 1 && HQ) {
              const T qj = sq[jj];
              const T qr3 = qj * rinv3;
              phi += qj * rinv;
              const T ex = qr3 * rx, ey = qr3 * ry, ez = qr3 * rz;
              eux += ex; euy += ey; euz += ez;
              edx += ex; edy += ey; edz += ez;
              const T c5 = T(3) * qr3 * rinv2;
              gxx += qr3 - c5 * rx * rx; gyy += qr3 - c5 * ry * ry; gzz += qr3 - c5 * rz * rz;
              gxy -= c5 * rx * ry; gxz -= c5 * rx * rz; gyz -= c5 * ry * rz;
            }
            if (MODE == 2 && DAMP) {
              // Thole term of dU/dalpha_i: (2 v^4 (mu_i.u)(mu_j.u) - 2 (v^3 - v^4) mu_i.mu_j) / (alpha_i r^3)
              const T ii = iti * sit[jj];
              const T rr = r2 * rinv;
              const T v = ii > T(0) ? fmin(rr * ii, T(1)) : T(1);
              if (valid && v < T(1)) {
                const T v3 = v * v * v, v4 = v3 * v;
                const T miu = (T(mui.x) * rx + T(mui.y) * ry + T(mui.z) * rz) * rinv;
                const T mju = (smx[jj] * rx + smy[jj] * ry + smz[jj] * rz) * rinv;
                const T mm = T(mui.x) * smx[jj] + T(mui.y) * smy[jj] + T(mui.z) * smz[jj];
                dsum += (double)((T(2) * v4 * miu * mju - T(2) * (v3 - v4) * mm) * rinv3);
              }
            }
            if ((MODE == 0 || MODE == 1 || MODE == 3) && HM) {
              const T mx = smx[jj], my = smy[jj], mz = smz[jj];
              const T rmu = rx * mx + ry * my + rz * mz;
              T v = T(1), v4 = T(1), ii = T(0);
              if constexpr (DAMP) {
                ii = iti * sit[jj];
                const T rr = r2 * rinv;
                v = ii > T(0) ? fmin(rr * ii, T(1)) : T(1);
                v4 = v * v * v * v;
              }
              const T ft = v4, fe = DAMP ? v * v * v * (T(4) - T(3) * v) : T(1);
              const T c3 = T(3) * ft * rmu * rinv2;
              edx += (c3 * rx - fe * mx) * rinv3;
              edy += (c3 * ry - fe * my) * rinv3;
              edz += (c3 * rz - fe * mz) * rinv3;
              if (MODE == 1) {
                phi += rmu * rinv3;
                const T cu = T(3) * rmu * rinv2;
                eux += (cu * rx - mx) * rinv3;
                euy += (cu * ry - my) * rinv3;
                euz += (cu * rz - mz) * rinv3;
                // The coefficient of u_a u_b u_c jumps at the edge of the damping cone (-3 inside, -15
                // outside: the linear model's third derivative is discontinuous at r = s).  Which
                // side a pair falls on is decided in float64 on both paths: near the edge the float32
                // ratio can round across it.
                bool inside = DAMP && v < T(1);
                if constexpr (DAMP && std::is_same<T, float>::value) {
                  if (ii > T(0) && fabs(v - T(1)) < T(1e-4)) {
                    const int j = sidx[jj];
                    const double4 Pj = pa.P[j];
                    const double dx = Pi.x - Pj.x, dy = Pi.y - Pj.y, dz = Pi.z - Pj.z;
                    inside = sqrt(dx * dx + dy * dy + dz * dz) * (pa.itau[i] * pa.itau[j]) < 1.0;
                  }
                }
                const T Ac = inside ? T(-3) * v4 : T(-15);
                const T Bc = T(3) * v4;
                const T rinv5 = rinv3 * rinv2;
                const T a7 = Ac * rmu * rinv5 * rinv2;  // A (u.mu) u_a u_b / r^4 = A rmu r_a r_b / r^7
                const T b5 = Bc * rinv5;
                gxx += a7 * rx * rx + b5 * (rmu + T(2) * rx * mx);
                gyy += a7 * ry * ry + b5 * (rmu + T(2) * ry * my);
                gzz += a7 * rz * rz + b5 * (rmu + T(2) * rz * mz);
                gxy += a7 * rx * ry + b5 * (rx * my + ry * mx);
                gxz += a7 * rx * rz + b5 * (rx * mz + rz * mx);
                gyz += a7 * ry * rz + b5 * (ry * mz + rz * my);
              }
            }
          }
        };
        if (S0 < adj_src)
          chunk(std::true_type{});
        else
          chunk(std::false_type{});
      }
    }
    // combine the G slices of every target (lanes slot, slot + T, slot + 2T, ...) in slice order
    if (G > 1) {
      constexpr int NR = (MODE == 1) ? 13 : (MODE == 2 ? 1 : 3);
      __shared__ T red[NR][TPB];
      __shared__ int redbad[TPB];
      T v[NR];
      if constexpr (MODE == 1) {
        v[0] = phi; v[1] = eux; v[2] = euy; v[3] = euz; v[4] = edx; v[5] = edy; v[6] = edz;
        v[7] = gxx; v[8] = gyy; v[9] = gzz; v[10] = gxy; v[11] = gxz; v[12] = gyz;
      } else if constexpr (MODE == 2) {
        v[0] = (T)dsum;
      } else {
        v[0] = edx; v[1] = edy; v[2] = edz;
      }
      __syncthreads();  // the staging arrays of the last chunk are no longer read
#pragma unroll
      for (int k = 0; k < NR; ++k) red[k][lane] = v[k];
      redbad[lane] = bad;
      __syncthreads();
      if (slice == 0) {
        for (int c = 1; c < G; ++c) {
#pragma unroll
          for (int k = 0; k < NR; ++k) v[k] += red[k][slot + c * T_];
          bad |= redbad[slot + c * T_];
        }
      }
      if constexpr (MODE == 1) {
        phi = v[0]; eux = v[1]; euy = v[2]; euz = v[3]; edx = v[4]; edy = v[5]; edz = v[6];
        gxx = v[7]; gyy = v[8]; gzz = v[9]; gxy = v[10]; gxz = v[11]; gyz = v[12];
      } else if constexpr (MODE == 2) {
        dsum = (double)v[0];
      } else {
        edx = v[0]; edy = v[1]; edz = v[2];
      }
    }
    if (!active || slice != 0) continue;
    if (bad) atomicOr(err, 1);
    if (MODE == 0) {
      out.Ed[3 * i] += (double)edx; out.Ed[3 * i + 1] += (double)edy; out.Ed[3 * i + 2] += (double)edz;
    } else if (MODE == 3) {
      out.Ed[3 * i] = (double)edx; out.Ed[3 * i + 1] = (double)edy; out.Ed[3 * i + 2] = (double)edz;
    } else if (MODE == 1) {
      out.phi[i] += (double)phi;
      out.Eu[3 * i] += (double)eux; out.Eu[3 * i + 1] += (double)euy; out.Eu[3 * i + 2] += (double)euz;
      out.Ed[3 * i] += (double)edx; out.Ed[3 * i + 1] += (double)edy; out.Ed[3 * i + 2] += (double)edz;
      double* G6 = out.G + 6 * (int64_t)i;
      G6[0] += (double)gxx; G6[1] += (double)gyy; G6[2] += (double)gzz;
      G6[3] += (double)gxy; G6[4] += (double)gxz; G6[5] += (double)gyz;
    } else {
      const double ai = pa.alpha[i];
      dal[i] = ai > 0.0 ? dsum / ai : 0.0;
    }
  }
}

template <typename T, bool LIST>
void p2p_dispatch(const TreeView& t, const Particles& pa, const double4* mu4, int mode, int sources,
                  FieldOut out, double* dal, int* err, const int* done, hipStream_t s, int nleaf,
                  double rc2) {
  const T r2 = (T)rc2;
  if (mode == 0)
    hipLaunchKernelGGL((k_p2p<T, 0, 2, LIST>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done, r2);
  else if (mode == 1 && sources == 1)
    hipLaunchKernelGGL((k_p2p<T, 1, 1, LIST>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done, r2);
  else if (mode == 1 && sources == 2)
    hipLaunchKernelGGL((k_p2p<T, 1, 2, LIST>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done, r2);
  else if (mode == 1 && sources == 3)
    hipLaunchKernelGGL((k_p2p<T, 1, 3, LIST>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done, r2);
  else if (mode == 2)
    hipLaunchKernelGGL((k_p2p<double, 2, 2, LIST>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done,
                       0.0);
  else
    throw Error(PFMM_ERR_INVALID_ARG, "internal: bad P2P mode");
}


// Excluded pairs (the starred sums of Sec. II.A): one thread per sorted target i takes the exact
// terms of each of its excluded partners off what the evaluation summed (the same pair kernels as
// above, in float64), in the order of the caller's list.  xptr/xidx are the exclusion rows in the
// caller's particle order; inv maps a caller index to its sorted position.  Modes as in k_p2p:
// 0 damped dipole field, 1 all outputs of the given sources, 2 the Thole term of dU/dalpha.
__global__ __launch_bounds__(256) void k_exclusions(Particles pa, const int* __restrict__ perm,
                                                    const int* __restrict__ inv, const int* __restrict__ xptr,
                                                    const int* __restrict__ xidx,
                                                    const double4* __restrict__ mu4, int mode, int sources,
                                                    FieldOut out, double* __restrict__ dal, const int* done) {
  if (done && *done) return;
  const bool hq = (sources & 1) != 0, hm = (sources & 2) != 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < pa.n; i += gridDim.x * blockDim.x) {
    const int o = perm[i];
    const int k0 = xptr[o], k1 = xptr[o + 1];
    if (k0 == k1) continue;
    const double4 Pi = pa.P[i];
    const double iti = pa.itau[i];
    const double4 mi = mode == 2 ? mu4[i] : make_double4(0, 0, 0, 0);
    double phi = 0, eu[3] = {0, 0, 0}, ed[3] = {0, 0, 0}, g[6] = {0, 0, 0, 0, 0, 0}, ds = 0;
    for (int k = k0; k < k1; ++k) {
      const int j = inv[xidx[k]];
      const double4 Pj = pa.P[j];
      const double r[3] = {Pi.x - Pj.x, Pi.y - Pj.y, Pi.z - Pj.z};
      const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      const double rinv = 1.0 / sqrt(r2), rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
      const double ii = iti * pa.itau[j];
      const double v = ii > 0.0 ? fmin(r2 * rinv * ii, 1.0) : 1.0;
      const double v3 = v * v * v, v4 = v3 * v;
      if (mode == 1 && hq) {
        const double qj = Pj.w, qr3 = qj * rinv3, c5 = 3.0 * qr3 * rinv2;
        phi += qj * rinv;
        for (int c = 0; c < 3; ++c) {
          eu[c] += qr3 * r[c];
          ed[c] += qr3 * r[c];
        }
        g[0] += qr3 - c5 * r[0] * r[0]; g[1] += qr3 - c5 * r[1] * r[1]; g[2] += qr3 - c5 * r[2] * r[2];
        g[3] -= c5 * r[0] * r[1]; g[4] -= c5 * r[0] * r[2]; g[5] -= c5 * r[1] * r[2];
      }
      if ((mode == 0 || mode == 1) && hm) {
        const double4 mj = mu4[j];
        const double m[3] = {mj.x, mj.y, mj.z};
        const double rmu = r[0] * m[0] + r[1] * m[1] + r[2] * m[2];
        const double fe = v3 * (4.0 - 3.0 * v), c3 = 3.0 * v4 * rmu * rinv2;
        for (int c = 0; c < 3; ++c) ed[c] += (c3 * r[c] - fe * m[c]) * rinv3;
        if (mode == 1) {
          phi += rmu * rinv3;
          const double cu = 3.0 * rmu * rinv2;
          for (int c = 0; c < 3; ++c) eu[c] += (cu * r[c] - m[c]) * rinv3;
          const double Ac = v < 1.0 ? -3.0 * v4 : -15.0, Bc = 3.0 * v4;
          const double rinv5 = rinv3 * rinv2, a7 = Ac * rmu * rinv5 * rinv2, b5 = Bc * rinv5;
          g[0] += a7 * r[0] * r[0] + b5 * (rmu + 2.0 * r[0] * m[0]);
          g[1] += a7 * r[1] * r[1] + b5 * (rmu + 2.0 * r[1] * m[1]);
          g[2] += a7 * r[2] * r[2] + b5 * (rmu + 2.0 * r[2] * m[2]);
          g[3] += a7 * r[0] * r[1] + b5 * (r[0] * m[1] + r[1] * m[0]);
          g[4] += a7 * r[0] * r[2] + b5 * (r[0] * m[2] + r[2] * m[0]);
          g[5] += a7 * r[1] * r[2] + b5 * (r[1] * m[2] + r[2] * m[1]);
        }
      }
      if (mode == 2 && v < 1.0) {
        const double4 mj = mu4[j];
        const double miu = (mi.x * r[0] + mi.y * r[1] + mi.z * r[2]) * rinv;
        const double mju = (mj.x * r[0] + mj.y * r[1] + mj.z * r[2]) * rinv;
        const double mm = mi.x * mj.x + mi.y * mj.y + mi.z * mj.z;
        ds += (2.0 * v4 * miu * mju - 2.0 * (v3 - v4) * mm) * rinv3;
      }
    }
    if (mode == 0) {
      for (int c = 0; c < 3; ++c) out.Ed[3 * i + c] -= ed[c];
    } else if (mode == 1) {
      out.phi[i] -= phi;
      for (int c = 0; c < 3; ++c) {
        out.Eu[3 * i + c] -= eu[c];
        out.Ed[3 * i + c] -= ed[c];
      }
      for (int c = 0; c < 6; ++c) out.G[6 * i + c] -= g[c];
    } else {
      const double ai = pa.alpha[i];
      if (ai > 0.0) dal[i] -= ds / ai;
    }
  }
}

__global__ __launch_bounds__(256) void k_inverse_perm(const int* __restrict__ perm, int n, int* __restrict__ inv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) inv[perm[i]] = i;
}

int grid256(int n) { return std::max(1, std::min((n + 255) / 256, 4096)); }

}  // namespace

void launch_exclusions(const Particles& pa, const int* perm, const int* inv, const int* xptr, const int* xidx,
                       const double4* mu4, int mode, int sources, FieldOut out, double* dal, const int* done,
                       hipStream_t s) {
  if (pa.n <= 0) return;
  hipLaunchKernelGGL(k_exclusions, dim3(grid256(pa.n)), dim3(256), 0, s, pa, perm, inv, xptr, xidx, mu4, mode,
                     sources, out, dal, done);
  PFMM_LAUNCH_CHECK();
}

void launch_inverse_perm(const int* perm, int n, int* inv, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_inverse_perm, dim3(grid256(n)), dim3(256), 0, s, perm, n, inv);
  PFMM_LAUNCH_CHECK();
}

void launch_p2p(const TreeView& t, const Particles& pa, const double4* mu4, int mode, int sources,
                bool fp32, FieldOut out, double* dal, int* err, const int* done, hipStream_t s,
                double rc) {
  const int nleaf = t.off[t.L + 1] - t.off[t.L];
  if (nleaf <= 0) return;
  // mode 3 (the preconditioner) takes the colleagues; mode 2 is float64 on both paths
  if (mode == 3) {
    if (fp32)
      hipLaunchKernelGGL((k_p2p<float, 3, 2, false>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done,
                         (float)(rc * rc));
    else
      hipLaunchKernelGGL((k_p2p<double, 3, 2, false>), dim3(nleaf), dim3(TPB), 0, s, t, pa, mu4, out, dal, err, done,
                         rc * rc);
  } else if (t.nptr) {
    if (fp32 && mode != 2)
      p2p_dispatch<float, true>(t, pa, mu4, mode, sources, out, dal, err, done, s, nleaf, rc * rc);
    else
      p2p_dispatch<double, true>(t, pa, mu4, mode, sources, out, dal, err, done, s, nleaf, rc * rc);
  } else {
    if (fp32 && mode != 2)
      p2p_dispatch<float, false>(t, pa, mu4, mode, sources, out, dal, err, done, s, nleaf, rc * rc);
    else
      p2p_dispatch<double, false>(t, pa, mu4, mode, sources, out, dal, err, done, s, nleaf, rc * rc);
  }
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

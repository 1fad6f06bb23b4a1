// The multipole acceptance criterion and dual tree walk of Sec. III (eq. mac) on the octree, and the
// M2L that runs from the lists they produce.
//
// A cell's enclosing radius r is the largest distance from its centre (the centre of its
// expansions) to one of its particles.  The walk goes level by level over a frontier of cell pairs
// (target B, source A) of one level, starting from (root, root).  A pair is
//   * accepted for M2L when A != B, the two cells are not adjacent (Chebyshev distance of their
//     coordinates >= 2, so that every pair of particles closer than a leaf edge, and with it every
//     Thole-damped pair, stays in the direct part), they hold at least ndirect particles together,
//     they are not leaves when leaf pairs are direct, and theta |z_B - z_A| > r_B + r_A (the
//     children of a pair below ndirect hold fewer particles still, so its descendants are all
//     direct: the paper's direct interaction of small pairs and of leaves);
//   * otherwise, at the leaf level, put on the near list (direct summation);
//   * otherwise replaced by the pairs of the two cells' non-empty children.
// Each level is a classify pass, inclusive prefix sums and an emit pass, so the lists come out in
// one fixed order; a stable radix sort by target then gives every cell its M2L row and every leaf
// its near row.  Every ordered pair of particles is covered exactly once: by the M2L of the one
// accepted pair of their ancestors, or by the near field of their leaves.
//
// The decisions are integers computed in floating point, so the lengths are formed exactly as
// written: centre = origin + (i + 1/2) w, |v| = sqrt((vx vx + vy vy) + vz vz), every operation
// rounded to float64 on its own (no fused multiply-adds) and the square root correctly rounded.
//
// The M2L of the lists: one wavefront per target cell walks its row in order, staging the source
// expansions and operator rows D(d) of four entries at a time in LDS; the lane of coefficient n
// accumulates
//   F~_n(B) = sum over the row of sum_{|m| <= q - |n|} D_{n+m}(d) M~_m(A)
// in float64 and writes it once (no atomics, fixed order).  The operator depends only on the
// integer offset d on every level (level-scaled expansions, tables.hpp).
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"
#include "morton.hpp"
#include "schedule.hpp"

namespace pfmm {

namespace {

__device__ inline void cell_coords(uint64_t k, int c[3]) {
  c[0] = compact3(k >> 2);
  c[1] = compact3(k >> 1);
  c[2] = compact3(k);
}

// |v| with each operation rounded on its own
__device__ inline double length3(double x, double y, double z) {
  return __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y)), __dmul_rn(z, z)));
}

__device__ inline int child_count(const TreeView& t, int g) {
  int k = 0;
  for (int o = 0; o < 8; ++o) k += t.child8[8 * g + o] >= 0 ? 1 : 0;
  return k;
}

constexpr int RTPB = 256;

// one workgroup per cell of the level
__global__ __launch_bounds__(RTPB) void k_mac_radii(TreeView t, const double4* __restrict__ P, int level,
                                                    double* __restrict__ renc) {
  __shared__ double red[RTPB];
  const int g = t.off[level] + blockIdx.x;
  const double w = ldexp(t.w, t.L - level);
  int c[3];
  cell_coords(t.key[g], c);
  double z[3];
  for (int a = 0; a < 3; ++a) z[a] = __dadd_rn(t.origin[a], __dmul_rn((double)c[a] + 0.5, w));
  const int first = t.first[g], cnt = t.count[g];
  double r = 0.0;
  for (int k = threadIdx.x; k < cnt; k += RTPB) {
    const double4 p = P[first + k];
    r = fmax(r, length3(__dsub_rn(p.x, z[0]), __dsub_rn(p.y, z[1]), __dsub_rn(p.z, z[2])));
  }
  red[threadIdx.x] = r;
  __syncthreads();
  for (int h = RTPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) renc[g] = red[0];
}

__global__ __launch_bounds__(256) void k_mac_classify(TreeView t, const double* __restrict__ renc, double theta,
                                                      int ndirect, int leaf_direct, int level,
                                                      const int2* __restrict__ fr, int nfr, int* __restrict__ acc,
                                                      int* __restrict__ kid) {
  const double w = ldexp(t.w, t.L - level);
  const bool leaves_direct = leaf_direct && level == t.L;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    const int B = fr[i].x, A = fr[i].y;
    bool accept = false;
    if (A != B && !leaves_direct && t.count[B] + t.count[A] >= ndirect) {
      int cb[3], ca[3];
      cell_coords(t.key[B], cb);
      cell_coords(t.key[A], ca);
      const int dx = cb[0] - ca[0], dy = cb[1] - ca[1], dz = cb[2] - ca[2];
      const int cheb = max(abs(dx), max(abs(dy), abs(dz)));
      if (cheb >= 2) {
        const double dist = length3(__dmul_rn((double)dx, w), __dmul_rn((double)dy, w), __dmul_rn((double)dz, w));
        accept = __dmul_rn(theta, dist) > __dadd_rn(renc[B], renc[A]);
      }
    }
    acc[i] = accept ? 1 : 0;
    kid[i] = accept ? 0 : (level == t.L ? 1 : child_count(t, B) * child_count(t, A));
  }
}

// bad: set when an accepted offset falls outside the operator table (cannot happen for theta >= 0.3)
__global__ __launch_bounds__(256) void k_mac_emit(TreeView t, int R, int level, const int2* __restrict__ fr, int nfr,
                                                  const int* __restrict__ acc_scan, const int* __restrict__ kid_scan,
                                                  int* __restrict__ m_tgt, unsigned long long* __restrict__ m_val,
                                                  int2* __restrict__ next, int* __restrict__ near_tgt,
                                                  int* __restrict__ near_src, int* bad) {
  const int side = 2 * R + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    const int B = fr[i].x, A = fr[i].y;
    const int a0 = i ? acc_scan[i - 1] : 0, k0 = i ? kid_scan[i - 1] : 0;
    if (acc_scan[i] > a0) {
      int cb[3], ca[3];
      cell_coords(t.key[B], cb);
      cell_coords(t.key[A], ca);
      const int dx = cb[0] - ca[0], dy = cb[1] - ca[1], dz = cb[2] - ca[2];
      if (abs(dx) > R || abs(dy) > R || abs(dz) > R) {
        atomicOr(bad, 1);
        continue;
      }
      const int slot = ((dx + R) * side + (dy + R)) * side + (dz + R);
      m_tgt[a0] = B;
      m_val[a0] = ((unsigned long long)(unsigned)A << 32) | (unsigned)slot;
    } else if (kid_scan[i] > k0) {
      if (level == t.L) {
        near_tgt[k0] = B;
        near_src[k0] = A;
      } else {
        int pos = k0;
        for (int ob = 0; ob < 8; ++ob) {
          const int b = t.child8[8 * B + ob];
          if (b < 0) continue;
          for (int oa = 0; oa < 8; ++oa) {
            const int a = t.child8[8 * A + oa];
            if (a >= 0) next[pos++] = make_int2(b, a);
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_mac_count(const int* __restrict__ keys, int n, int key0, int* cnt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(&cnt[keys[i] - key0], 1);
}

__global__ __launch_bounds__(256) void k_mac_near_pairs(TreeView t, const int* __restrict__ nt,
                                                        const int* __restrict__ ns, int n,
                                                        unsigned long long* pairs) {
  __shared__ unsigned long long red[256];
  unsigned long long v = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int B = nt[i], A = ns[i];
    const unsigned long long cb = (unsigned long long)t.count[B], ca = (unsigned long long)t.count[A];
    v += cb * ca - (A == B ? cb : 0ULL);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0]) atomicAdd(pairs, red[0]);
}

constexpr int LTPB = 64;   // one wavefront per target cell
constexpr int NSTAGE = 4;  // row entries staged per round

template <int P>
__global__ __launch_bounds__(LTPB) void k_m2l_list(TreeView t, OpTables op, MacView mv, const double* __restrict__ M,
                                                   double* __restrict__ F, const int* done, const int* qcap) {
  if (done && *done) return;
  constexpr int NC = mi_count(P);
  constexpr int KPT = (NC + LTPB - 1) / LTPB;
  __shared__ double sM[NSTAGE][NC];
  __shared__ double sD[NSTAGE][NC];
  __shared__ int smi[NC];  // exponents of m packed as mx | my << 8 | mz << 16
  const int lane = threadIdx.x;
  const int row = blockIdx.x;
  const int64_t g = (int64_t)t.off[2] + row;
  const int q = qcap ? min(P, max(0, *qcap)) : P;
  const int nq = mi_count(q);
  for (int k = lane; k < NC; k += LTPB) smi[k] = op.mi[3 * k] | (op.mi[3 * k + 1] << 8) | (op.mi[3 * k + 2] << 16);
  int ex[KPT][3], nm[KPT];
  double acc[KPT];
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const int n = lane + r * LTPB;
    acc[r] = 0.0;
    nm[r] = 0;
    ex[r][0] = ex[r][1] = ex[r][2] = 0;
    if (n < nq) {
      for (int a = 0; a < 3; ++a) ex[r][a] = op.mi[3 * n + a];
      nm[r] = mi_count(q - ex[r][0] - ex[r][1] - ex[r][2]);
    }
  }
  const int e0 = mv.mptr[row], e1 = mv.mptr[row + 1];
  const int stride = op.stride;
  for (int eb = e0; eb < e1; eb += NSTAGE) {
    const int nb = min(NSTAGE, e1 - eb);
    __syncthreads();  // the previous round's staged rows are no longer read
    for (int b = 0; b < nb; ++b) {
      const unsigned long long v = mv.mval[eb + b];
      const double* Ms = M + (int64_t)(v >> 32) * stride;
      const double* Ds = mv.dvec + (int64_t)(v & 0xffffffffULL) * NC;
      for (int k = lane; k < nq; k += LTPB) {
        sM[b][k] = Ms[k];
        sD[b][k] = Ds[k];
      }
    }
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        double a = acc[r];
        for (int m = 0; m < nm[r]; ++m) {
          const int e = smi[m];
          a += sD[b][mi_index(ex[r][0] + (e & 255), ex[r][1] + ((e >> 8) & 255), ex[r][2] + (e >> 16))] * sM[b][m];
        }
        acc[r] = a;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const int n = lane + r * LTPB;
    if (n < NC) F[g * stride + n] = n < nq ? acc[r] : 0.0;
  }
}

int grid_of(int64_t n, int tpb = 256) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + tpb - 1) / tpb, 65536)); }

}  // namespace

void launch_mac_radii(const TreeView& t, const double4* P, int level, double* renc, hipStream_t s) {
  const int nc = t.off[level + 1] - t.off[level];
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_mac_radii, dim3(nc), dim3(RTPB), 0, s, t, P, level, renc);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_classify(const TreeView& t, const double* renc, double theta, int ndirect, bool leaf_direct,
                         int level, const int2* fr, int nfr, int* acc, int* kid, hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_classify, dim3(grid_of(nfr)), dim3(256), 0, s, t, renc, theta, ndirect,
                     leaf_direct ? 1 : 0, level, fr, nfr, acc, kid);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_emit(const TreeView& t, int R, int level, const int2* fr, int nfr, const int* acc_scan,
                     const int* kid_scan, int* m_tgt, unsigned long long* m_val, int2* next, int* near_tgt,
                     int* near_src, int* bad, hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_emit, dim3(grid_of(nfr)), dim3(256), 0, s, t, R, level, fr, nfr, acc_scan, kid_scan,
                     m_tgt, m_val, next, near_tgt, near_src, bad);
  PFMM_LAUNCH_CHECK();
}

size_t mac_sort_temp_bytes(int n, int end_bit, bool wide) {
  size_t b = 0;
  if (wide)
    PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const int*)nullptr, (int*)nullptr,
                                                (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                                n, 0, end_bit));
  else
    PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const int*)nullptr, (int*)nullptr, (const int*)nullptr,
                                                (int*)nullptr, n, 0, end_bit));
  return std::max<size_t>(b, 16);
}

void launch_mac_sort(void* tmp, size_t tmp_bytes, const int* kin, int* kout, const void* vin, void* vout, int n,
                     int end_bit, bool wide, hipStream_t s) {
  if (n <= 0) return;
  if (wide)
    PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, (const unsigned long long*)vin,
                                                (unsigned long long*)vout, n, 0, end_bit, s));
  else
    PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, (const int*)vin, (int*)vout, n, 0,
                                                end_bit, s));
}

void launch_mac_count(const int* keys, int n, int key0, int* cnt, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mac_count, dim3(grid_of(n)), dim3(256), 0, s, keys, n, key0, cnt);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_near_pairs(const TreeView& t, const int* near_tgt, const int* near_src, int n,
                           unsigned long long* pairs, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mac_near_pairs, dim3(std::min(grid_of(n), 1024)), dim3(256), 0, s, t, near_tgt, near_src, n,
                     pairs);
  PFMM_LAUNCH_CHECK();
}

void launch_m2l_list(const TreeView& t, const OpTables& op, const MacView& mv, const double* M, double* F,
                     const int* done, const int* qcap, hipStream_t s) {
  if (t.L < 2) return;
  const int rows = t.ncell - t.off[2];
  if (rows <= 0) return;
#define PFMM_M2L_LIST(PP)                                                                                   \
  case PP:                                                                                                   \
    hipLaunchKernelGGL(k_m2l_list<PP>, dim3(rows), dim3(LTPB), 0, s, t, op, mv, M, F, done, qcap);            \
    break;
  switch (op.p) {
    PFMM_M2L_LIST(1) PFMM_M2L_LIST(2) PFMM_M2L_LIST(3) PFMM_M2L_LIST(4) PFMM_M2L_LIST(5)
    PFMM_M2L_LIST(6) PFMM_M2L_LIST(7) PFMM_M2L_LIST(8) PFMM_M2L_LIST(9) PFMM_M2L_LIST(10)
    default: throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  }
#undef PFMM_M2L_LIST
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

// The multipole acceptance criterion and dual tree walk of Sec. III (eq. mac) on the octree.
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
//   * otherwise split: replaced by the pairs of the two cells' non-empty children.
// Each level is a classify pass, inclusive prefix sums and an emit pass, so the outputs come out in
// one fixed order.  Every ordered pair of particles is covered exactly once: by the M2L of the one
// accepted pair of their ancestors, or by the near field of their leaves.
//
// Outputs: the near list, sorted by target leaf (a stable radix sort), for the P2P; the number of
// accepted pairs; and for every cell of levels < L the table of its split partners.  A split pair
// whose children can be accepted failed the criterion, so theta |D| w <= r_B + r_A <= sqrt(3) w: its
// offset lies within Rp = floor(sqrt(3) / theta) cells (or it is adjacent).  The M2L kernel walks
// these partners as the ws lists' colleagues and applies the criterion to their children itself
// (mac.hpp), so the accepted pairs need not be stored.
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"
#include "mac.hpp"

namespace pfmm {

namespace {

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
  mac_coords(t.key[g], c);
  double z[3];
  for (int a = 0; a < 3; ++a) z[a] = __dadd_rn(t.origin[a], __dmul_rn((double)c[a] + 0.5, w));
  const int first = t.first[g], cnt = t.count[g];
  double r = 0.0;
  for (int k = threadIdx.x; k < cnt; k += RTPB) {
    const double4 p = P[first + k];
    r = fmax(r, mac_length3(__dsub_rn(p.x, z[0]), __dsub_rn(p.y, z[1]), __dsub_rn(p.z, z[2])));
  }
  red[threadIdx.x] = r;
  __syncthreads();
  for (int h = RTPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) renc[g] = red[0];
}

__global__ __launch_bounds__(256) void k_mac_classify(TreeView t, MacView mv, int level, const int2* __restrict__ fr,
                                                      int nfr, int* __restrict__ acc, int* __restrict__ kid) {
  const double w = ldexp(t.w, t.L - level);
  const bool leaves_direct = mv.leaf_direct && level == t.L;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    const int B = fr[i].x, A = fr[i].y;
    bool accept = false;
    if (!leaves_direct) {
      int cb[3], ca[3];
      mac_coords(t.key[B], cb);
      mac_coords(t.key[A], ca);
      accept = mac_accept(t, mv.renc, mv.theta, mv.ndirect, w, B, A, cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2]);
    }
    acc[i] = accept ? 1 : 0;
    kid[i] = accept ? 0 : (level == t.L ? 1 : child_count(t, B) * child_count(t, A));
  }
}

__global__ __launch_bounds__(256) void k_mac_emit(TreeView t, MacView mv, int level, const int2* __restrict__ fr,
                                                  int nfr, const int* __restrict__ acc_scan,
                                                  const int* __restrict__ kid_scan, int2* __restrict__ next,
                                                  int* __restrict__ split, int* __restrict__ near_tgt,
                                                  int* __restrict__ near_src, int* bad) {
  const int side = 2 * mv.Rp + 1, nn = side * side * side;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    const int B = fr[i].x, A = fr[i].y;
    const int a0 = i ? acc_scan[i - 1] : 0, k0 = i ? kid_scan[i - 1] : 0;
    if (acc_scan[i] > a0 || kid_scan[i] == k0) continue;  // accepted (counted only), or nothing below
    if (level == t.L) {
      near_tgt[k0] = B;
      near_src[k0] = A;
      continue;
    }
    int pos = k0;
    for (int ob = 0; ob < 8; ++ob) {
      const int b = t.child8[8 * B + ob];
      if (b < 0) continue;
      for (int oa = 0; oa < 8; ++oa) {
        const int a = t.child8[8 * A + oa];
        if (a >= 0) next[pos++] = make_int2(b, a);
      }
    }
    int cb[3], ca[3];
    mac_coords(t.key[B], cb);
    mac_coords(t.key[A], ca);
    const int e0 = ca[0] - cb[0], e1 = ca[1] - cb[1], e2 = ca[2] - cb[2];
    if (max(abs(e0), max(abs(e1), abs(e2))) <= mv.Rp)
      split[(int64_t)B * nn + ((e0 + mv.Rp) * side + (e1 + mv.Rp)) * side + (e2 + mv.Rp)] = A;
    else if (t.count[B] + t.count[A] >= mv.ndirect)
      atomicOr(bad, 1);  // split by the criterion farther out than the radii allow
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

int grid_of(int64_t n, int tpb = 256) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + tpb - 1) / tpb, 65536)); }

}  // namespace

void launch_mac_radii(const TreeView& t, const double4* P, int level, double* renc, hipStream_t s) {
  const int nc = t.off[level + 1] - t.off[level];
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_mac_radii, dim3(nc), dim3(RTPB), 0, s, t, P, level, renc);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_classify(const TreeView& t, const MacView& mv, int level, const int2* fr, int nfr, int* acc, int* kid,
                         hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_classify, dim3(grid_of(nfr)), dim3(256), 0, s, t, mv, level, fr, nfr, acc, kid);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_emit(const TreeView& t, const MacView& mv, int level, const int2* fr, int nfr, const int* acc_scan,
                     const int* kid_scan, int2* next, int* split, int* near_tgt, int* near_src, int* bad,
                     hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_emit, dim3(grid_of(nfr)), dim3(256), 0, s, t, mv, level, fr, nfr, acc_scan, kid_scan,
                     next, split, near_tgt, near_src, bad);
  PFMM_LAUNCH_CHECK();
}

size_t mac_sort_temp_bytes(int n, int end_bit) {
  size_t b = 0;
  PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const int*)nullptr, (int*)nullptr, (const int*)nullptr,
                                              (int*)nullptr, n, 0, end_bit));
  return std::max<size_t>(b, 16);
}

void launch_mac_sort(void* tmp, size_t tmp_bytes, const int* kin, int* kout, const int* vin, int* vout, int n,
                     int end_bit, hipStream_t s) {
  if (n <= 0) return;
  PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, end_bit, s));
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

}  // namespace pfmm

// The dual tree walk of Sec. III on the octree: the multipole acceptance criterion (eq. mac), the
// well-separation rule, and the adaptive octree whose cells split only above leaf_max particles.
//
// A cell's enclosing radius r is the largest distance from its centre (the centre of its
// expansions) to one of its particles.  The walk goes level by level over a frontier of cell pairs
// (target B, source A) of one level, starting from (root, root).  A pair is
//   * accepted for M2L when A != B, the two cells are at Chebyshev distance >= minsep (with the
//     criterion 2, so that every pair of particles closer than a leaf edge, and with it every
//     Thole-damped pair, stays in the direct part; with the ws rule ws + 1), they hold at least
//     ndirect particles together, they are not two terminal cells when leaf pairs are direct, and,
//     with the criterion, theta |z_B - z_A| > r_B + r_A (the children of a pair below ndirect hold
//     fewer particles still, so its descendants are all direct: the paper's direct interaction of
//     small pairs and of leaves);
//   * otherwise, when both cells are terminal (level L; on the adaptive octree every cell that is not
//     split), summed directly: one near-list entry per level-L cell below B, with source A;
//   * otherwise split: replaced by the pairs of the two cells' non-empty children.
// Each level is a classify pass, inclusive prefix sums and an emit pass, so the outputs come out in
// one fixed order.  Every ordered pair of particles is covered exactly once: by the M2L of the one
// accepted pair of their ancestors, or by one direct pair of cells holding them.
//
// Outputs: the near list, sorted by target (a stable radix sort), for the P2P; the number of
// accepted pairs; and for every cell of levels < L the table of its split partners.  A split pair
// whose children can be accepted failed the criterion (or the ws rule), so theta |D| w <=
// r_B + r_A <= sqrt(3) w (or |D| <= ws): its offset lies within Rp = floor(sqrt(3) / theta) (or ws)
// cells.  The M2L kernel walks these partners as the ws lists' colleagues and applies the rule to
// their children itself (mac.hpp), so the accepted pairs need not be stored.
//
// Adaptive octree: the cells below a leaf keep their expansions (P2M at level L, M2M, L2L and L2P
// there are exact translations of the leaf's own), so when a leaf meets a finer neighbour the walk
// splits both and the leaf's part of the interaction runs at the neighbour's level.
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
                                                      int nfr, int* __restrict__ acc, int* __restrict__ kid,
                                                      int* __restrict__ nearc) {
  const double w = ldexp(t.w, t.L - level);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    const int B = fr[i].x, A = fr[i].y;
    int cb[3], ca[3];
    mac_coords(t.key[B], cb);
    mac_coords(t.key[A], ca);
    const bool accept = mac_accept(t, mv, w, B, A, cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2]);
    const bool direct = !accept && mac_terminal(t, mv, B) && mac_terminal(t, mv, A);
    acc[i] = accept ? 1 : 0;
    kid[i] = accept || direct ? 0 : child_count(t, B) * child_count(t, A);
    nearc[i] = direct ? (mv.lcount ? mv.lcount[B] : 1) : 0;
  }
}

// useful flops of the accepted pairs of a frontier, 2 C(q + 6, 6) per pair at its order q (p with
// the criterion; the ws lists' per-offset order with the ws rule): st[0] at the pairs' orders,
// st[1 + c] with every order capped at c <= p
__global__ __launch_bounds__(256) void k_mac_flops(TreeView t, MacView mv, const int2* __restrict__ fr, int nfr,
                                                   const int* __restrict__ acc, const unsigned char* __restrict__ dorder,
                                                   int p, unsigned long long* st) {
  __shared__ unsigned long long red[256];
  auto fl = [](unsigned long long q) {
    return 2 * ((q + 1) * (q + 2) * (q + 3) * (q + 4) * (q + 5) * (q + 6) / 720);
  };
  unsigned long long f[MAX_P + 2] = {};
  const int R = 2 * mv.Rp + 1, cube = 2 * R + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    if (!acc[i]) continue;
    int q = p;
    if (!mv.use_theta) {
      int cb[3], ca[3];
      mac_coords(t.key[fr[i].x], cb);
      mac_coords(t.key[fr[i].y], ca);
      q = min(p, (int)dorder[((cb[0] - ca[0] + R) * cube + (cb[1] - ca[1] + R)) * cube + (cb[2] - ca[2] + R)]);
    }
    f[0] += fl(q);
#pragma unroll
    for (int c = 0; c <= MAX_P; ++c)
      if (c <= p) f[1 + c] += fl(min(q, c));
  }
  for (int k = 0; k < MAX_P + 2; ++k) {
    red[threadIdx.x] = f[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(&st[k], red[0]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_mac_emit(TreeView t, MacView mv, int level, const int2* __restrict__ fr,
                                                  int nfr, const int* __restrict__ kid_scan,
                                                  const int* __restrict__ near_scan,
                                                  int2* __restrict__ next, int* __restrict__ split,
                                                  int* __restrict__ near_tgt, int* __restrict__ near_src, int* bad) {
  const int side = 2 * mv.Rp + 1, nn = side * side * side;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfr; i += gridDim.x * blockDim.x) {
    const int B = fr[i].x, A = fr[i].y;
    const int k0 = i ? kid_scan[i - 1] : 0, n0 = i ? near_scan[i - 1] : 0;
    if (near_scan[i] > n0) {
      // the level-L cells below B (B itself at level L), each with the source cell A
      const int b0 = mv.lfirst ? mv.lfirst[B] : B, nb = near_scan[i] - n0;
      for (int j = 0; j < nb; ++j) {
        near_tgt[n0 + j] = b0 + j;
        near_src[n0 + j] = A;
      }
      continue;
    }
    if (kid_scan[i] == k0) continue;  // accepted (counted only)
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

// the cells of a level holding more than leaf_max particles (never at level L) are split
__global__ __launch_bounds__(256) void k_adapt_init(TreeView t, int level, int leaf_max, int* __restrict__ nonleaf) {
  const int n = t.off[level + 1] - t.off[level];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = t.off[level] + i;
    nonleaf[g] = level < t.L && t.count[g] > leaf_max ? 1 : 0;
  }
}

// index of the cell with key want among the cells of a level, or -1
__device__ inline int find_cell(const TreeView& t, int level, uint64_t want) {
  int lo = t.off[level], hi = t.off[level + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const uint64_t km = t.key[mid];
    if (km == want) return mid;
    if (km < want) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// For each split cell c of level l + 1: the cells of level l whose closed boxes touch c's.  In units
// of level l + 1 a cell b of level l spans [2 b, 2 b + 2] and c spans [c, c + 1] on each axis, so they
// touch when b is (c - 1) >> 1 or (c + 1) >> 1 on every axis (one of them c's parent).
__global__ __launch_bounds__(256) void k_adapt_balance(TreeView t, int level, int* __restrict__ nonleaf) {
  const int n = t.off[level + 2] - t.off[level + 1];
  const int lim = 1 << level;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 8 * n; i += gridDim.x * blockDim.x) {
    const int g = t.off[level + 1] + i / 8, v = i % 8;
    if (!nonleaf[g]) continue;
    int c[3];
    mac_coords(t.key[g], c);
    const int bx = (c[0] + ((v >> 2) & 1 ? 1 : -1)) >> 1;
    const int by = (c[1] + ((v >> 1) & 1 ? 1 : -1)) >> 1;
    const int bz = (c[2] + (v & 1 ? 1 : -1)) >> 1;
    if (bx < 0 || by < 0 || bz < 0 || bx >= lim || by >= lim || bz >= lim) continue;
    const int b = find_cell(t, level, morton3(bx, by, bz));
    if (b >= 0) nonleaf[b] = 1;  // every writer stores the same value
  }
}

// the level-L cells below each cell of a level: keys in [k 8^(L - l), (k + 1) 8^(L - l))
__global__ __launch_bounds__(256) void k_leaf_range(TreeView t, int level, int* __restrict__ lfirst,
                                                    int* __restrict__ lcount) {
  const int n = t.off[level + 1] - t.off[level];
  const int sh = 3 * (t.L - level);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = t.off[level] + i;
    const uint64_t lo_key = t.key[g] << sh, hi_key = (t.key[g] + 1) << sh;
    auto lower = [&](uint64_t want) {  // first level-L cell with key >= want
      int lo = t.off[t.L], hi = t.off[t.L + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t.key[mid] < want) lo = mid + 1; else hi = mid;
      }
      return lo;
    };
    const int f = lower(lo_key);
    lfirst[g] = f;
    lcount[g] = lower(hi_key) - f;
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
    const bool inside = t.first[B] >= t.first[A] && t.first[B] < t.first[A] + t.count[A];
    v += cb * ca - (inside ? cb : 0ULL);
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
                         int* nearc, hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_classify, dim3(grid_of(nfr)), dim3(256), 0, s, t, mv, level, fr, nfr, acc, kid, nearc);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_flops(const TreeView& t, const MacView& mv, const int2* fr, int nfr, const int* acc,
                      const unsigned char* dorder, int p, unsigned long long* st, hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_flops, dim3(std::min(grid_of(nfr), 1024)), dim3(256), 0, s, t, mv, fr, nfr, acc, dorder,
                     p, st);
  PFMM_LAUNCH_CHECK();
}

void launch_mac_emit(const TreeView& t, const MacView& mv, int level, const int2* fr, int nfr, const int* kid_scan,
                     const int* near_scan, int2* next, int* split, int* near_tgt, int* near_src, int* bad,
                     hipStream_t s) {
  if (nfr <= 0) return;
  hipLaunchKernelGGL(k_mac_emit, dim3(grid_of(nfr)), dim3(256), 0, s, t, mv, level, fr, nfr, kid_scan, near_scan,
                     next, split, near_tgt, near_src, bad);
  PFMM_LAUNCH_CHECK();
}

void launch_adapt_init(const TreeView& t, int level, int leaf_max, int* nonleaf, hipStream_t s) {
  const int n = t.off[level + 1] - t.off[level];
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adapt_init, dim3(grid_of(n)), dim3(256), 0, s, t, level, leaf_max, nonleaf);
  PFMM_LAUNCH_CHECK();
}

void launch_adapt_balance(const TreeView& t, int level, int* nonleaf, hipStream_t s) {
  if (level < 0 || level >= t.L) return;
  const int n = t.off[level + 2] - t.off[level + 1];
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adapt_balance, dim3(grid_of(8 * (int64_t)n)), dim3(256), 0, s, t, level, nonleaf);
  PFMM_LAUNCH_CHECK();
}

void launch_leaf_range(const TreeView& t, int level, int* lfirst, int* lcount, hipStream_t s) {
  const int n = t.off[level + 1] - t.off[level];
  if (n <= 0) return;
  hipLaunchKernelGGL(k_leaf_range, dim3(grid_of(n)), dim3(256), 0, s, t, level, lfirst, lcount);
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

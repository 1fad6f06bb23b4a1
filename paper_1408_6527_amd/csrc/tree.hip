// Octree construction on the device: input scan and bounding box, Morton keys, key sort, level
// cells, parent/child links and colleague lists.  All passes are memory-bound integer work.
//
// The paper builds an adaptive kd-tree (Sec. III); this library uses a uniform-depth octree whose
// cells at one level are a regular grid, so that every M2L between cells at the same relative
// offset uses the same operator (see m2l.hip).
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"
#include "morton.hpp"

namespace pfmm {

namespace {

constexpr int TPB = 256;

inline int grid_for(int64_t n, int tpb = TPB, int cap = 1 << 20) {
  int64_t g = (n + tpb - 1) / tpb;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// flags bit 0: non-finite input; bit 1: negative polarisability.  Per-block partials of
// (min x, min y, min z, max x, max y, max z, max alpha).  q may be null (no charges).
constexpr int NRED = 7;

__global__ __launch_bounds__(TPB) void k_scan_inputs(const double* __restrict__ pos,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ alpha, int n,
                                                     double* __restrict__ partial, int* flags) {
  __shared__ double red[NRED][TPB];
  double v[NRED] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  int f = 0;
  for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const double qi = q ? q[i] : 0.0, ai = alpha[i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(qi) || !isfinite(ai)) f |= 1;
    if (ai < 0.0) f |= 2;
    v[0] = fmin(v[0], x); v[1] = fmin(v[1], y); v[2] = fmin(v[2], z);
    v[3] = fmax(v[3], x); v[4] = fmax(v[4], y); v[5] = fmax(v[5], z);
    v[6] = fmax(v[6], ai);
  }
  if (f) atomicOr(flags, f);
  for (int a = 0; a < NRED; ++a) red[a][threadIdx.x] = v[a];
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + h]);
      for (int a = 3; a < NRED; ++a) red[a][threadIdx.x] = fmax(red[a][threadIdx.x], red[a][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < NRED) partial[blockIdx.x * NRED + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(TPB) void k_bbox_final(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ bbox) {
  __shared__ double red[NRED][TPB];
  double v[NRED] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int b = threadIdx.x; b < nblk; b += TPB) {
    for (int a = 0; a < 3; ++a) v[a] = fmin(v[a], partial[NRED * b + a]);
    for (int a = 3; a < NRED; ++a) v[a] = fmax(v[a], partial[NRED * b + a]);
  }
  for (int a = 0; a < NRED; ++a) red[a][threadIdx.x] = v[a];
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + h]);
      for (int a = 3; a < NRED; ++a) red[a][threadIdx.x] = fmax(red[a][threadIdx.x], red[a][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < NRED) bbox[threadIdx.x] = red[threadIdx.x][0];
}

// Leaf coordinate i_a = floor((x_a - o_a) / w), clamped to [0, 2^L - 1]; key = Morton interleave.
__global__ __launch_bounds__(TPB) void k_morton(const double* __restrict__ pos, int n, double ox,
                                                double oy, double oz, double w, int L,
                                                uint64_t* __restrict__ keys, int* __restrict__ vals) {
  const int hiC = (1 << L) - 1;
  for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
    int c[3];
    const double o[3] = {ox, oy, oz};
    for (int a = 0; a < 3; ++a) {
      double t = floor((pos[3 * i + a] - o[a]) / w);
      t = fmin(fmax(t, 0.0), (double)hiC);
      c[a] = (int)t;
    }
    keys[i] = morton3(c[0], c[1], c[2]);
    vals[i] = i;
  }
}

__global__ __launch_bounds__(TPB) void k_gather(const int* __restrict__ perm,
                                                const double* __restrict__ pos,
                                                const double* __restrict__ q,
                                                const double* __restrict__ alpha, int n, double sqrt_a,
                                                double4* __restrict__ P, double* __restrict__ al,
                                                double* __restrict__ sqa, double* __restrict__ tau,
                                                double* __restrict__ itau) {
  for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
    const int j = perm[i];
    P[i] = make_double4(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], q ? q[j] : 0.0);
    const double a = alpha[j];
    al[i] = a;
    sqa[i] = sqrt(a);
    const double t = (a > 0.0 && sqrt_a > 0.0) ? sqrt_a * pow(a, 1.0 / 6.0) : 0.0;
    tau[i] = t;
    itau[i] = t > 0.0 ? 1.0 / t : 0.0;
  }
}

__global__ __launch_bounds__(TPB) void k_level_flags(const uint64_t* __restrict__ keys, int n,
                                                     int shift, int* __restrict__ flags) {
  for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB)
    flags[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_level_count(const int* __restrict__ cid, int n, int* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = n > 0 ? cid[n - 1] : 0;
}

__global__ __launch_bounds__(TPB) void k_fill_int(int* __restrict__ p, int64_t count, int v) {
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < count; i += (int64_t)gridDim.x * TPB)
    p[i] = v;
}

__global__ __launch_bounds__(TPB) void k_fill_double(double* __restrict__ p, int64_t count, double v) {
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < count; i += (int64_t)gridDim.x * TPB)
    p[i] = v;
}

__global__ __launch_bounds__(TPB) void k_cells(const uint64_t* __restrict__ keys, int n, int L, int l,
                                               const int* __restrict__ cid_l,
                                               const int* __restrict__ cid_par, int off_l, int off_par,
                                               uint64_t* __restrict__ ckey, int* __restrict__ cfirst,
                                               int* __restrict__ cparent, int* __restrict__ child8) {
  const int shift = 3 * (L - l);
  for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
    const uint64_t k = keys[i] >> shift;
    const bool head = (i == 0) || ((keys[i - 1] >> shift) != k);
    if (!head) continue;
    const int g = off_l + cid_l[i] - 1;
    ckey[g] = k;
    cfirst[g] = i;
    if (l > 0) {
      const int par = off_par + cid_par[i] - 1;
      cparent[g] = par;
      child8[8 * par + (int)(k & 7)] = g;
    } else {
      cparent[g] = -1;
    }
  }
}

__global__ __launch_bounds__(TPB) void k_cell_counts(const int* __restrict__ cfirst, int off_l,
                                                     int ncell_l, int n, int* __restrict__ ccount) {
  for (int c = blockIdx.x * TPB + threadIdx.x; c < ncell_l; c += gridDim.x * TPB) {
    const int nxt = (c + 1 < ncell_l) ? cfirst[off_l + c + 1] : n;
    ccount[off_l + c] = nxt - cfirst[off_l + c];
  }
}

// Colleagues of every cell of level l: the cells at Chebyshev distance <= ws, in offset order
// e = (ex, ey, ez) in [-ws, ws]^3 (x slowest), found by binary search of the Morton key among the
// level's sorted cell keys; -1 where no such cell exists.
__global__ __launch_bounds__(TPB) void k_colleagues(const uint64_t* __restrict__ ckey, int off_l,
                                                    int ncell_l, int l, int ws,
                                                    int* __restrict__ coll) {
  const int side = 2 * ws + 1, nn = side * side * side;
  const int lim = 1 << l;
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < (int64_t)ncell_l * nn;
       t += (int64_t)gridDim.x * TPB) {
    const int c = (int)(t / nn), e = (int)(t % nn);
    const uint64_t k = ckey[off_l + c];
    const int x = compact3(k >> 2) + e / (side * side) - ws;
    const int y = compact3(k >> 1) + (e / side) % side - ws;
    const int z = compact3(k) + e % side - ws;
    int found = -1;
    if (x >= 0 && y >= 0 && z >= 0 && x < lim && y < lim && z < lim) {
      const uint64_t want = morton3(x, y, z);
      int lo = 0, hi = ncell_l - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const uint64_t km = ckey[off_l + mid];
        if (km == want) { found = off_l + mid; break; }
        if (km < want) lo = mid + 1; else hi = mid - 1;
      }
    }
    coll[(int64_t)(off_l + c) * nn + e] = found;
  }
}

// stats[0] += M2L pairs with a non-empty source; stats[1] += ordered near-field particle pairs;
// stats[2] += useful M2L flops, 2 C(q+6, 6) per pair at its truncation order q.
__device__ __forceinline__ unsigned long long m2l_pair_flops(unsigned long long q) {
  return 2 * ((q + 1) * (q + 2) * (q + 3) * (q + 4) * (q + 5) * (q + 6) / 720);
}

__global__ __launch_bounds__(TPB) void k_tree_stats(TreeView t, const int* __restrict__ m2l_code,
                                                    const unsigned char* __restrict__ dorder, int noff, int p,
                                                    unsigned long long* stats) {
  const int first2 = t.L >= 2 ? t.off[2] : t.ncell;
  unsigned long long m2l = 0, p2p = 0, flops = 0;
  unsigned long long fcap[MAX_P + 1] = {};
  for (int g = blockIdx.x * TPB + threadIdx.x; g < t.ncell; g += gridDim.x * TPB) {
    if (g >= first2) {
      const int oct = (int)(t.key[g] & 7);
      const int par = t.parent[g];
      for (int j = 0; j < noff; ++j) {
        const int code = m2l_code[oct * noff + j];
        const int pc = t.coll[(int64_t)par * t.nnear + ((code >> 12) & 0xff)];
        if (pc >= 0 && t.child8[8 * pc + ((code >> 20) & 7)] >= 0) {
          ++m2l;
          const unsigned long long q = dorder[code & 0xfff];
          flops += m2l_pair_flops(q);
#pragma unroll
          for (int c = 0; c <= MAX_P; ++c)
            if (c <= p) fcap[c] += m2l_pair_flops(q < (unsigned long long)c ? q : (unsigned long long)c);
        }
      }
    }
    if (g >= t.off[t.L]) {
      const int cb = t.count[g];
      for (int k = 0; k < t.nnear; ++k) {
        const int a = t.coll[(int64_t)g * t.nnear + k];
        if (a >= 0) p2p += (unsigned long long)cb * (unsigned long long)t.count[a];
      }
      p2p -= (unsigned long long)cb;
    }
  }
  if (m2l) atomicAdd(&stats[0], m2l);
  if (p2p) atomicAdd(&stats[1], p2p);
  if (flops) atomicAdd(&stats[2], flops);
#pragma unroll
  for (int c = 0; c <= MAX_P; ++c)
    if (c <= p && fcap[c]) atomicAdd(&stats[3 + c], fcap[c]);
}

}  // namespace

void launch_scan_inputs(const double* pos, const double* q, const double* alpha, int n,
                        double* partial, int nblk, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_inputs, dim3(nblk), dim3(TPB), 0, s, pos, q, alpha, n, partial, flags);
  PFMM_LAUNCH_CHECK();
}

void launch_bbox_final(const double* partial, int nblk, double* bbox, hipStream_t s) {
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(TPB), 0, s, partial, nblk, bbox);
  PFMM_LAUNCH_CHECK();
}

void launch_morton(const double* pos, int n, const double origin[3], double w, int L,
                   uint64_t* keys, int* vals, hipStream_t s) {
  hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(TPB), 0, s, pos, n, origin[0], origin[1],
                     origin[2], w, L, keys, vals);
  PFMM_LAUNCH_CHECK();
}

size_t sort_temp_bytes(int n, int end_bit) {
  size_t bytes = 0;
  PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr,
                                               (uint64_t*)nullptr, (const int*)nullptr,
                                               (int*)nullptr, n, 0, end_bit));
  return bytes;
}

void launch_sort(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin,
                 int* vout, int n, int end_bit, hipStream_t s) {
  PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, end_bit, s));
}

void launch_gather(const int* perm, const double* pos, const double* q, const double* alpha, int n,
                   double sqrt_a, double4* P, double* al, double* sqa, double* tau, double* itau,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(TPB), 0, s, perm, pos, q, alpha, n, sqrt_a,
                     P, al, sqa, tau, itau);
  PFMM_LAUNCH_CHECK();
}

size_t scan_temp_bytes(int n) {
  size_t bytes = 0;
  PFMM_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, (const int*)nullptr, (int*)nullptr, n));
  return bytes;
}

void launch_inclusive_scan(void* tmp, size_t tmp_bytes, const int* in, int* out, int n, hipStream_t s) {
  PFMM_HIP(hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, in, out, n, s));
}

void launch_level_scan(const uint64_t* keys, int n, int shift, int* flags, int* cid, int* count_out,
                       void* tmp, size_t tmp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_level_flags, dim3(grid_for(n)), dim3(TPB), 0, s, keys, n, shift, flags);
  PFMM_LAUNCH_CHECK();
  PFMM_HIP(hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, flags, cid, n, s));
  hipLaunchKernelGGL(k_level_count, dim3(1), dim3(64), 0, s, cid, n, count_out);
  PFMM_LAUNCH_CHECK();
}

void launch_fill_int(int* p, int64_t count, int value, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3(grid_for(count, TPB, 4096)), dim3(TPB), 0, s, p, count, value);
  PFMM_LAUNCH_CHECK();
}

void launch_fill_double(double* p, int64_t count, double value, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_double, dim3(grid_for(count, TPB, 4096)), dim3(TPB), 0, s, p, count,
                     value);
  PFMM_LAUNCH_CHECK();
}

void launch_cells(const uint64_t* keys, int n, int L, int l, const int* cid_l, const int* cid_parent,
                  int off_l, int off_parent, uint64_t* ckey, int* cfirst, int* cparent, int* child8,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_cells, dim3(grid_for(n)), dim3(TPB), 0, s, keys, n, L, l, cid_l, cid_parent,
                     off_l, off_parent, ckey, cfirst, cparent, child8);
  PFMM_LAUNCH_CHECK();
}

void launch_cell_counts(const int* cfirst, int off_l, int ncell_l, int n, int* ccount, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_counts, dim3(grid_for(ncell_l)), dim3(TPB), 0, s, cfirst, off_l, ncell_l,
                     n, ccount);
  PFMM_LAUNCH_CHECK();
}

void launch_colleagues(const uint64_t* ckey, int off_l, int ncell_l, int l, int ws, int* coll,
                       hipStream_t s) {
  const int side = 2 * ws + 1;
  hipLaunchKernelGGL(k_colleagues, dim3(grid_for((int64_t)ncell_l * side * side * side)), dim3(TPB),
                     0, s, ckey, off_l, ncell_l, l, ws, coll);
  PFMM_LAUNCH_CHECK();
}

void launch_tree_stats(const TreeView& t, const int* m2l_code, const unsigned char* dorder, int noff,
                       int p, unsigned long long* stats, hipStream_t s) {
  if (p < 0 || p > MAX_P) throw Error(PFMM_ERR_INVALID_ARG, "internal: order out of range in tree stats");
  hipLaunchKernelGGL(k_tree_stats, dim3(grid_for(t.ncell)), dim3(TPB), 0, s, t, m2l_code, dorder, noff, p,
                     stats);
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

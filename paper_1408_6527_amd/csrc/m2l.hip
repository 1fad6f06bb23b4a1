// M2L on the matrix cores (Sec. II.B, local expansion from a multipole expansion):
//   F~_n(B) = sum_{|m| <= p - |n|} D_{n+m}(d) M~_m(A),   d = B - A in cells of the level.
//
// In level-scaled form the operator depends only on the integer offset d, so all cell pairs at
// the same offset share one matrix K_d (homogeneity of 1/r).  A target B in octant o of its
// parent meets the same set of offsets as every other target in octant o, so targets are grouped
// by octant into tiles of 16 (one wavefront each).  For each offset the wave gathers the 16
// source expansions as the B operand of 16x16x4 MFMAs and multiplies them by K_d, block by block
// along the degree staircase (schedule.hpp).  Accumulators stay in registers for the whole offset
// loop and every target's F~ is written exactly once: no atomics, deterministic.
//
// FP64 path: v_mfma_f64_16x16x4f64.  Mixed path: v_mfma_f32_16x16x4f32 with float32 K and
// operands and float32 accumulation, except for targets at levels <= fp64_max_level.
#include <hipcub/hipcub.hpp>

#include <type_traits>

#include "kernels.hpp"
#include "schedule.hpp"

namespace pfmm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TPB = 256;
constexpr int WAVES = TPB / 64;

__device__ inline int level_of(const TreeView& t, int g) {
  int l = 0;
  while (l < t.L && g >= t.off[l + 1]) ++l;
  return l;
}

__global__ __launch_bounds__(TPB) void k_octant_keys(TreeView t, int* __restrict__ keys,
                                                     int* __restrict__ vals,
                                                     int* __restrict__ oct_count) {
  const int g0 = t.off[2];
  const int n = t.ncell - g0;
  for (int i = blockIdx.x * TPB + threadIdx.x; i < n; i += gridDim.x * TPB) {
    const int g = g0 + i;
    const int o = (int)(t.key[g] & 7);
    keys[i] = o;
    vals[i] = g;
    atomicAdd(&oct_count[o], 1);
  }
}

// Wave-tile w of octant o covers targets [16 (w - tile0(o)), +16) of that octant's segment.
__device__ inline bool locate_tile(const int* oct_count, int wtile, int& o, int& seg_start,
                                   int& in_oct) {
  int tstart = 0, start = 0;
  for (int oc = 0; oc < 8; ++oc) {
    const int cnt = oct_count[oc];
    const int nt = (cnt + 15) >> 4;
    if (wtile < tstart + nt) {
      o = oc;
      seg_start = start;
      in_oct = wtile - tstart;
      return true;
    }
    tstart += nt;
    start += cnt;
  }
  return false;
}

// Source cell of every (tile, offset, column): list[(tile * noff + j) * 16 + col], -1 if empty.
__global__ __launch_bounds__(TPB) void k_m2l_list(TreeView t, const int* __restrict__ m2l_code,
                                                  int noff, const int* __restrict__ tgt_list,
                                                  const int* __restrict__ oct_count, int ntiles,
                                                  int* __restrict__ list) {
  const int64_t total = (int64_t)ntiles * noff * 16;
  for (int64_t idx = blockIdx.x * (int64_t)TPB + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * TPB) {
    const int col = (int)(idx & 15);
    const int j = (int)((idx >> 4) % noff);
    const int tile = (int)((idx >> 4) / noff);
    int o, seg, in_oct;
    int A = -1;
    if (locate_tile(oct_count, tile, o, seg, in_oct)) {
      const int tl = in_oct * 16 + col;
      if (tl < oct_count[o]) {
        const int B = tgt_list[seg + tl];
        const int code = m2l_code[o * noff + j];
        const int pc = t.coll[(int64_t)t.parent[B] * t.nnear + ((code >> 12) & 0xff)];
        if (pc >= 0) A = t.child8[8 * pc + ((code >> 20) & 7)];
      }
    }
    list[idx] = A;
  }
}

template <int P, bool F32>
__global__ __launch_bounds__(TPB) void k_m2l(TreeView t, OpTables op, const int* __restrict__ tgt_list,
                                             const int* __restrict__ oct_count,
                                             const int* __restrict__ list,
                                             const double* __restrict__ M, double* __restrict__ F,
                                             int fp64_max_level, const int* done) {
  if (done && *done) return;
  constexpr int NRB = sched_nrb(P);
  constexpr int MAXS = sched_maxsteps(P);
  constexpr int NB = sched_nblocks(P);
  constexpr int NC = mi_count(P);
  constexpr int STRIDE = sched_stride(P);
  const int lane = threadIdx.x & 63;
  const int wtile = blockIdx.x * WAVES + (threadIdx.x >> 6);
  int o, seg, in_oct;
  if (!locate_tile(oct_count, wtile, o, seg, in_oct)) return;
  const int col = lane & 15;
  const int tl = in_oct * 16 + col;
  int B = tl < oct_count[o] ? tgt_list[seg + tl] : -1;
  if (B >= 0) {
    const int lev = level_of(t, B);
    const bool mine = F32 ? (lev > fp64_max_level) : (lev <= fp64_max_level);
    if (!mine) B = -1;
  }
  if (__ballot(B >= 0) == 0) return;
  const int zero_row = t.ncell;
  const int kq = lane >> 4;

  using acc_t = typename std::conditional<F32, f4, d4>::type;
  acc_t acc[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) acc[rb] = acc_t{0, 0, 0, 0};

  const int* lst = list + (int64_t)wtile * op.noff * 16 + col;
  int A_next = lst[0];
  for (int j = 0; j < op.noff; ++j) {
    const int A = A_next;
    if (j + 1 < op.noff) A_next = lst[(j + 1) * 16];
    const int code = op.m2l_code[o * op.noff + j];
    if (__ballot(A >= 0 && B >= 0) == 0) continue;
    const int src = (A >= 0 && B >= 0) ? A : zero_row;
    const double* Mrow = M + (int64_t)src * STRIDE + kq;
    const int slot = code & 0xfff;
    if constexpr (F32) {
      const float* K = op.kpack32 + (int64_t)slot * NB * 64 + lane;
      int blk = 0;
#pragma unroll
      for (int s = 0; s < MAXS; ++s) {
        const float b = (float)Mrow[4 * s];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          if (sched_nsteps(P, rb) > s) {
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(K[blk * 64], b, acc[rb], 0, 0, 0);
            ++blk;
          }
        }
      }
    } else {
      const double* K = op.kpack + (int64_t)slot * NB * 64 + lane;
      int blk = 0;
#pragma unroll
      for (int s = 0; s < MAXS; ++s) {
        const double b = Mrow[4 * s];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          if (sched_nsteps(P, rb) > s) {
            acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(K[blk * 64], b, acc[rb], 0, 0, 0);
            ++blk;
          }
        }
      }
    }
  }
  if (B < 0) return;
  double* Fr = F + (int64_t)B * STRIDE;
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // f64 16x16x4: lane l, register r holds row 4 r + l/16; f32 16x16x4: row 4 (l/16) + r
      const int row = 16 * rb + (F32 ? (4 * kq + r) : (4 * r + kq));
      if (row < NC) Fr[row] = (double)acc[rb][r];
    }
  }
}

template <int P>
void m2l_dispatch(const TreeView& t, const OpTables& op, const int* tgt, const int* oc,
                  const int* list, int nblk, const double* M, double* F, bool fp32, int fp64_max,
                  const int* done, hipStream_t s) {
  if (!fp32 || fp64_max >= 2)
    hipLaunchKernelGGL((k_m2l<P, false>), dim3(nblk), dim3(TPB), 0, s, t, op, tgt, oc, list, M, F,
                       fp32 ? fp64_max : t.L, done);
  if (fp32)
    hipLaunchKernelGGL((k_m2l<P, true>), dim3(nblk), dim3(TPB), 0, s, t, op, tgt, oc, list, M, F,
                       fp64_max, done);
}

}  // namespace

void launch_octant_keys(const TreeView& t, int* keys, int* vals, int* oct_count, hipStream_t s) {
  const int n = t.ncell - t.off[2];
  if (n <= 0) return;
  int g = (n + TPB - 1) / TPB;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_octant_keys, dim3(g), dim3(TPB), 0, s, t, keys, vals, oct_count);
  PFMM_LAUNCH_CHECK();
}

size_t octsort_temp_bytes(int n) {
  size_t bytes = 0;
  PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const int*)nullptr, (int*)nullptr,
                                               (const int*)nullptr, (int*)nullptr, n, 0, 3));
  return bytes;
}

void launch_octant_sort(void* tmp, size_t bytes, const int* kin, int* kout, const int* vin, int* vout,
                        int n, hipStream_t s) {
  PFMM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, n, 0, 3, s));
}

int m2l_max_tiles(int ntgt) { return (ntgt + 15) / 16 + 8; }

void launch_m2l_list(const TreeView& t, const OpTables& op, const int* tgt_list, const int* oct_count,
                     int ntiles, int* list, hipStream_t s) {
  const int64_t total = (int64_t)ntiles * op.noff * 16;
  if (total <= 0) return;
  int64_t g = (total + TPB - 1) / TPB;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_m2l_list, dim3((int)g), dim3(TPB), 0, s, t, op.m2l_code, op.noff, tgt_list,
                     oct_count, ntiles, list);
  PFMM_LAUNCH_CHECK();
}

void launch_m2l(const TreeView& t, const OpTables& op, const int* tgt_list, const int* oct_count,
                int ntgt, const int* list, const double* M, double* F, bool fp32, int fp64_max_level,
                const int* done, hipStream_t s) {
  if (ntgt <= 0) return;
  const int ntiles = m2l_max_tiles(ntgt);
  const int nblk = (ntiles + WAVES - 1) / WAVES;
  switch (op.p) {
    case 1: m2l_dispatch<1>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 2: m2l_dispatch<2>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 3: m2l_dispatch<3>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 4: m2l_dispatch<4>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 5: m2l_dispatch<5>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 6: m2l_dispatch<6>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 7: m2l_dispatch<7>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 8: m2l_dispatch<8>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 9: m2l_dispatch<9>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    case 10: m2l_dispatch<10>(t, op, tgt_list, oct_count, list, nblk, M, F, fp32, fp64_max_level, done, s); break;
    default: throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  }
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

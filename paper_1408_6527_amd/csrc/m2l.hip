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

// Work split: a workgroup of 4 waves owns 4 * NCB consecutive 16-target tiles of one octant and
// one slice of that octant's offset list (the slices of a target are summed by the downward
// pass).  For every offset in its slice the workgroup stages K_d in LDS once; each wave then runs
// the degree-blocked MFMA schedule on NCB target tiles, reusing every K_d block from LDS NCB times.
// The next offset's K_d is fetched into registers while the current one is being used.
template <int P, bool F32, int NCB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2))) void k_m2l(TreeView t, OpTables op, const int* __restrict__ tgt_list,
                                             const int* __restrict__ oct_count,
                                             const int* __restrict__ list,
                                             const double* __restrict__ M, double* __restrict__ F,
                                             int64_t split_stride, int nsplit, int fp64_max_level,
                                             const int* done) {
  if (done && *done) return;
  using kt = typename std::conditional<F32, float, double>::type;
  using acc_t = typename std::conditional<F32, f4, d4>::type;
  constexpr int NRB = sched_nrb(P);
  constexpr int MAXS = sched_maxsteps(P);
  constexpr int NB = sched_nblocks(P);
  constexpr int NC = mi_count(P);
  constexpr int STRIDE = sched_stride(P);
  constexpr int KSZ = NB * 64;                 // K_d values per offset
  constexpr int KPT = (KSZ + TPB - 1) / TPB;   // K_d values staged per thread
  constexpr int TPW = WAVES * NCB;             // 16-target tiles per workgroup
  __shared__ kt sK[KSZ];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int split = blockIdx.x % nsplit;
  const int wg = blockIdx.x / nsplit;
  // locate the workgroup's octant and its first 16-target tile
  int o = -1, seg = 0, t16_0 = 0, tiles_before = 0, nt_o = 0;
  {
    int wstart = 0, start = 0, tb = 0;
    for (int oc = 0; oc < 8; ++oc) {
      const int cnt = oct_count[oc];
      const int nt = (cnt + 15) >> 4;
      const int nw = (nt + TPW - 1) / TPW;
      if (o < 0 && wg < wstart + nw) {
        o = oc; seg = start; t16_0 = (wg - wstart) * TPW; tiles_before = tb; nt_o = nt;
      }
      wstart += nw; start += cnt; tb += nt;
    }
  }
  if (o < 0) return;  // whole workgroup: no barrier has been reached yet
  const int noff = op.noff;
  const int j0 = (int)((int64_t)noff * split / nsplit), j1 = (int)((int64_t)noff * (split + 1) / nsplit);
  const int col = lane & 15, kq = lane >> 4;
  const int cnt_o = oct_count[o];
  int B[NCB];
  const int* lst[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int t16 = t16_0 + wave * NCB + cb;
    const int tl = t16 * 16 + col;
    int b = (t16 < nt_o && tl < cnt_o) ? tgt_list[seg + tl] : -1;
    if (b >= 0) {
      const int lev = level_of(t, b);
      if (F32 ? (lev <= fp64_max_level) : (lev > fp64_max_level)) b = -1;
    }
    B[cb] = b;
    lst[cb] = list + ((int64_t)(tiles_before + (t16 < nt_o ? t16 : 0)) * noff) * 16 + col;
  }
  {
    // workgroups whose targets all belong to the other precision's kernel leave together
    int mine = 0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) mine |= B[cb] >= 0;
    if (!__syncthreads_or(mine)) return;
  }
  const int zero_row = t.ncell;
  acc_t acc[NCB][NRB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[cb][rb] = acc_t{0, 0, 0, 0};

  const kt* kbase = F32 ? (const kt*)op.kpack32 : (const kt*)op.kpack;
  kt kreg[KPT];
  auto fetch_k = [&](int j) {
    const int slot = op.m2l_code[o * noff + j] & 0xfff;
    const kt* src = kbase + (int64_t)slot * KSZ;
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int e = threadIdx.x + i * TPB;
      kreg[i] = e < KSZ ? src[e] : kt(0);
    }
  };
  if (j0 < j1) fetch_k(j0);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();  // every wave is done with the previous K_d
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int e = threadIdx.x + i * TPB;
      if (e < KSZ) sK[e] = kreg[i];
    }
    __syncthreads();
    if (j + 1 < j1) fetch_k(j + 1);
    int src[NCB];
    bool any = false;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int A = B[cb] >= 0 ? lst[cb][j * 16] : -1;
      src[cb] = A >= 0 ? A : zero_row;
      any |= A >= 0;
    }
    if (__ballot(any) == 0) continue;
    const kt* K = sK + lane;
    int blk = 0;
#pragma unroll
    for (int s2 = 0; s2 < MAXS; s2 += 2) {
      // one 16-byte load per lane serves steps s2 and s2 + 1 (coefficients m(s2, q), m(s2, q) + 1)
      double2 bb[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        bb[cb] = *reinterpret_cast<const double2*>(M + (int64_t)src[cb] * STRIDE + sched_coef(s2, kq));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int s = s2 + h;
        if (s >= MAXS) break;
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          if (sched_nsteps(P, rb) > s) {
            const kt a = K[blk * 64];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
              const kt b = (kt)(h == 0 ? bb[cb].x : bb[cb].y);
              if constexpr (F32)
                acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[cb][rb], 0, 0, 0);
              else
                acc[cb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb][rb], 0, 0, 0);
            }
            ++blk;
          }
        }
      }
    }
  }
  double* Fs = F + (int64_t)split * split_stride;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    if (B[cb] < 0) continue;
    double* Fr = Fs + (int64_t)B[cb] * STRIDE;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4: lane l, register r holds row 4 r + l/16; f32 16x16x4: row 4 (l/16) + r
        const int row = 16 * rb + (F32 ? (4 * kq + r) : (4 * r + kq));
        if (row < NC) Fr[row] = (double)acc[cb][rb][r];
      }
    }
  }
}

template <int P>
constexpr int ncb_for() { return P <= 4 ? 4 : (P <= 6 ? 3 : (P <= 8 ? 2 : 1)); }

template <int P>
int m2l_wgs(const int* oc_host) {
  int n = 0;
  for (int o = 0; o < 8; ++o) n += (((oc_host[o] + 15) >> 4) + WAVES * ncb_for<P>() - 1) / (WAVES * ncb_for<P>());
  return n;
}

template <int P>
void m2l_dispatch(const TreeView& t, const OpTables& op, const int* tgt, const int* oc, const int* list,
                  int nwg, int nsplit, const double* M, double* F, int64_t split_stride, bool fp32,
                  int fp64_max, const int* done, hipStream_t s) {
  constexpr int NCB = ncb_for<P>();
  const int grid = nwg * nsplit;
  if (!fp32 || fp64_max >= 2)
    hipLaunchKernelGGL((k_m2l<P, false, NCB>), dim3(grid), dim3(TPB), 0, s, t, op, tgt, oc, list, M, F,
                       split_stride, nsplit, fp32 ? fp64_max : t.L, done);
  if (fp32)
    hipLaunchKernelGGL((k_m2l<P, true, NCB>), dim3(grid), dim3(TPB), 0, s, t, op, tgt, oc, list, M, F,
                       split_stride, nsplit, fp64_max, done);
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

int m2l_workgroups(int p, const int* oct_count_host) {
  switch (p) {
    case 1: return m2l_wgs<1>(oct_count_host);
    case 2: return m2l_wgs<2>(oct_count_host);
    case 3: return m2l_wgs<3>(oct_count_host);
    case 4: return m2l_wgs<4>(oct_count_host);
    case 5: return m2l_wgs<5>(oct_count_host);
    case 6: return m2l_wgs<6>(oct_count_host);
    case 7: return m2l_wgs<7>(oct_count_host);
    case 8: return m2l_wgs<8>(oct_count_host);
    case 9: return m2l_wgs<9>(oct_count_host);
    case 10: return m2l_wgs<10>(oct_count_host);
  }
  throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
}

void launch_m2l(const TreeView& t, const OpTables& op, const int* tgt_list, const int* oct_count,
                int nwg, int nsplit, const int* list, const double* M, double* F, int64_t split_stride,
                bool fp32, int fp64_max_level, const int* done, hipStream_t s) {
  if (nwg <= 0) return;
  switch (op.p) {
#define PFMM_M2L_CASE(PP)                                                                            \
  case PP:                                                                                           \
    m2l_dispatch<PP>(t, op, tgt_list, oct_count, list, nwg, nsplit, M, F, split_stride, fp32,        \
                     fp64_max_level, done, s);                                                       \
    break;
    PFMM_M2L_CASE(1) PFMM_M2L_CASE(2) PFMM_M2L_CASE(3) PFMM_M2L_CASE(4) PFMM_M2L_CASE(5)
    PFMM_M2L_CASE(6) PFMM_M2L_CASE(7) PFMM_M2L_CASE(8) PFMM_M2L_CASE(9) PFMM_M2L_CASE(10)
#undef PFMM_M2L_CASE
    default: throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  }
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm

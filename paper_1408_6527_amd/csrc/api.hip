// C interface and host orchestration of the pfmm library (declarations in include/pfmm.h).
//
// A solve runs the three stages of Sec. III on one device stream:
//   tree      bounding box, Morton sort, cells, colleagues, M2L launch shape    (tree.hip)
//   stage 1   field of the charges: phi^q, E^q, grad E^q                       (one FMM pass)
//   stage 2   conjugate gradients on (I - S T~ S) y = S E^q, one FMM pass of the
//             dipoles per iteration                                             (solver.hip)
//   stage 3   field of the converged dipoles, energy, forces, un-permutation
// An FMM pass is P2M -> M2M (up) -> M2L -> L2L (down) -> L2P, plus P2P over colleague leaves; with
// mac_theta or adaptive_leaf_max the M2L and P2P run from the lists of the dual tree walk (mac.hip).
#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "schedule.hpp"
#include "tables.hpp"

using namespace pfmm;

namespace {

constexpr int NRED = 7;  // bbox partial width (tree.hip)
constexpr double EANG_TO_DEBYE = 4.80320;

// Device scratch of pfmm_field_noalloc: one array on every GPU the library runs on, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not device memory: its device
// address comes from hipGetSymbolAddress, once per device (scratch_address), and only that address
// is handed to kernels and copies.
constexpr size_t SCRATCH_BYTES = PFMM_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;
__device__ __align__(256) char scratch[SCRATCH_BYTES];
std::mutex g_scratch_mutex;
char* g_scratch[MAX_DEVICES] = {};

// Device address of the scratch array on the current device (looked up on the first call per device).
char* scratch_address() {
  int d = 0;
  PFMM_HIP(hipGetDevice(&d));
  if (d < 0 || d >= MAX_DEVICES) throw Error(PFMM_ERR_INVALID_ARG, "device ordinal out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[d]) {
    void* p = nullptr;
    PFMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(PFMM_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[d] = static_cast<char*>(p);
  }
  return g_scratch[d];
}

// While a pfmm_field_noalloc call runs on this thread, every workspace buffer is carved from the
// scratch array instead of being allocated.
thread_local Arena* g_arena = nullptr;

struct HostPinned {
  void* p = nullptr;
  size_t bytes = 0;
  ~HostPinned() { if (p) (void)hipHostFree(p); }
  void* get(size_t b) {
    if (b > bytes) {
      if (g_arena) throw Error(PFMM_ERR_INVALID_ARG, "host staging buffer too small for an allocation-free call");
      if (p) (void)hipHostFree(p);
      p = nullptr;
      PFMM_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
      bytes = b;
    }
    return p;
  }
};

}  // namespace

// Per-launch HIP events on the call's stream, grouped by kernel class (PFMM_TIMING only).
struct KernelTimer {
  bool on = false;
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> marks;  // (class, index of the start event; end = start + 1)
  std::vector<int> tags;                   // per mark: the M2L truncation cap of the launch (M2L only)
  int tag = -1;                            // cap of the next M2L launch, set by the caller
  size_t used = 0;
  ~KernelTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  void reset(bool on_, hipStream_t s_) {
    on = on_;
    s = s_;
    marks.clear();
    tags.clear();
    used = 0;
  }
  int begin() {
    if (!on) return -1;
    if (used + 2 > pool.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        PFMM_HIP(hipEventCreate(&e));
        pool.push_back(e);
      }
    }
    PFMM_HIP(hipEventRecord(pool[used], s));
    used += 2;
    return (int)used - 2;
  }
  void end(int cls, int start) {
    if (!on || start < 0) return;
    PFMM_HIP(hipEventRecord(pool[start + 1], s));
    marks.emplace_back(cls, start);
    tags.push_back(tag);
  }
  void collect(double* ms, int* count) {
    if (!on) return;
    PFMM_HIP(hipStreamSynchronize(s));
    for (auto& m : marks) {
      float t = 0.f;
      PFMM_HIP(hipEventElapsedTime(&t, pool[m.second], pool[m.second + 1]));
      ms[m.first] += t;
      count[m.first] += 1;
    }
  }
  // M2L launches split into those at the full orders (cap >= p) and the capped ones of a relaxed
  // solve: summed time, launch count and useful flops (flops_full per full launch, flops_cap[c] per
  // launch capped at c).
  void collect_m2l(int cls, int p, int64_t flops_full, const int64_t* flops_cap, double* ms, int* count,
                   int64_t* flops) {
    if (!on) return;
    for (size_t k = 0; k < marks.size(); ++k) {
      if (marks[k].first != cls) continue;
      float t = 0.f;
      PFMM_HIP(hipEventElapsedTime(&t, pool[marks[k].second], pool[marks[k].second + 1]));
      const int c = tags[k] < 0 || tags[k] >= p ? 0 : 1;
      ms[c] += t;
      count[c] += 1;
      flops[c] += c == 0 ? flops_full : flops_cap[tags[k]];
    }
  }
};
// A captured sequence of launches, re-instantiated only when its topology changes
// (hipGraphExecUpdate otherwise refreshes the kernel arguments of the existing executable graph).
// Capture happens on a private stream (the caller's stream may be the null stream, which cannot
// be captured); the executable graph is then launched on the caller's stream.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  ~GraphCache() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
  template <class F>
  void capture(F&& body) {
    if (!cap) PFMM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t s = cap;
    hipGraph_t g = nullptr;
    PFMM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      body();
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(s, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    PFMM_HIP(hipStreamEndCapture(s, &g));
    bool updated = false;
    if (exec) {
      hipGraphNode_t err_node = nullptr;
      hipGraphExecUpdateResult why;
      updated = hipGraphExecUpdate(exec, g, &err_node, &why) == hipSuccess && why == hipGraphExecUpdateSuccess;
      if (!updated) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
      }
    }
    if (!updated) {
      hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        exec = nullptr;
        PFMM_HIP(e);
      }
    }
    PFMM_HIP(hipGraphDestroy(g));
  }
  void launch(hipStream_t s) { PFMM_HIP(hipGraphLaunch(exec, s)); }
};

enum { KC_P2M = 0, KC_M2M, KC_M2L, KC_L2L, KC_L2P, KC_P2P_SCF, KC_P2P_FULL, KC_SOLVER };

struct pfmm_handle {
  KernelTimer kt;
  GraphCache graph;
  pfmm_config cfg{};
  HostTables tab;
  OpTables op;
  int device = 0;
  // constant tables
  DevBuf t_mi, t_p2m, t_ifact, t_l2p, t_code, t_dvec, t_dvec32, t_hidx, t_dorder, t_slotq;
  // tree workspace
  DevBuf w_partial, w_flags, w_bbox, w_keys_in, w_keys, w_vals_in, w_perm, w_sort_tmp, w_scan_tmp,
      w_lvl_flags, w_cid, w_counts, w_ckey, w_cfirst, w_ccount, w_cparent, w_child8, w_coll, w_stats;
  // particles
  DevBuf w_P, w_al, w_sqa, w_tau, w_itau, w_mu4;
  // expansions
  DevBuf w_M, w_F, w_M32;
  // fields (sorted order)
  DevBuf f_phiq, f_Eq, f_Eq2, f_Gq, f_phim, f_Eum, f_Edm, f_Gm, f_E;
  DevBuf f_phiqE, f_EqE, f_EqE2, f_GqE, w_PE, w_qEs;  // the field charges q^E and their field
  // solver
  DevBuf cg_y, cg_r, cg_p, cg_Ap, w_red, w_state, w_ep, w_dal;
  // preconditioner: z, inner residual, direction and product, near field, dipoles
  DevBuf pc_z, pc_r, pc_p, pc_Ap, pc_E, pc_mu4;
  // saved for backward
  DevBuf s_F, s_phi, s_Etot, s_phiE;
  bool saved = false;
  bool saved_qE = false;  // the saved solve had separate field charges q^E
  int64_t solves = 0;     // successful solves on this handle; the saved state is that of solve saved_id
  int64_t saved_id = 0;
  double saved_bn2 = 0.0;  // ||alpha E^q||^2 of the saved solve (scale of its dipoles)
  // adjoint of the dipole equations (pfmm_backward_mu): dL/dmu sorted, the solution's dipoles, the
  // adjoint dipoles, their fields, the dipole sets of the Thole polarisation identity
  DevBuf a_G, a_mu4, a_lam4, a_phi, a_Eu, a_Ed, a_G6, a_pl4, a_mi4, a_dalp, a_dalm;
  // the tree of the polarisable sites (dipole_tree, T^mu of Sec. III), held by an inner handle: flags
  // and prefix sum of alpha > 0, the sites' caller indices, positions, polarisabilities and zero
  // charges; for the sorted order of the site tree, each site's caller index (comp) and its index in
  // this handle's sorted order (map); the right-hand side of the site tree's solves
  pfmm_handle* sites = nullptr;
  DevBuf t_flag, t_scan, t_scan_tmp, t_idx, t_pos, t_alpha, t_q, t_comp, t_map, t_rhs;
  int n_sites = 0;
  bool sites_active = false;
  ~pfmm_handle() { delete sites; }
  // excluded pairs (rows in the caller's particle order) for systems of x_n particles; x_active:
  // they apply to the current tree, whose sorted position of each caller index is in w_inv
  DevBuf x_ptr, x_idx, w_inv;
  int x_n = -1;
  bool x_active = false;
  int saved_n = 0;
  HostPinned pinned;
  std::string err;
  TreeView tv;
  Particles pa;
  int m2l_tiles = 0, nsplit = 1;
  int n_cu = 0;  // compute units of the device (M2L workgroup rounds)
  int64_t split_stride = 0;
  int64_t n_m2l = 0, n_p2p = 0, m2l_flops = 0;
  int64_t m2l_flops_cap[MAX_P + 1] = {};  // useful M2L flops per evaluation with every order capped at c
  int n_evals = 0;
  // lists of the dual tree walk (mac_theta > 0 or adaptive_leaf_max > 0): operator rows of the offsets
  // in [-(2 Rp + 1), 2 Rp + 1]^3, enclosing radii, split partners, the frontier pairs of the walk and
  // their prefix sums, the near pairs and their rows sorted by target; on the adaptive octree the
  // split flags of the cells and the level-L cells below each cell
  bool mac = false;
  int leaf_max = 0;
  MacView mv;
  DevBuf t_mdvec, t_mdvec32, m_renc, m_split, m_bad, m_acc, m_kid, m_accs, m_kids, m_stmp, m_stmp2, m_nt, m_ns, m_sort_tmp,
      m_cnt, m_nkout, m_nvout, m_nptr, m_nearc, m_nears, m_nonleaf, m_lfirst, m_lcount, m_flops;
  DevBuf m_fr[2];
};

namespace {

// Workspace of count elements in buffer b: its own (grown) allocation, or a region of the scratch
// array during an allocation-free call.
void* raw(DevBuf& b, size_t bytes) {
  if (g_arena) {
    void* p = g_arena->take(bytes, "workspace");
    b.borrow(p, bytes);
    return p;
  }
  return b.reserve(bytes);
}

template <class T>
T* dev(DevBuf& b, int64_t count) {
  return static_cast<T*>(raw(b, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
}

template <class T>
void upload(DevBuf& b, const std::vector<T>& v) {
  T* p = dev<T>(b, (int64_t)v.size());
  if (!v.empty()) PFMM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

void sync_read(pfmm_handle* h, const void* dsrc, void* hdst, size_t bytes, hipStream_t s) {
  void* pin = h->pinned.get(bytes);
  PFMM_HIP(hipMemcpyAsync(pin, dsrc, bytes, hipMemcpyDeviceToHost, s));
  PFMM_HIP(hipStreamSynchronize(s));
  std::memcpy(hdst, pin, bytes);
}

void validate_config(const pfmm_config* c) {
  if (!c) throw Error(PFMM_ERR_INVALID_ARG, "config is NULL");
  if (c->order_p < 1 || c->order_p > MAX_P)
    throw Error(PFMM_ERR_INVALID_ARG, "order_p must be in 1.." + std::to_string(MAX_P));
  if (c->ws < 1 || c->ws > 2) throw Error(PFMM_ERR_INVALID_ARG, "ws must be 1 or 2");
  if (!(c->leaf_width >= 0.0) || !std::isfinite(c->leaf_width))
    throw Error(PFMM_ERR_INVALID_ARG, "leaf_width must be >= 0");
  if (c->precision != PFMM_FP64 && c->precision != PFMM_MIXED)
    throw Error(PFMM_ERR_INVALID_ARG, "precision must be PFMM_FP64 or PFMM_MIXED");
  if (!(c->scf_tol > 0.0)) throw Error(PFMM_ERR_INVALID_ARG, "scf_tol must be > 0");
  if (c->scf_max_iter < 1) throw Error(PFMM_ERR_INVALID_ARG, "scf_max_iter must be >= 1");
  if (c->graph_iters < 0) throw Error(PFMM_ERR_INVALID_ARG, "graph_iters must be >= 0");
  if (!(c->thole_a >= 0.0) || !std::isfinite(c->thole_a))
    throw Error(PFMM_ERR_INVALID_ARG, "thole_a must be >= 0");
  if (!std::isfinite(c->coulomb_k)) throw Error(PFMM_ERR_INVALID_ARG, "coulomb_k must be finite");
  if (c->m2l_order_slack < -1) throw Error(PFMM_ERR_INVALID_ARG, "m2l_order_slack must be >= -1");
  if (!(c->precond_cutoff >= 0.0) || !std::isfinite(c->precond_cutoff))
    throw Error(PFMM_ERR_INVALID_ARG, "precond_cutoff must be >= 0");
  if (!(c->scf_relax >= 0.0 && c->scf_relax < 1.0))
    throw Error(PFMM_ERR_INVALID_ARG, "scf_relax must be in [0, 1)");
  if (!(c->dipole_pair_dl >= 0.0 && c->dipole_pair_dl <= 1.0))
    throw Error(PFMM_ERR_INVALID_ARG, "dipole_pair_dl must be in [0, 1] Angstrom");
  if (c->precond_cutoff > 0.0 && (c->precond_iters < 1 || c->precond_iters > 64))
    throw Error(PFMM_ERR_INVALID_ARG, "precond_iters must be in 1..64");
  if (c->dipole_tree != 0 && c->dipole_tree != 1) throw Error(PFMM_ERR_INVALID_ARG, "dipole_tree must be 0 or 1");
  if (!(c->mac_theta == 0.0 || (c->mac_theta >= 0.3 && c->mac_theta < 1.0)))
    throw Error(PFMM_ERR_INVALID_ARG, "mac_theta must be 0 or in [0.3, 1)");
  if (c->mac_ndirect < 0) throw Error(PFMM_ERR_INVALID_ARG, "mac_ndirect must be >= 0");
  if (c->mac_leaf_direct != 0 && c->mac_leaf_direct != 1)
    throw Error(PFMM_ERR_INVALID_ARG, "mac_leaf_direct must be 0 or 1");
  if (c->adaptive_leaf_max < 0) throw Error(PFMM_ERR_INVALID_ARG, "adaptive_leaf_max must be >= 0");
  const bool walk = c->mac_theta > 0.0 || c->adaptive_leaf_max > 0;
  if (walk && c->order_p > MAX_P_MAC)
    throw Error(PFMM_ERR_INVALID_ARG, "mac_theta and adaptive_leaf_max support order_p up to " + std::to_string(MAX_P_MAC));
  if (c->mac_theta > 0.0 && c->m2l_order_slack >= 0)
    throw Error(PFMM_ERR_INVALID_ARG, "mac_theta runs every M2L at order p: m2l_order_slack must be -1");
}

// ------------------------------------------------------------------------------------------------
// Tree build.  Leaves h->tv / h->pa describing the sorted particles and the octree.
// ------------------------------------------------------------------------------------------------
void build_mac_lists(pfmm_handle* h, hipStream_t s);
void build_tree_stats(pfmm_handle* h, hipStream_t s);
void set_m2l_split(pfmm_handle* h);

void build_tree(pfmm_handle* h, int n, const double* pos, const double* q, const double* alpha,
                hipStream_t s) {
  const pfmm_config& c = h->cfg;
  PFMM_HIP(hipGetDevice(&h->device));
  PFMM_HIP(hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
  const int nblk = std::min(1024, std::max(1, (n + 255) / 256));
  double* partial = dev<double>(h->w_partial, (int64_t)nblk * NRED);
  int* flags = dev<int>(h->w_flags, 4);
  double* bbox = dev<double>(h->w_bbox, NRED);
  launch_fill_int(flags, 4, 0, s);
  launch_scan_inputs(pos, q, alpha, n, partial, nblk, flags, s);
  launch_bbox_final(partial, nblk, bbox, s);
  struct { double bb[NRED]; int fl[4]; } hb;
  // two small readbacks share one synchronisation
  void* pin = h->pinned.get(sizeof(hb));
  PFMM_HIP(hipMemcpyAsync(pin, bbox, NRED * sizeof(double), hipMemcpyDeviceToHost, s));
  PFMM_HIP(hipMemcpyAsync((char*)pin + offsetof(decltype(hb), fl), flags, 4 * sizeof(int),
                          hipMemcpyDeviceToHost, s));
  PFMM_HIP(hipStreamSynchronize(s));
  std::memcpy(&hb, pin, sizeof(hb));
  if (hb.fl[0] & 1) throw Error(PFMM_ERR_NONFINITE, "non-finite position, charge or polarizability");
  if (hb.fl[0] & 2) throw Error(PFMM_ERR_INVALID_ARG, "negative polarizability");

  double lo[3], hi[3], cen[3], extent = 0.0;
  for (int a = 0; a < 3; ++a) {
    lo[a] = hb.bb[a];
    hi[a] = hb.bb[3 + a];
    cen[a] = (lo[a] + hi[a]) * 0.5;
    extent = std::max(extent, hi[a] - lo[a]);
  }
  const double alpha_max = hb.bb[6];
  // leaves whose pairs are always summed directly: within ws, or below the separation that the dual
  // tree walk accepts (adjacent with the criterion, within ws with the ws rule)
  const int reach = h->mac ? h->mv.minsep - 1 : c.ws;
  const double s_max = c.thole_a * std::cbrt(alpha_max);  // a (alpha_max^2)^(1/6)
  double w = c.leaf_width;
  if (w == 0.0) {
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= std::max(hi[a] - lo[a], 1.0);
    const double occ = c.ws == 1 ? 24.0 : 12.0;
    w = std::cbrt(occ * vol / std::max(n, 1));
    w = std::max(w, 1.0001 * s_max / reach);
    w = std::max(w, 1e-3);
  }
  if (s_max > reach * w)
    throw Error(PFMM_ERR_INVALID_ARG,
                "Thole damping radius " + std::to_string(s_max) + " exceeds the near-field range " +
                    (reach == 1 ? std::string("leaf_width = ") : std::string("ws * leaf_width = ")) +
                    std::to_string(reach * w) + "; increase leaf_width" + (h->mv.use_theta && h->mac ? "" : " or ws"));
  int L = 0;
  while (w * std::ldexp(1.0, L) < extent * (1.0 + std::ldexp(1.0, -20))) {
    ++L;
    if (L > MAX_LEVELS) throw Error(PFMM_ERR_INVALID_ARG, "leaf_width too small for the extent (more than 21 levels)");
  }
  const double side = w * std::ldexp(1.0, L);
  double origin[3];
  for (int a = 0; a < 3; ++a) origin[a] = cen[a] - side * 0.5;

  // Morton keys and sort
  uint64_t* keys_in = dev<uint64_t>(h->w_keys_in, n);
  uint64_t* keys = dev<uint64_t>(h->w_keys, n);
  int* vals_in = dev<int>(h->w_vals_in, n);
  int* perm = dev<int>(h->w_perm, n);
  launch_morton(pos, n, origin, w, L, keys_in, vals_in, s);
  if (L > 0) {
    size_t tb = sort_temp_bytes(n, 3 * L);
    void* tmp = raw(h->w_sort_tmp, tb);
    launch_sort(tmp, tb, keys_in, keys, vals_in, perm, n, 3 * L, s);
  } else {
    PFMM_HIP(hipMemcpyAsync(keys, keys_in, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    PFMM_HIP(hipMemcpyAsync(perm, vals_in, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  }
  double4* P = dev<double4>(h->w_P, n);
  double* al = dev<double>(h->w_al, n);
  double* sqa = dev<double>(h->w_sqa, n);
  double* tau = dev<double>(h->w_tau, n);
  double* itau = dev<double>(h->w_itau, n);
  launch_gather(perm, pos, q, alpha, n, std::sqrt(c.thole_a), P, al, sqa, tau, itau, s);

  // level cells
  int* lflags = dev<int>(h->w_lvl_flags, n);
  int* cid = dev<int>(h->w_cid, (int64_t)n * (L + 1));
  int* counts = dev<int>(h->w_counts, L + 2);
  size_t sb = scan_temp_bytes(n);
  void* stmp = raw(h->w_scan_tmp, sb);
  for (int l = 0; l <= L; ++l)
    launch_level_scan(keys, n, 3 * (L - l), lflags, cid + (int64_t)l * n, counts + l, stmp, sb, s);
  std::vector<int> cnt(L + 1);
  sync_read(h, counts, cnt.data(), sizeof(int) * (L + 1), s);

  TreeView& t = h->tv;
  t = TreeView();
  t.L = L;
  t.off[0] = 0;
  for (int l = 0; l <= L; ++l) t.off[l + 1] = t.off[l] + cnt[l];
  t.ncell = t.off[L + 1];
  for (int a = 0; a < 3; ++a) t.origin[a] = origin[a];
  t.w = w;
  t.ws = c.ws;
  t.nnear = h->tab.nnear;
  t.damp_adjacent = s_max * (1.0 + 1e-9) <= w ? 1 : 0;
  const int ncell = t.ncell;
  uint64_t* ckey = dev<uint64_t>(h->w_ckey, ncell);
  int* cfirst = dev<int>(h->w_cfirst, ncell);
  int* ccount = dev<int>(h->w_ccount, ncell);
  int* cparent = dev<int>(h->w_cparent, ncell);
  int* child8 = dev<int>(h->w_child8, (int64_t)ncell * 8);
  int* coll = dev<int>(h->w_coll, (int64_t)ncell * t.nnear);
  launch_fill_int(child8, (int64_t)ncell * 8, -1, s);
  for (int l = 0; l <= L; ++l) {
    launch_cells(keys, n, L, l, cid + (int64_t)l * n, l > 0 ? cid + (int64_t)(l - 1) * n : nullptr,
                 t.off[l], l > 0 ? t.off[l - 1] : 0, ckey, cfirst, cparent, child8, s);
    launch_cell_counts(cfirst, t.off[l], cnt[l], n, ccount, s);
    launch_colleagues(ckey, t.off[l], cnt[l], l, c.ws, coll, s);
  }
  t.key = ckey; t.first = cfirst; t.count = ccount; t.parent = cparent; t.child8 = child8; t.coll = coll;

  Particles& pa = h->pa;
  pa.n = n; pa.P = P; pa.alpha = al; pa.sqa = sqa; pa.tau = tau; pa.itau = itau;

  if (h->mac) {
    build_mac_lists(h, s);
  } else {
    build_tree_stats(h, s);
  }
  set_m2l_split(h);
  // expansions (one extra zero row serves empty M2L sources); F holds nsplit partial copies
  const int64_t rows = (int64_t)ncell + 1;
  h->split_stride = rows * h->op.stride;
  double* M = dev<double>(h->w_M, rows * h->op.stride);
  dev<double>(h->w_F, rows * h->op.stride * h->nsplit);
  if (c.precision == PFMM_MIXED) dev<float>(h->w_M32, rows * h->op.stride);
  launch_fill_double(M + (int64_t)ncell * h->op.stride, h->op.stride, 0.0, s);
  h->n_evals = 0;
}

// Pair statistics of the well-separation lists: M2L pairs, near particle pairs, useful M2L flops
// (also with every order capped at c).
void build_tree_stats(pfmm_handle* h, hipStream_t s) {
  const TreeView& t = h->tv;
  constexpr int NST = 3 + MAX_P + 1;
  unsigned long long* stats = dev<unsigned long long>(h->w_stats, NST);
  PFMM_HIP(hipMemsetAsync(stats, 0, NST * sizeof(unsigned long long), s));
  launch_tree_stats(t, h->op.m2l_code, h->op.dorder, h->op.noff, h->op.p, stats, s);
  unsigned long long st[NST];
  {
    void* pin = h->pinned.get(sizeof(st));
    PFMM_HIP(hipMemcpyAsync(pin, stats, sizeof(st), hipMemcpyDeviceToHost, s));
    PFMM_HIP(hipStreamSynchronize(s));
    std::memcpy(st, pin, sizeof(st));
  }
  h->n_m2l = (int64_t)st[0];
  h->n_p2p = (int64_t)st[1];
  h->m2l_flops = (int64_t)st[2];
  for (int c = 0; c <= MAX_P; ++c) h->m2l_flops_cap[c] = c <= h->op.p ? (int64_t)st[3 + c] : 0;
}

void set_m2l_split(pfmm_handle* h) {
  const pfmm_config& c = h->cfg;
  const TreeView& t = h->tv;
  const int L = t.L;
  // Split each parent tile's colleague offsets over nsplit workgroups (one per CU at a time).  The
  // launch takes ceil(tiles * nsplit / CUs) rounds of workgroups, each 1/nsplit of a tile's work,
  // plus a fixed cost per round (staging the index table, the first offset's loads), and L2L reads
  // one partial copy of F~ per split: choose the nsplit that minimises
  // rounds / nsplit + 0.004 rounds + 0.006 nsplit (in units of one round of whole tiles), with at
  // least one round of workgroups and at least 4 offsets per split.
  // the acceptance-criterion M2L: float64 tiles, over the split partners instead of the colleagues
  const bool mac = h->mac;
  const int side = 2 * h->mv.Rp + 1;
  const int nn = mac ? side * side * side : t.nnear;
  const int lp_hi = L - 1 - (mac && h->mv.leaf_direct ? 1 : 0);
  h->nsplit = 1;
  if (c.order_p > MAX_P_MFMA) {  // the vector M2L: one workgroup per target cell, no splits
    h->m2l_tiles = 0;
    return;
  }
  h->m2l_tiles = L >= 2 ? m2l_tiles(t, 1, lp_hi, mac ? 1 : m2l_tile_ncb(c.order_p, c.precision == PFMM_MIXED)) : 0;
  if (h->m2l_tiles > 0) {
    const int64_t T = h->m2l_tiles, C = std::max(1, h->n_cu);
    const int hi = std::max(1, std::min(32, nn / 4));
    const int lo = (int)std::min<int64_t>(hi, std::max<int64_t>(1, (C + T - 1) / T));
    double best = 0.0;
    for (int ns = lo; ns <= hi; ++ns) {
      const int64_t rounds = (T * ns + C - 1) / C;
      const double cost = (double)rounds / ns + 0.004 * (double)rounds + 0.006 * ns;
      if (ns == lo || cost < best - 1e-12) {
        best = cost;
        h->nsplit = ns;
      }
    }
  }
}

// The dual tree walk (mac.hip) for the tree in h->tv, with the acceptance criterion or, on the
// adaptive octree, the ws rule: the split flags of the adaptive cells, the split partners of every
// cell of levels < L (h->mv.split, read by the M2L), each leaf's near row (h->tv.nptr / nidx: source
// cells of any level) and the pair statistics.  One synchronisation per level reads the sizes of the
// next frontier and of the level's near entries.
void build_mac_lists(pfmm_handle* h, hipStream_t s) {
  TreeView& t = h->tv;
  MacView& mv = h->mv;
  const int L = t.L, ncell = t.ncell;
  mv.renc = nullptr;
  if (mv.use_theta) {
    double* renc = dev<double>(h->m_renc, ncell);
    for (int l = 0; l <= L; ++l) launch_mac_radii(t, h->pa.P, l, renc, s);
    mv.renc = renc;
  }
  mv.nonleaf = mv.lfirst = mv.lcount = nullptr;
  if (h->leaf_max > 0) {
    // the adaptive octree: over-full cells split, then the 2:1 balance from the finest level up (a
    // cell's flag is final once the level below it is done)
    int* nonleaf = dev<int>(h->m_nonleaf, ncell);
    int* lfirst = dev<int>(h->m_lfirst, ncell);
    int* lcount = dev<int>(h->m_lcount, ncell);
    for (int l = 0; l <= L; ++l) {
      launch_adapt_init(t, l, h->leaf_max, nonleaf, s);
      launch_leaf_range(t, l, lfirst, lcount, s);
    }
    for (int l = L - 1; l >= 0; --l) launch_adapt_balance(t, l, nonleaf, s);
    mv.nonleaf = nonleaf;
    mv.lfirst = lfirst;
    mv.lcount = lcount;
  }
  const int side = 2 * mv.Rp + 1, nn = side * side * side;
  int* split = dev<int>(h->m_split, (int64_t)std::max(t.off[L], 1) * nn);
  launch_fill_int(split, (int64_t)std::max(t.off[L], 1) * nn, -1, s);
  mv.split = split;
  int* bad = dev<int>(h->m_bad, 1);
  launch_fill_int(bad, 1, 0, s);
  // the accepted pairs' useful flops (at their orders, and capped at each c <= p)
  unsigned long long* fst = dev<unsigned long long>(h->m_flops, MAX_P + 2);
  launch_fill_int(reinterpret_cast<int*>(fst), 2 * (MAX_P + 2), 0, s);
  int cur = 0;
  int2* fr = dev<int2>(h->m_fr[cur], 1);
  launch_fill_int(reinterpret_cast<int*>(fr), 2, 0, s);  // (root, root)
  int64_t nfr = 1, nm = 0, nnear = 0;
  // near entries of all levels, appended level by level: the buffers start at a guess and grow
  // keeping their contents (from the scratch array during an allocation-free call)
  {
    const int64_t guess = std::max<int64_t>(1024, 32LL * (t.off[L + 1] - t.off[L]));
    dev<int>(h->m_nt, guess);
    dev<int>(h->m_ns, guess);
  }
  auto near_room = [&](int64_t want) {
    const size_t b = (size_t)want * sizeof(int);
    if (b <= h->m_nt.bytes && b <= h->m_ns.bytes) return;
    DevBuf nt2, ns2;
    int* a = dev<int>(nt2, 2 * want);
    int* c = dev<int>(ns2, 2 * want);
    if (nnear > 0) {
      PFMM_HIP(hipMemcpyAsync(a, h->m_nt.ptr, (size_t)nnear * sizeof(int), hipMemcpyDeviceToDevice, s));
      PFMM_HIP(hipMemcpyAsync(c, h->m_ns.ptr, (size_t)nnear * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    PFMM_HIP(hipStreamSynchronize(s));  // the old buffers may be released below
    if (g_arena) {
      h->m_nt.borrow(a, nt2.bytes);
      h->m_ns.borrow(c, ns2.bytes);
      return;
    }
    for (auto [dst, src] : {std::pair<DevBuf*, DevBuf*>{&h->m_nt, &nt2}, {&h->m_ns, &ns2}}) {
      std::swap(dst->own, src->own);
      std::swap(dst->own_bytes, src->own_bytes);
      dst->ptr = dst->own;
      dst->bytes = dst->own_bytes;
      src->ptr = src->own;
      src->bytes = src->own_bytes;
    }
  };
  for (int l = 0; l <= L; ++l) {
    // the child pairs of a split pair are at most 64; the prefix sums are 32-bit
    if (l < L && nfr * 64 > INT_MAX)
      throw Error(PFMM_ERR_INVALID_ARG, "dual-walk lists too large (" + std::to_string(nfr) +
                                            " cell pairs at level " + std::to_string(l) +
                                            "); raise leaf_width, mac_theta or adaptive_leaf_max");
    const int nf = (int)nfr;
    int* acc = dev<int>(h->m_acc, nf);
    int* kid = dev<int>(h->m_kid, nf);
    int* nearc = dev<int>(h->m_nearc, nf);
    int* accs = dev<int>(h->m_accs, nf);
    int* kids = dev<int>(h->m_kids, nf);
    int* nears = dev<int>(h->m_nears, nf);
    launch_mac_classify(t, mv, l, fr, nf, acc, kid, nearc, s);
    launch_mac_flops(t, mv, fr, nf, acc, h->op.dorder, h->op.p, fst, s);
    const size_t tb = scan_temp_bytes(nf);
    void* tmp = raw(h->m_stmp, tb);
    launch_inclusive_scan(tmp, tb, acc, accs, nf, s);
    launch_inclusive_scan(tmp, tb, kid, kids, nf, s);
    launch_inclusive_scan(tmp, tb, nearc, nears, nf, s);
    int tot[3];
    void* pin = h->pinned.get(sizeof(tot));
    PFMM_HIP(hipMemcpyAsync(pin, accs + (nf - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    PFMM_HIP(hipMemcpyAsync((char*)pin + sizeof(int), kids + (nf - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    PFMM_HIP(hipMemcpyAsync((char*)pin + 2 * sizeof(int), nears + (nf - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    PFMM_HIP(hipStreamSynchronize(s));
    std::memcpy(tot, pin, sizeof(tot));
    nm += tot[0];
    if (l == L && tot[1] != 0) throw Error(PFMM_ERR_HIP, "internal: the walk split a pair of leaves");
    if (nnear + tot[2] > INT_MAX) throw Error(PFMM_ERR_INVALID_ARG, "dual-walk near list too large");
    near_room(std::max<int64_t>(nnear + tot[2], 1));
    int2* next = l < L ? dev<int2>(h->m_fr[cur ^ 1], tot[1]) : nullptr;
    launch_mac_emit(t, mv, l, fr, nf, kids, nears, next, split, h->m_nt.as<int>() + nnear,
                    h->m_ns.as<int>() + nnear, bad, s);
    nnear += tot[2];
    if (l < L) {
      fr = next;
      nfr = tot[1];
      cur ^= 1;
      if (nfr == 0) break;
    }
  }
  int* near_t = h->m_nt.as<int>();
  int* near_s = h->m_ns.as<int>();
  const int nnear_i = (int)nnear;
  int badh = 0;
  sync_read(h, bad, &badh, sizeof(int), s);
  if (badh) throw Error(PFMM_ERR_INVALID_ARG, "internal: a split cell pair lies beyond the partner table");

  // near rows of the leaves, sorted by target (stable)
  int bits = 1;
  while ((1LL << bits) <= (int64_t)ncell) ++bits;
  const int nleaf = t.off[L + 1] - t.off[L];
  int* nkey = dev<int>(h->m_nkout, nnear_i);
  int* nsrc = dev<int>(h->m_nvout, nnear_i);
  const size_t sortb = mac_sort_temp_bytes(nnear_i, bits);
  launch_mac_sort(raw(h->m_sort_tmp, sortb), sortb, near_t, nkey, near_s, nsrc, nnear_i, bits, s);
  int* nptr = dev<int>(h->m_nptr, (int64_t)nleaf + 1);
  launch_fill_int(nptr, (int64_t)nleaf + 1, 0, s);
  int* cnt = dev<int>(h->m_cnt, nleaf);
  launch_fill_int(cnt, nleaf, 0, s);
  launch_mac_count(nkey, nnear_i, t.off[L], cnt, s);
  const size_t scanb = scan_temp_bytes(nleaf);
  launch_inclusive_scan(raw(h->m_stmp2, scanb), scanb, cnt, nptr + 1, nleaf, s);
  t.nptr = nptr;
  t.nidx = nsrc;

  unsigned long long* pairs = dev<unsigned long long>(h->w_stats, 1);
  launch_fill_int(reinterpret_cast<int*>(pairs), 2, 0, s);
  launch_mac_near_pairs(t, nkey, nsrc, nnear_i, pairs, s);
  unsigned long long np = 0, fl[MAX_P + 2];
  sync_read(h, pairs, &np, sizeof(np), s);
  sync_read(h, fst, fl, sizeof(fl), s);
  h->n_m2l = nm;
  h->n_p2p = (int64_t)np;
  h->m2l_flops = (int64_t)fl[0];
  for (int c = 0; c <= MAX_P; ++c) h->m2l_flops_cap[c] = c <= h->op.p ? (int64_t)fl[1 + c] : 0;
}

// One FMM evaluation: sources 1 = charges, 2 = dipoles (mu4), 3 = both.
// mode 0: Ed only; mode 1: phi, Eu, Ed, G.
// pa_src replaces the handle's particles as sources and targets (same positions and order; the
// field charges q^E in place of q).
void fmm_pass(pfmm_handle* h, int sources, int mode, FieldOut out, int* err, const int* done,
              hipStream_t s, const int* qcap = nullptr, const Particles* pa_src = nullptr) {
  const Particles& pa = pa_src ? *pa_src : h->pa;
  const TreeView& t = h->tv;
  const OpTables& op = h->op;
  const bool fp32 = h->cfg.precision == PFMM_MIXED;
  const int n = h->pa.n;
  double* M = h->w_M.as<double>();
  double* F = h->w_F.as<double>();
  const double4* mu4 = h->w_mu4.as<double4>();
  KernelTimer& kt = h->kt;
  if (t.L >= 2) {
    int e = kt.begin();
    launch_p2m(t, op, pa, mu4, sources, h->cfg.dipole_pair_dl, M, done, s);
    kt.end(KC_P2M, e);
    e = kt.begin();
    for (int lp = t.L - 1; lp >= 2; --lp) launch_m2m(t, op, lp, M, done, s);
    kt.end(KC_M2M, e);
    e = kt.begin();
    if (h->mac) {
      // with leaf pairs direct no M2L runs for the leaves: their F~ (and its partial sums of the
      // offset splits, which the L2L adds) start from zero
      if (h->mv.leaf_direct)
        for (int sp = 0; sp < h->nsplit; ++sp)
          launch_fill_double(F + sp * h->split_stride + (int64_t)t.off[t.L] * op.stride,
                             (int64_t)(t.ncell - t.off[t.L]) * op.stride, 0.0, s);
    }
    float* M32 = nullptr;
    if (fp32 && op.p <= MAX_P_MFMA) {
      M32 = h->w_M32.as<float>();
      launch_to_float(M, M32, ((int64_t)t.ncell + 1) * op.stride, done, s);
    }
    launch_m2l(t, op, h->nsplit, M, M32, F, h->split_stride, fp32 && op.p <= MAX_P_MFMA, 3, done, qcap, s,
               h->mac ? &h->mv : nullptr);
    kt.end(KC_M2L, e);
    e = kt.begin();
    for (int lc = 2; lc <= t.L; ++lc) launch_l2l(t, op, lc, F, h->nsplit, h->split_stride, done, s);
    kt.end(KC_L2L, e);
    e = kt.begin();
    launch_l2p(t, op, pa, F, mode, out, done, s);
    kt.end(KC_L2P, e);
  } else {
    launch_fill_double(out.Ed, 3 * (int64_t)n, 0.0, s);
    if (mode == 1) {
      launch_fill_double(out.phi, n, 0.0, s);
      launch_fill_double(out.Eu, 3 * (int64_t)n, 0.0, s);
      launch_fill_double(out.G, 6 * (int64_t)n, 0.0, s);
    }
  }
  int e = kt.begin();
  launch_p2p(t, pa, mu4, mode == 0 ? 0 : 1, sources, fp32, out, nullptr, err, done, s);
  if (h->x_active)
    launch_exclusions(pa, h->w_perm.as<int>(), h->w_inv.as<int>(), h->x_ptr.as<int>(), h->x_idx.as<int>(), mu4,
                      mode == 0 ? 0 : 1, sources, out, nullptr, done, s);
  kt.end(mode == 0 ? KC_P2P_SCF : KC_P2P_FULL, e);
  h->n_evals += 1;
}

// The handle's exclusions apply to systems of the size they were given for (after build_tree).
void activate_exclusions(pfmm_handle* h, int n, hipStream_t s) {
  h->x_active = false;
  if (h->x_n < 0) return;
  if (h->x_n != n)
    throw Error(PFMM_ERR_INVALID_ARG, "exclusions were set for " + std::to_string(h->x_n) + " particles, not " +
                                          std::to_string(n));
  launch_inverse_perm(h->w_perm.as<int>(), n, dev<int>(h->w_inv, n), s);
  h->x_active = true;
}

struct Timer {
  bool on;
  hipStream_t s;
  hipEvent_t ev[8];
  int k = 0;
  Timer(bool on_, hipStream_t s_) : on(on_), s(s_) {
    if (on)
      for (auto& e : ev) PFMM_HIP(hipEventCreate(&e));
  }
  ~Timer() {
    if (on)
      for (auto& e : ev) (void)hipEventDestroy(e);
  }
  void mark() {
    if (on && k < 8) PFMM_HIP(hipEventRecord(ev[k++], s));
  }
  void fill(double* out) {
    if (!on) return;
    PFMM_HIP(hipEventSynchronize(ev[k - 1]));
    for (int i = 0; i + 1 < k && i < 5; ++i) {
      float ms = 0;
      PFMM_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      out[i] = ms;
    }
    float tot = 0;
    PFMM_HIP(hipEventElapsedTime(&tot, ev[0], ev[k - 1]));
    out[5] = tot;
  }
};

pfmm_status fail(pfmm_handle* h, const Error& e) {
  if (h) h->err = e.what();
  return e.status;
}

void check_flag(pfmm_handle* h, int* dflag, hipStream_t s) {
  int f = 0;
  sync_read(h, dflag, &f, sizeof(int), s);
  if (f) throw Error(PFMM_ERR_COINCIDENT, "two particles share the same position");
}

// The tree of the dipole solve.  With dipole_tree, when the polarisable sites (alpha > 0) are a
// proper non-empty subset, they get a tree of their own (T^mu of Sec. III), held by the inner handle
// h->sites: the solve's field evaluations then involve the sites only, while the charge field and the
// final pass stay on the tree of all particles.  Returns the handle whose tree the solve runs on
// (h itself otherwise).  pos and alpha are the caller's arrays; call after build_tree(h, ...).
pfmm_handle* site_tree(pfmm_handle* h, int n, const double* pos, const double* alpha, hipStream_t s) {
  h->sites_active = false;
  if (!h->cfg.dipole_tree) return h;
  if (h->x_active) throw Error(PFMM_ERR_INVALID_ARG, "dipole_tree does not apply excluded pairs");
  int* flags = dev<int>(h->t_flag, n);
  int* scan = dev<int>(h->t_scan, n);
  launch_flag_polarisable(alpha, n, flags, s);
  const size_t tb = scan_temp_bytes(n);
  launch_inclusive_scan(raw(h->t_scan_tmp, tb), tb, flags, scan, n, s);
  int m = 0;
  sync_read(h, scan + (n - 1), &m, sizeof(int), s);
  if (m == 0 || m == n) return h;
  if (!h->sites) {
    pfmm_config ci = h->cfg;
    ci.dipole_tree = 0;
    pfmm_handle* hi = nullptr;
    const pfmm_status st = pfmm_create(&ci, &hi);
    if (st != PFMM_OK) throw Error(st, "creating the handle of the polarisable sites' tree failed");
    h->sites = hi;
  }
  pfmm_handle* hm = h->sites;
  int* idx = dev<int>(h->t_idx, m);
  double* spos = dev<double>(h->t_pos, 3 * (int64_t)m);
  double* sal = dev<double>(h->t_alpha, m);
  double* sq = dev<double>(h->t_q, m);
  launch_compact_sites(scan, pos, alpha, n, idx, spos, sal, sq, s);
  hm->kt.reset((h->cfg.flags & PFMM_TIMING) != 0, s);
  hm->kt.tag = h->cfg.order_p;
  build_tree(hm, m, spos, sq, sal, s);
  hm->x_active = false;
  int* inv = dev<int>(h->w_inv, n);
  launch_inverse_perm(h->w_perm.as<int>(), n, inv, s);
  launch_site_maps(hm->w_perm.as<int>(), idx, inv, m, dev<int>(h->t_comp, m), dev<int>(h->t_map, m), s);
  h->n_sites = m;
  h->sites_active = true;
  return hm;
}

// Stage 2 of Sec. III on the current tree: conjugate gradients on (I - S T~ S) y = S Ee for the
// right-hand-side field Ee (sorted order, 3n; the static field E^q for the dipoles, or any other
// vector for the adjoint solve), preconditioned by the near field when configured, with relaxed
// field evaluations from rp.start (0: none).  warm_now: start from the dipoles in h->w_mu4.  On
// return h->cg_y holds y (mu = S y) and the host copy of the state is returned; *evals counts the
// full-order field evaluations made outside the iterations.  st: two CGState (outer, inner).
CGState dipole_cg(pfmm_handle* h, const double* Ee, bool warm_now, const RelaxParams& rp, CGState* st, int* err,
                  hipStream_t s, int* evals) {
  const pfmm_config& c = h->cfg;
  const Particles& pa = h->pa;
  const int n = pa.n;
  double4* mu4 = h->w_mu4.as<double4>();
  double* y = dev<double>(h->cg_y, 3 * (int64_t)n);
  double* r = dev<double>(h->cg_r, 3 * (int64_t)n);
  double* pv = dev<double>(h->cg_p, 3 * (int64_t)n);
  double* Ap = dev<double>(h->cg_Ap, 3 * (int64_t)n);
  double* E = dev<double>(h->f_E, 3 * (int64_t)n);
  double* part = dev<double>(h->w_red, RED_BLOCKS * 8);
  CGState* inner = st + 1;
  const bool pc = c.precond_cutoff > 0.0;
  double* z = pc ? dev<double>(h->pc_z, 3 * (int64_t)n) : nullptr;
  double* ri = pc ? dev<double>(h->pc_r, 3 * (int64_t)n) : nullptr;
  double* pi = pc ? dev<double>(h->pc_p, 3 * (int64_t)n) : nullptr;
  double* Api = pc ? dev<double>(h->pc_Ap, 3 * (int64_t)n) : nullptr;
  double* Epc = pc ? dev<double>(h->pc_E, 3 * (int64_t)n) : nullptr;
  double4* mu4pc = pc ? dev<double4>(h->pc_mu4, n) : nullptr;
  // z = inner CG approximation of (I - S T~_near S)^-1 r (the near field in float32)
  auto precondition = [&](hipStream_t q) {
    int ev = h->kt.begin();
    launch_pc_init(3 * n, r, z, ri, pi, part, inner, st, q);
    for (int k = 0; k < c.precond_iters; ++k) {
      launch_make_dipoles(pa, pi, mu4pc, &inner->done, q);
      launch_p2p(h->tv, pa, mu4pc, 3, 2, true, FieldOut{nullptr, nullptr, Epc, nullptr}, nullptr, err,
                 &inner->done, q, c.precond_cutoff);
      launch_cg_ap(pa, pi, Epc, Api, part, inner, q);
      launch_cg_update(pa, z, ri, pi, Api, part, inner, -1.0, c.precond_iters, q);
      launch_cg_direction(3 * n, ri, pi, inner, q);
    }
    h->kt.end(KC_SOLVER, ev);
  };
  FieldOut fo{nullptr, nullptr, E, nullptr};
  const int* done = &st->done;
  const bool timing = (c.flags & PFMM_TIMING) != 0;
  // with timing, test convergence after every iteration so that no launch runs past it
  const int chunk = timing ? 1 : (c.graph_iters > 0 ? c.graph_iters : 4);
  const bool use_graph = c.graph_iters > 0 && !timing;
  const bool relaxed = rp.start > 0.0;
  const int* qcap = relaxed ? &st->qcap : nullptr;
  const double tol = c.scf_tol * (relaxed ? rp.tol_scale : 1.0);
  if (pc && !warm_now) {
    // the preconditioned solve starts from y0 = 0: r0 = S Ee costs no field evaluation, and
    // p0 = z0 is a better first direction than the Jacobi guess alpha Ee
    launch_cg_init_zero(pa, Ee, y, r, part, st, tol, s);
  } else {
    launch_cg_init(pa, Ee, mu4, warm_now, y, pv, mu4, part, st, s);
    fmm_pass(h, 2, 0, fo, err, nullptr, s);
    ++*evals;
    launch_cg_residual0(pa, Ee, E, y, r, pv, part, st, tol, s);
  }
  if (pc) {
    precondition(s);
    launch_cg_direction(3 * n, z, pv, st, s);  // b = 0 here: p0 = z0
  }
  CGState hs{};
  auto iteration = [&](hipStream_t q) {
    int ev = h->kt.begin();
    launch_make_dipoles(pa, pv, mu4, done, q);
    h->kt.end(KC_SOLVER, ev);
    // with timing the state is read back after every iteration, so the cap is known here
    h->kt.tag = qcap ? hs.qcap : c.order_p;
    fmm_pass(h, 2, 0, fo, err, done, q, qcap);
    h->kt.tag = c.order_p;
    if (pc) {
      ev = h->kt.begin();
      launch_pcg_ap(pa, pv, E, r, Ap, part, st, q);
      launch_cg_update(pa, y, r, pv, Ap, part, st, tol, c.scf_max_iter, q, rp);
      h->kt.end(KC_SOLVER, ev);
      precondition(q);
      ev = h->kt.begin();
      launch_pcg_zq(3 * n, z, Ap, part, st, q);
      launch_cg_direction(3 * n, z, pv, st, q);
      h->kt.end(KC_SOLVER, ev);
      return;
    }
    ev = h->kt.begin();
    launch_cg_ap(pa, pv, E, Ap, part, st, q);
    launch_cg_update(pa, y, r, pv, Ap, part, st, tol, c.scf_max_iter, q, rp);
    launch_cg_direction(3 * n, r, pv, st, q);
    h->kt.end(KC_SOLVER, ev);
  };
  sync_read(h, st, &hs, sizeof(hs), s);
  int launched = 0;
  if (use_graph && !hs.done) {
    // chunk iterations captured as one HIP graph; every kernel in it returns at once when the
    // device-side `done` flag is set, so replays past convergence are no-ops
    h->graph.capture([&]() {
      for (int k = 0; k < chunk; ++k) iteration(h->graph.cap);
    });
    while (!hs.done && launched < c.scf_max_iter) {
      h->graph.launch(s);
      launched += chunk;
      sync_read(h, st, &hs, sizeof(hs), s);
    }
  } else {
    while (!hs.done && launched < c.scf_max_iter) {
      for (int k = 0; k < chunk && launched < c.scf_max_iter; ++k, ++launched) iteration(s);
      sync_read(h, st, &hs, sizeof(hs), s);
    }
  }
  return hs;
}

pfmm_status solve_impl(pfmm_handle* h, int64_t n64, const double* pos, const double* q, const double* qE,
                       const double* alpha, double* mu, double* forces, double* phi, double* phi_E,
                       pfmm_result* res, hipStream_t s) {
  const pfmm_config& c = h->cfg;
  if (n64 < 0 || n64 > INT_MAX / 8) throw Error(PFMM_ERR_INVALID_ARG, "n out of range");
  if (!res) throw Error(PFMM_ERR_INVALID_ARG, "res is NULL");
  std::memset(res, 0, sizeof(*res));
  h->saved = false;
  const int n = (int)n64;
  const bool want_f = (c.flags & PFMM_WANT_FORCES) != 0;
  const bool want_phi = (c.flags & PFMM_WANT_POTENTIALS) != 0;
  if (n > 0 && (!pos || !q || !alpha || !mu)) throw Error(PFMM_ERR_INVALID_ARG, "NULL input or mu");
  if (phi_E && !qE) throw Error(PFMM_ERR_INVALID_ARG, "phi_E needs the field charges qE");
  if (n > 0 && want_f && !forces) throw Error(PFMM_ERR_INVALID_ARG, "forces is NULL with PFMM_WANT_FORCES");
  if (n > 0 && want_phi && !phi) throw Error(PFMM_ERR_INVALID_ARG, "phi is NULL with PFMM_WANT_POTENTIALS");
  if (n == 0) {
    h->saved = true;
    h->saved_n = 0;
    h->saved_qE = qE != nullptr;
    h->saved_id = ++h->solves;
    res->solve_id = h->saved_id;
    return PFMM_OK;
  }
  PFMM_HIP(hipGetDevice(&h->device));

  Timer tm((c.flags & PFMM_TIMING) != 0, s);
  h->kt.reset((c.flags & PFMM_TIMING) != 0, s);
  h->kt.tag = c.order_p;
  tm.mark();
  if ((c.flags & PFMM_WARM_START) != 0) {
    int* fl = dev<int>(h->w_flags, 4);
    launch_fill_int(fl, 1, 0, s);
    launch_check_finite(mu, 3 * n64, fl, s);
    int f = 0;
    sync_read(h, fl, &f, sizeof(int), s);
    if (f) throw Error(PFMM_ERR_NONFINITE, "non-finite warm-start dipole");
  }
  if (qE) {
    int* fl = dev<int>(h->w_flags, 4);
    launch_fill_int(fl, 1, 0, s);
    launch_check_finite(qE, n64, fl, s);
    int f = 0;
    sync_read(h, fl, &f, sizeof(int), s);
    if (f) throw Error(PFMM_ERR_NONFINITE, "non-finite field charge qE");
  }
  build_tree(h, n, pos, q, alpha, s);
  activate_exclusions(h, n, s);
  tm.mark();
  const Particles& pa = h->pa;
  double4* mu4 = dev<double4>(h->w_mu4, n);
  int* err = dev<int>(h->w_flags, 4);
  launch_fill_int(err, 4, 0, s);

  // stage 1: field of the charges
  double* phiq = dev<double>(h->f_phiq, n);
  double* Eq = dev<double>(h->f_Eq, 3 * (int64_t)n);
  double* Eq2 = dev<double>(h->f_Eq2, 3 * (int64_t)n);
  double* Gq = dev<double>(h->f_Gq, 6 * (int64_t)n);
  fmm_pass(h, 1, 1, FieldOut{phiq, Eq, Eq2, Gq}, err, nullptr, s);
  check_flag(h, err, s);
  // the static field that polarises the dipoles: that of the field charges q^E when they are given
  // (a second charge pass over the same tree), else that of q
  FieldCharges fc{nullptr, Eq, Gq};
  if (qE) {
    double4* PE = dev<double4>(h->w_PE, n);
    double* qEs = dev<double>(h->w_qEs, n);
    launch_field_charges(h->w_perm.as<int>(), n, pa.P, qE, PE, qEs, s);
    Particles pe = pa;
    pe.P = PE;
    double* EqE = dev<double>(h->f_EqE, 3 * (int64_t)n);
    double* GqE = dev<double>(h->f_GqE, 6 * (int64_t)n);
    fmm_pass(h, 1, 1, FieldOut{dev<double>(h->f_phiqE, n), EqE, dev<double>(h->f_EqE2, 3 * (int64_t)n), GqE},
             err, nullptr, s, nullptr, &pe);
    check_flag(h, err, s);
    fc = FieldCharges{qEs, EqE, GqE};
  }
  const double* Ee = fc.E;
  tm.mark();

  // stage 2: conjugate gradients, on the tree of all particles or on that of the polarisable sites
  pfmm_handle* hm = site_tree(h, n, pos, alpha, s);
  const bool on_sites = hm != h;
  const int m = on_sites ? h->n_sites : n;
  CGState* st = static_cast<CGState*>(hm->w_state.reserve(2 * sizeof(CGState)));
  const double* Ecg = Ee;  // the right-hand side in the order of the solve's tree
  double4* mu4cg = mu4;
  int* errcg = err;
  if (on_sites) {
    double* rhs = dev<double>(h->t_rhs, 3 * (int64_t)m);
    launch_permute_vec3(h->t_map.as<int>(), m, Ee, rhs, s);
    Ecg = rhs;
    mu4cg = dev<double4>(hm->w_mu4, m);
    errcg = dev<int>(hm->w_flags, 4);
    launch_fill_int(errcg, 4, 0, s);
  }
  const bool warm = (c.flags & PFMM_WARM_START) != 0;
  if (warm)
    launch_permute_dipoles(on_sites ? h->t_comp.as<int>() : h->w_perm.as<int>(), m, mu, hm->pa.tau, mu4cg, s);
  // relaxed field evaluations: the update kernel of each iteration picks the order cap of the next
  RelaxParams rp;
  rp.p = c.order_p;
  rp.qmin = (c.order_p + 1) / 2;
  rp.track = 1;
  rp.start = c.scf_relax;
  rp.lrho = 2.0 * std::log((c.ws + 1.0) / std::sqrt(3.0));
  // the float32 products of the mixed path add their rounding to every relaxed product: the relaxed
  // phase stops at half the tolerance, leaving room for it in the final check at the full orders
  rp.tol_scale = c.precision == PFMM_MIXED ? 0.5 : 1.0;
  launch_fill_int(&st->qcap, 1, c.order_p, s);
  launch_fill_int(st->ncap, 16, 0, s);
  double* phim = dev<double>(h->f_phim, n);
  double* Eum = dev<double>(h->f_Eum, 3 * (int64_t)n);
  double* Edm = dev<double>(h->f_Edm, 3 * (int64_t)n);
  double* Gm = dev<double>(h->f_Gm, 6 * (int64_t)n);
  double* Fs = dev<double>(h->s_F, 3 * (int64_t)n);
  double* phs = dev<double>(h->s_phi, n);
  double* phEs = dev<double>(h->s_phiE, n);
  double* Ets = dev<double>(h->s_Etot, 3 * (int64_t)n);
  EnergyParts* ep = static_cast<EnergyParts*>(h->w_ep.reserve(sizeof(EnergyParts)));
  CGState hs{};
  EnergyParts he{};
  int total_iters = 0, restarts = 0, full_evals = qE ? 2 : 1, cg_evals = 0;  // the charge passes
  bool warm_now = warm;
  double* part = dev<double>(h->w_red, RED_BLOCKS * 8);
  const bool pair = c.dipole_pair_dl > 0.0;
  for (;;) {
    const bool relaxed = rp.start > 0.0;
    hs = dipole_cg(hm, Ecg, warm_now, rp, st, errcg, s, &cg_evals);
    total_iters += hs.iters;
    if (on_sites && (relaxed || pair) && !hs.notspd && !hs.maxed) {
      // On the site tree the stopping rule is checked with that tree's own field at the full orders
      // (the full tree's field differs from it by the two trees' FMM errors): a warm-started solve
      // without the cap from the final dipoles, which stops at once when the rule already holds
      // (twice at most for charge-pair multipoles, whose field is not additive in the dipoles).
      RelaxParams r0 = rp;
      r0.start = 0.0;
      for (int k = 0; k < (pair ? 2 : 1); ++k) {
        launch_make_dipoles(hm->pa, hm->cg_y.as<double>(), mu4cg, nullptr, s);
        launch_fill_int(&st->qcap, 1, c.order_p, s);
        const CGState h2 = dipole_cg(hm, Ecg, true, r0, st, errcg, s, &cg_evals);
        total_iters += h2.iters;
        hs = h2;
        if (h2.iters == 0 || h2.notspd || h2.maxed) break;
        ++restarts;
      }
    }
    const double* y = hm->cg_y.as<double>();
    tm.mark();

    // stage 3: field of the converged dipoles (full orders), energy and forces, on all particles
    if (on_sites) {
      launch_make_dipoles(hm->pa, y, mu4cg, nullptr, s);
      launch_place_site_dipoles(h->t_map.as<int>(), m, mu4cg, n, pa.tau, mu4, s);
    } else {
      launch_make_dipoles(pa, y, mu4, nullptr, s);
    }
    fmm_pass(h, 2, 1, FieldOut{phim, Eum, Edm, Gm}, err, nullptr, s);
    ++full_evals;
    tm.mark();
    launch_assemble(pa, h->w_perm.as<int>(), mu4, phiq, Eq, fc, phim, Eum, Edm, Gm, c.coulomb_k, mu,
                    want_f ? forces : nullptr, want_phi ? phi : nullptr, phi_E, Fs, phs, phEs, Ets, part, ep,
                    s);
    tm.mark();
    sync_read(h, ep, &he, sizeof(he), s);
    const double true_res = he.bn2 > 0.0 ? std::sqrt(he.res2 / he.bn2) : 0.0;
    // a relaxed solve must meet the stopping rule with the full orders too; otherwise continue from
    // the final dipoles (in mu4) without the cap.  With charge-pair multipoles the field is not
    // additive in the dipoles (the pair departs from the point dipole by O((dl/w)^2), differently for
    // a sum than for its terms), so the recursive residual of the conjugate gradients can converge
    // while the true one has not: continue the same way, each time on a correction that is smaller
    // by the residual's factor, so that the non-additive part shrinks with it.
    if (!on_sites && (relaxed || pair) && !hs.notspd && !hs.maxed && true_res > c.scf_tol &&
        restarts < (pair ? 2 : 1)) {
      ++restarts;
      rp.start = 0.0;
      launch_fill_int(&st->qcap, 1, c.order_p, s);
      warm_now = true;
      continue;
    }
    // after the continuations allowed, a relaxed or charge-pair solve whose final dipoles still miss
    // the stopping rule at the full orders has not converged
    if (!on_sites && (relaxed || pair || restarts > 0) && true_res > c.scf_tol) {
      hs.maxed = 1;
      hs.res = true_res;
    }
    break;
  }
  tm.fill(res->t_phase_ms);
  h->kt.collect(res->t_kernel_ms, res->kernel_launches);
  h->kt.collect_m2l(KC_M2L, c.order_p, h->m2l_flops, h->m2l_flops_cap, res->t_m2l_split_ms, res->m2l_split_launches,
                    res->m2l_split_flops);
  if (on_sites) {
    hm->kt.collect(res->t_kernel_ms, res->kernel_launches);
    hm->kt.collect_m2l(KC_M2L, c.order_p, hm->m2l_flops, hm->m2l_flops_cap, res->t_m2l_split_ms,
                       res->m2l_split_launches, res->m2l_split_flops);
  }
  res->n_sites = m;

  const double ke = c.coulomb_k;
  res->U_qq = ke * he.Uqq;
  res->U_pol = ke * (he.Amu - he.muEq - 0.5 * he.muEd);
  res->U_total = res->U_qq + res->U_pol;
  res->iters = total_iters;
  res->residual = he.bn2 > 0.0 ? std::sqrt(he.res2 / he.bn2) : 0.0;
  res->residual_max_debye = he.resmax * EANG_TO_DEBYE;
  res->levels = h->tv.L;
  res->leaf_width = h->tv.w;
  res->n_leaves = h->tv.off[h->tv.L + 1] - h->tv.off[h->tv.L];
  res->n_cells = h->tv.ncell;
  res->n_m2l = h->n_m2l;
  res->n_p2p = h->n_p2p;
  res->m2l_flops = h->m2l_flops;
  // charge field, initial residuals (not on the cold-started preconditioned path), final passes: full
  // orders; the iterations at the caps they used
  int ncap[16];
  {
    CGState hc{};
    sync_read(h, st, &hc, sizeof(hc), s);
    std::memcpy(ncap, hc.ncap, sizeof(ncap));
  }
  int64_t flops_total = (int64_t)full_evals * h->m2l_flops + (int64_t)cg_evals * hm->m2l_flops;
  int cap_min = c.order_p;
  for (int q = 0; q <= c.order_p; ++q) {
    flops_total += (int64_t)ncap[q] * (q == c.order_p ? hm->m2l_flops : hm->m2l_flops_cap[q]);
    if (ncap[q] > 0) cap_min = std::min(cap_min, q);
  }
  res->n_evals = full_evals + cg_evals + total_iters;
  res->m2l_flops_total = flops_total;
  res->m2l_order_cap_min = cap_min;
  res->scf_restarts = restarts;
  if (hs.notspd) throw Error(PFMM_ERR_NOT_SPD, "conjugate gradients met p.Ap <= 0: the dipole system is not positive definite");
  if (!hs.done || (hs.maxed && hs.res > c.scf_tol))
    throw Error(PFMM_ERR_NOT_CONVERGED, "dipole solve did not converge: residual " + std::to_string(hs.res) +
                                            " after " + std::to_string(total_iters) + " iterations");
  // only a converged solve leaves state for the backward
  h->saved = true;
  h->saved_n = n;
  h->saved_qE = qE != nullptr;
  h->saved_id = ++h->solves;
  h->saved_bn2 = hs.bnorm2;
  res->solve_id = h->saved_id;
  return PFMM_OK;
}

}  // namespace

extern "C" {

void pfmm_config_default(pfmm_config* c) {
  if (!c) return;
  c->order_p = 6;
  c->ws = 2;
  c->leaf_width = 0.0;
  c->precision = PFMM_FP64;
  c->scf_tol = 1e-6;
  c->scf_max_iter = 200;
  c->graph_iters = 4;
  c->thole_a = 2.0;
  c->coulomb_k = 332.06371;
  c->flags = PFMM_WANT_FORCES | PFMM_WANT_POTENTIALS | PFMM_SAVE_FOR_BACKWARD;
  c->m2l_order_slack = -1;
  c->precond_cutoff = 0.0;
  c->precond_iters = 4;
  c->scf_relax = 0.0;
  c->dipole_pair_dl = 0.0;
  c->dipole_tree = 0;
  c->mac_theta = 0.0;
  c->mac_ndirect = 64;
  c->mac_leaf_direct = 1;
  c->adaptive_leaf_max = 0;
}

pfmm_status pfmm_create(const pfmm_config* cfg, pfmm_handle** out) {
  if (!out) return PFMM_ERR_INVALID_ARG;
  *out = nullptr;
  pfmm_handle* h = nullptr;
  try {
    validate_config(cfg);
    h = new pfmm_handle();
    h->cfg = *cfg;
    h->tab.build(cfg->order_p, cfg->ws, cfg->m2l_order_slack);
    const HostTables& T = h->tab;
    upload(h->t_mi, T.mi);
    upload(h->t_p2m, T.p2m_coef);
    upload(h->t_ifact, T.inv_fact);
    upload(h->t_l2p, T.l2p_tab);
    upload(h->t_code, T.m2l_code);
    upload(h->t_dvec, T.dvec);
    upload(h->t_hidx, T.hidx);
    upload(h->t_dorder, T.dorder);
    upload(h->t_slotq, T.slotq);
    if (cfg->precision == PFMM_MIXED) {
      std::vector<float> d32(T.dvec.begin(), T.dvec.end());
      upload(h->t_dvec32, d32);
    }
    OpTables& op = h->op;
    op.p = T.p; op.nc = T.nc; op.stride = T.stride;
    op.mi = h->t_mi.as<int>();
    op.p2m_coef = h->t_p2m.as<double>();
    op.inv_fact = h->t_ifact.as<double>();
    op.l2p_tab = h->t_l2p.as<int>();
    op.m2l_code = h->t_code.as<int>();
    op.noff = T.noff;
    op.dvec = h->t_dvec.as<double>();
    op.dvec32 = cfg->precision == PFMM_MIXED ? h->t_dvec32.as<float>() : nullptr;
    op.hidx = h->t_hidx.as<unsigned short>();
    op.dorder = h->t_dorder.as<unsigned char>();
    op.slotq = h->t_slotq.as<unsigned char>();
    op.nblocks = T.nblocks;
    if (cfg->mac_theta > 0.0 || cfg->adaptive_leaf_max > 0) {
      h->mac = true;
      h->leaf_max = cfg->adaptive_leaf_max;
      MacView& mv = h->mv;
      if (cfg->mac_theta > 0.0) {
        // a split pair whose children can be accepted failed the criterion (or was adjacent): its
        // offset D has |D| <= (r_A + r_B) / (theta w) <= sqrt(3) / theta, as every particle of a cell
        // lies within sqrt(3) w / 2 of its centre; the child offsets 2 D + (o_B - o_A) then lie within
        // 2 Rp + 1, the radius of the operator table
        mv.use_theta = 1;
        mv.minsep = 2;
        mv.theta = cfg->mac_theta;
        mv.ndirect = cfg->mac_ndirect;
        mv.leaf_direct = cfg->mac_leaf_direct;
        mv.Rp = std::max(1, (int)std::floor(std::sqrt(3.0) / cfg->mac_theta * (1.0 + 1e-9)));
      } else {
        // the ws rule on the adaptive octree: split pairs lie within ws, accepted ones beyond
        mv.use_theta = 0;
        mv.minsep = cfg->ws + 1;
        mv.theta = 0.0;
        mv.ndirect = 0;
        mv.leaf_direct = 0;
        mv.Rp = cfg->ws;
      }
      const std::vector<double> rows = mac_operator_rows(T, 2 * mv.Rp + 1);
      upload(h->t_mdvec, rows);
      mv.dvec = h->t_mdvec.as<double>();
      if (cfg->precision == PFMM_MIXED) {
        upload(h->t_mdvec32, std::vector<float>(rows.begin(), rows.end()));
        mv.dvec32 = h->t_mdvec32.as<float>();
      }
    }
    PFMM_HIP(hipGetDevice(&h->device));
    // host staging for the small read-backs, so that later calls need not allocate it
    h->pinned.get(4096);
    // the device address of the scratch array on this device (pfmm_field_noalloc)
    (void)scratch_address();
    *out = h;
    return PFMM_OK;
  } catch (const Error& e) {
    delete h;
    return e.status;
  } catch (const std::bad_alloc&) {
    delete h;
    return PFMM_ERR_OOM;
  }
}

void pfmm_destroy(pfmm_handle* h) { delete h; }

pfmm_status pfmm_solve(pfmm_handle* h, int64_t n, const double* pos, const double* q, const double* alpha,
                       double* mu, double* forces, double* phi, pfmm_result* res, void* stream) {
  return pfmm_solve_qe(h, n, pos, q, nullptr, alpha, mu, forces, phi, nullptr, res, stream);
}

pfmm_status pfmm_solve_qe(pfmm_handle* h, int64_t n, const double* pos, const double* q, const double* qE,
                          const double* alpha, double* mu, double* forces, double* phi, double* phi_E,
                          pfmm_result* res, void* stream) {
  if (!h) return PFMM_ERR_INVALID_ARG;
  h->err.clear();
  try {
    return solve_impl(h, n, pos, q, qE, alpha, mu, forces, phi, phi_E, res, (hipStream_t)stream);
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return PFMM_ERR_OOM;
  }
}

pfmm_status pfmm_backward(pfmm_handle* h, double g, double* grad_pos, double* grad_q, double* grad_alpha,
                          void* stream) {
  return pfmm_backward_qe(h, 0, g, grad_pos, grad_q, nullptr, grad_alpha, stream);
}

pfmm_status pfmm_backward_qe(pfmm_handle* h, int64_t solve_id, double g, double* grad_pos, double* grad_q,
                             double* grad_qE, double* grad_alpha, void* stream) {
  if (!h) return PFMM_ERR_INVALID_ARG;
  h->err.clear();
  try {
    if (!h->saved || !(h->cfg.flags & PFMM_SAVE_FOR_BACKWARD))
      throw Error(PFMM_ERR_NO_STATE, "pfmm_backward needs a preceding successful pfmm_solve with PFMM_SAVE_FOR_BACKWARD");
    if (solve_id != 0 && solve_id != h->saved_id)
      throw Error(PFMM_ERR_NO_STATE, "the state of solve " + std::to_string(solve_id) +
                                         " is gone: the handle holds that of solve " + std::to_string(h->saved_id));
    if (!std::isfinite(g)) throw Error(PFMM_ERR_NONFINITE, "non-finite upstream gradient");
    if (grad_qE && !h->saved_qE)
      throw Error(PFMM_ERR_INVALID_ARG, "grad_qE needs a preceding solve with field charges qE");
    hipStream_t s = (hipStream_t)stream;
    const int n = h->saved_n;
    if (n == 0) return PFMM_OK;
    double* dal = nullptr;
    if (grad_alpha && h->cfg.thole_a > 0.0) {
      dal = dev<double>(h->w_dal, n);
      launch_p2p(h->tv, h->pa, h->w_mu4.as<double4>(), 2, 2, false, FieldOut{}, dal, nullptr, nullptr, s);
      if (h->x_active)
        launch_exclusions(h->pa, h->w_perm.as<int>(), h->w_inv.as<int>(), h->x_ptr.as<int>(), h->x_idx.as<int>(),
                          h->w_mu4.as<double4>(), 2, 2, FieldOut{}, dal, nullptr, s);
    }
    launch_backward(h->pa, h->w_perm.as<int>(), h->w_mu4.as<double4>(), h->s_F.as<double>(),
                    h->s_phi.as<double>(), h->s_Etot.as<double>(), h->s_phiE.as<double>(), dal,
                    h->cfg.coulomb_k, g, grad_pos, grad_q, grad_qE, grad_alpha, s);
    return PFMM_OK;
  } catch (const Error& e) {
    return fail(h, e);
  }
}

pfmm_status pfmm_backward_mu(pfmm_handle* h, int64_t solve_id, const double* g_mu, double* grad_pos, double* grad_q,
                             double* grad_qE, double* grad_alpha, void* stream) {
  if (!h) return PFMM_ERR_INVALID_ARG;
  h->err.clear();
  try {
    if (!h->saved || !(h->cfg.flags & PFMM_SAVE_FOR_BACKWARD))
      throw Error(PFMM_ERR_NO_STATE, "pfmm_backward_mu needs a preceding successful pfmm_solve with PFMM_SAVE_FOR_BACKWARD");
    if (solve_id != 0 && solve_id != h->saved_id)
      throw Error(PFMM_ERR_NO_STATE, "the state of solve " + std::to_string(solve_id) +
                                         " is gone: the handle holds that of solve " + std::to_string(h->saved_id));
    if (grad_qE && !h->saved_qE)
      throw Error(PFMM_ERR_INVALID_ARG, "grad_qE needs a preceding solve with field charges qE");
    const int n = h->saved_n;
    if (n == 0) return PFMM_OK;
    if (!g_mu) throw Error(PFMM_ERR_INVALID_ARG, "dL/dmu is NULL");
    hipStream_t s = (hipStream_t)stream;
    const pfmm_config& c = h->cfg;
    const Particles& pa = h->pa;
    const int* perm = h->w_perm.as<int>();
    h->kt.reset(false, s);
    int* err = dev<int>(h->w_flags, 4);
    launch_fill_int(err, 4, 0, s);
    launch_check_finite(g_mu, 3 * (int64_t)n, err + 1, s);
    double* Gs = dev<double>(h->a_G, 3 * (int64_t)n);
    launch_permute_vec3(perm, n, g_mu, Gs, s);
    // the solution's dipoles: the adjoint solve uses the dipole buffer for its search directions
    double4* mu4 = h->w_mu4.as<double4>();
    double4* mus = dev<double4>(h->a_mu4, n);
    PFMM_HIP(hipMemcpyAsync(mus, mu4, sizeof(double4) * (size_t)n, hipMemcpyDeviceToDevice, s));
    // the adjoint lambda = A^-1 dL/dmu: the same symmetric operator (same tree, orders and
    // preconditioner) with dL/dmu in place of the static field; every evaluation at the full orders
    // on the tree the forward solve ran on (that of the polarisable sites with dipole_tree)
    pfmm_handle* hm = h->sites_active ? h->sites : h;
    const int m = h->sites_active ? h->n_sites : n;
    const double* Gcg = Gs;
    int* errcg = err;
    if (h->sites_active) {
      double* gm = dev<double>(h->t_rhs, 3 * (int64_t)m);
      launch_permute_vec3(h->t_comp.as<int>(), m, g_mu, gm, s);
      Gcg = gm;
      dev<double4>(hm->w_mu4, m);
      errcg = dev<int>(hm->w_flags, 4);
      launch_fill_int(errcg, 4, 0, s);
      hm->kt.reset(false, s);
    }
    CGState* st = static_cast<CGState*>(hm->w_state.reserve(2 * sizeof(CGState)));
    RelaxParams rp;
    rp.p = c.order_p;
    rp.qmin = (c.order_p + 1) / 2;
    rp.track = 0;
    rp.start = 0.0;
    rp.lrho = 2.0 * std::log((c.ws + 1.0) / std::sqrt(3.0));
  // the float32 products of the mixed path add their rounding to every relaxed product: the relaxed
  // phase stops at half the tolerance, leaving room for it in the final check at the full orders
  rp.tol_scale = c.precision == PFMM_MIXED ? 0.5 : 1.0;
    launch_fill_int(&st->qcap, 1, c.order_p, s);
    int evals = 0;
    const CGState hs = dipole_cg(hm, Gcg, false, rp, st, errcg, s, &evals);
    if (hs.notspd) throw Error(PFMM_ERR_NOT_SPD, "adjoint solve met p.Ap <= 0");
    if (!hs.done || (hs.maxed && hs.res > c.scf_tol))
      throw Error(PFMM_ERR_NOT_CONVERGED, "adjoint solve did not converge: residual " + std::to_string(hs.res));
    double4* lam4 = dev<double4>(h->a_lam4, n);
    if (h->sites_active) {
      double4* lm = hm->w_mu4.as<double4>();
      launch_make_dipoles(hm->pa, hm->cg_y.as<double>(), lm, nullptr, s);
      launch_place_site_dipoles(h->t_map.as<int>(), m, lm, n, pa.tau, lam4, s);
    } else {
      launch_make_dipoles(pa, h->cg_y.as<double>(), lam4, nullptr, s);
    }
    // fields of the adjoint dipoles (potential, undamped and damped field, damped gradient)
    PFMM_HIP(hipMemcpyAsync(mu4, lam4, sizeof(double4) * (size_t)n, hipMemcpyDeviceToDevice, s));
    FieldOut lf{dev<double>(h->a_phi, n), dev<double>(h->a_Eu, 3 * (int64_t)n), dev<double>(h->a_Ed, 3 * (int64_t)n),
                dev<double>(h->a_G6, 6 * (int64_t)n)};
    fmm_pass(h, 2, 1, lf, err, nullptr, s);
    // the bilinear Thole term from the quadratic one, with lambda scaled to the dipoles' size
    double *dalp = nullptr, *dalm = nullptr;
    double inv2c = 0.0;
    if (grad_alpha && c.thole_a > 0.0) {
      const double sc = hs.bnorm2 > 0.0 && h->saved_bn2 > 0.0 ? std::sqrt(h->saved_bn2 / hs.bnorm2) : 1.0;
      double4* pl = dev<double4>(h->a_pl4, n);
      double4* mi = dev<double4>(h->a_mi4, n);
      launch_dipole_pm(n, mus, lam4, sc, pl, mi, s);
      dalp = dev<double>(h->a_dalp, n);
      dalm = dev<double>(h->a_dalm, n);
      for (int k = 0; k < 2; ++k) {
        double4* d4 = k == 0 ? pl : mi;
        double* dd = k == 0 ? dalp : dalm;
        launch_p2p(h->tv, pa, d4, 2, 2, false, FieldOut{}, dd, nullptr, nullptr, s);
        if (h->x_active)
          launch_exclusions(pa, perm, h->w_inv.as<int>(), h->x_ptr.as<int>(), h->x_idx.as<int>(), d4, 2, 2,
                            FieldOut{}, dd, nullptr, s);
      }
      inv2c = 0.5 / sc;
    }
    PFMM_HIP(hipMemcpyAsync(mu4, mus, sizeof(double4) * (size_t)n, hipMemcpyDeviceToDevice, s));
    const bool sep = h->saved_qE;
    launch_backward_mu(pa, perm, mus, lam4, lf, sep ? h->f_GqE.as<double>() : h->f_Gq.as<double>(),
                       h->f_Gm.as<double>(), h->s_Etot.as<double>(), Gs, sep ? h->w_qEs.as<double>() : nullptr,
                       dalp, dalm, inv2c, grad_pos, grad_q, grad_qE, grad_alpha, s);
    int flags[2];
    sync_read(h, err, flags, sizeof(flags), s);
    if (flags[1]) throw Error(PFMM_ERR_NONFINITE, "non-finite dL/dmu");
    return PFMM_OK;
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return PFMM_ERR_OOM;
  }
}

pfmm_status pfmm_set_exclusions(pfmm_handle* h, int64_t n64, const int* xptr, const int* xidx) {
  if (!h) return PFMM_ERR_INVALID_ARG;
  h->err.clear();
  try {
    if (n64 == 0 || !xptr) {
      h->saved = false;
      h->x_n = -1;
      h->x_active = false;
      return PFMM_OK;
    }
    if (n64 < 0 || n64 > INT_MAX / 8) throw Error(PFMM_ERR_INVALID_ARG, "n out of range");
    const int n = (int)n64;
    if (xptr[0] != 0) throw Error(PFMM_ERR_INVALID_ARG, "exclusion rows must start at 0");
    for (int i = 0; i < n; ++i)
      if (xptr[i + 1] < xptr[i]) throw Error(PFMM_ERR_INVALID_ARG, "exclusion row starts must not decrease");
    const int nnz = xptr[n];
    if (nnz > 0 && !xidx) throw Error(PFMM_ERR_INVALID_ARG, "exclusion indices are NULL");
    // every pair listed once in each of its two rows, no self pairs, indices in range
    std::vector<uint64_t> keys;
    keys.reserve(nnz);
    for (int i = 0; i < n; ++i)
      for (int k = xptr[i]; k < xptr[i + 1]; ++k) {
        const int j = xidx[k];
        if (j < 0 || j >= n || j == i) throw Error(PFMM_ERR_INVALID_ARG, "exclusion index out of range or self");
        const uint64_t a = (uint64_t)std::min(i, j), b = (uint64_t)std::max(i, j);
        keys.push_back((a << 32) | b);
      }
    std::sort(keys.begin(), keys.end());
    for (size_t k = 0; k < keys.size(); k += 2)
      if (k + 1 >= keys.size() || keys[k] != keys[k + 1] || (k + 2 < keys.size() && keys[k + 2] == keys[k]))
        throw Error(PFMM_ERR_INVALID_ARG, "each excluded pair must appear once in both of its rows");
    int* dp = dev<int>(h->x_ptr, n + 1);
    int* di = dev<int>(h->x_idx, std::max(nnz, 1));
    PFMM_HIP(hipMemcpy(dp, xptr, sizeof(int) * (size_t)(n + 1), hipMemcpyHostToDevice));
    if (nnz > 0) PFMM_HIP(hipMemcpy(di, xidx, sizeof(int) * (size_t)nnz, hipMemcpyHostToDevice));
    h->x_n = n;
    h->x_active = false;
    h->saved = false;  // a saved solve no longer matches the handle's exclusions
    return PFMM_OK;
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return PFMM_ERR_OOM;
  }
}

}  // extern "C"

namespace {

// One FMM evaluation of fixed sources (pfmm_field and pfmm_field_noalloc).
pfmm_status field_impl(pfmm_handle* h, int64_t n64, const double* pos, const double* q, const double* mu,
                       const double* alpha, double* phi, double* E, double* E_damped, double* grad_E,
                       void* stream) {
  {
    hipStream_t s = (hipStream_t)stream;
    if (n64 < 0 || n64 > INT_MAX / 8) throw Error(PFMM_ERR_INVALID_ARG, "n out of range");
    h->saved = false;
    const int n = (int)n64;
    if (n == 0) return PFMM_OK;
    if (!pos || !alpha) throw Error(PFMM_ERR_INVALID_ARG, "NULL positions or polarizabilities");
    build_tree(h, n, pos, q, alpha, s);
    activate_exclusions(h, n, s);
    double4* mu4 = dev<double4>(h->w_mu4, n);
    int* err = dev<int>(h->w_flags, 4);
    launch_fill_int(err, 4, 0, s);
    if (mu) {
      launch_check_finite(mu, 3 * n64, err + 1, s);
      launch_permute_dipoles(h->w_perm.as<int>(), n, mu, h->pa.tau, mu4, s);
    }
    const int sources = (q ? 1 : 0) | (mu ? 2 : 0);
    double* ph = dev<double>(h->f_phim, n);
    double* Eu = dev<double>(h->f_Eum, 3 * (int64_t)n);
    double* Ed = dev<double>(h->f_Edm, 3 * (int64_t)n);
    double* G = dev<double>(h->f_Gm, 6 * (int64_t)n);
    FieldOut fo{ph, Eu, Ed, G};
    if (sources == 0) {
      launch_fill_double(ph, n, 0.0, s);
      launch_fill_double(Eu, 3 * n64, 0.0, s);
      launch_fill_double(Ed, 3 * n64, 0.0, s);
      launch_fill_double(G, 6 * n64, 0.0, s);
    } else {
      fmm_pass(h, sources, 1, fo, err, nullptr, s);
    }
    int flags[2];
    sync_read(h, err, flags, sizeof(flags), s);
    if (flags[1]) throw Error(PFMM_ERR_NONFINITE, "non-finite dipole");
    if (flags[0]) throw Error(PFMM_ERR_COINCIDENT, "two particles share the same position");
    launch_unpermute_field(h->w_perm.as<int>(), n, fo, phi, E, E_damped, grad_E, s);
    PFMM_HIP(hipStreamSynchronize(s));
    return PFMM_OK;
  }
}

// Makes the workspace of the calls on this thread come from a region of device memory.
struct ArenaScope {
  Arena arena;
  explicit ArenaScope(char* base, size_t cap) {
    arena.base = base;
    arena.cap = cap;
    g_arena = &arena;
  }
  ~ArenaScope() { g_arena = nullptr; }
};

}  // namespace

extern "C" {

pfmm_status pfmm_field(pfmm_handle* h, int64_t n64, const double* pos, const double* q, const double* mu,
                       const double* alpha, double* phi, double* E, double* E_damped, double* grad_E,
                       void* stream) {
  if (!h) return PFMM_ERR_INVALID_ARG;
  h->err.clear();
  try {
    return field_impl(h, n64, pos, q, mu, alpha, phi, E, E_damped, grad_E, stream);
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return PFMM_ERR_OOM;
  }
}

pfmm_status pfmm_field_noalloc(pfmm_handle* h, int64_t n64, const double* pos, const double* q, const double* mu,
                               const double* alpha, double* phi, double* E, double* E_damped, double* grad_E,
                               void* stream) {
  if (!h) return PFMM_ERR_INVALID_ARG;
  h->err.clear();
  try {
    ArenaScope scope(scratch_address(), SCRATCH_BYTES);
    return field_impl(h, n64, pos, q, mu, alpha, phi, E, E_damped, grad_E, stream);
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return PFMM_ERR_OOM;
  }
}

const char* pfmm_status_string(pfmm_status s) {
  switch (s) {
    case PFMM_OK: return "ok";
    case PFMM_ERR_INVALID_ARG: return "invalid argument";
    case PFMM_ERR_NONFINITE: return "non-finite input";
    case PFMM_ERR_COINCIDENT: return "coincident particles";
    case PFMM_ERR_NOT_CONVERGED: return "dipole solve did not converge";
    case PFMM_ERR_NOT_SPD: return "dipole system not positive definite";
    case PFMM_ERR_OOM: return "out of memory";
    case PFMM_ERR_HIP: return "HIP runtime error";
    case PFMM_ERR_NO_STATE: return "no saved state for backward";
  }
  return "unknown status";
}

const char* pfmm_last_error(const pfmm_handle* h) { return h ? h->err.c_str() : ""; }

const char* pfmm_version(void) { return "pfmm 0.1.0 (gfx950)"; }

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Internal inspection hook for tests and debugging (not part of the public interface): device
// pointer and size of a named workspace buffer of the last tree build / evaluation.
// ------------------------------------------------------------------------------------------------
extern "C" int pfmm_internal_buffer(pfmm_handle* h, const char* name, void** ptr, int64_t* bytes) {
  if (!h || !name || !ptr || !bytes) return PFMM_ERR_INVALID_ARG;
  const std::string s(name);
  const TreeView& t = h->tv;
  const int64_t rows = (int64_t)t.ncell + 1;
  struct Item { const char* n; const DevBuf* b; int64_t size; };
  const Item items[] = {
      {"M", &h->w_M, rows * h->op.stride * 8}, {"F", &h->w_F, rows * h->op.stride * 8},
      {"ckey", &h->w_ckey, (int64_t)t.ncell * 8}, {"cfirst", &h->w_cfirst, (int64_t)t.ncell * 4},
      {"ccount", &h->w_ccount, (int64_t)t.ncell * 4}, {"cparent", &h->w_cparent, (int64_t)t.ncell * 4},
      {"child8", &h->w_child8, (int64_t)t.ncell * 32}, {"coll", &h->w_coll, (int64_t)t.ncell * t.nnear * 4},
      {"perm", &h->w_perm, (int64_t)h->pa.n * 4},
      {"P", &h->w_P, (int64_t)h->pa.n * 32}};
  for (const auto& it : items)
    if (s == it.n) {
      *ptr = it.b->ptr;
      *bytes = it.size;
      return PFMM_OK;
    }
  if (s == "tree") {  // host copy of the level offsets and geometry: int L, int ncell, int off[23], double origin[3], double w
    static thread_local char buf[4 + 4 + 4 * (MAX_LEVELS + 2) + 8 * 4];
    std::memcpy(buf, &t.L, 4);
    std::memcpy(buf + 4, &t.ncell, 4);
    std::memcpy(buf + 8, t.off, 4 * (MAX_LEVELS + 2));
    std::memcpy(buf + 8 + 4 * (MAX_LEVELS + 2), t.origin, 24);
    std::memcpy(buf + 8 + 4 * (MAX_LEVELS + 2) + 24, &t.w, 8);
    *ptr = buf;
    *bytes = sizeof(buf);
    return PFMM_OK;
  }
  return PFMM_ERR_INVALID_ARG;
}

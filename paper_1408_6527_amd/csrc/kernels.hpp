// Launchers of the HIP kernels of the pfmm library (one translation unit per group).
// Every launcher enqueues on the given stream and checks the launch; none synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace pfmm {

constexpr int MAX_LEVELS = 21;  // 63-bit Morton keys
constexpr int MAX_P = 12;       // highest expansion order
constexpr int MAX_P_MFMA = 10;  // highest order of the matrix-core M2L (its tile's LDS and registers);
                                // orders above run the vector M2L (m2l.hip, k_m2l_vector)
constexpr int MAX_P_MAC = 9;    // highest order of the acceptance-criterion M2L

// Device view of the octree.  Cells of all levels live in one array, level by level; inside a
// level they are in Morton order, so each cell's particles are a contiguous range of the sorted
// particle arrays and each cell's children are contiguous in the next level.
struct TreeView {
  int L = 0;                       // leaf level
  int ncell = 0;                   // cells on all levels
  int off[MAX_LEVELS + 2] = {0};   // first cell of each level; off[L + 1] = ncell
  double origin[3] = {0, 0, 0};
  double w = 1.0;                  // leaf edge
  int ws = 1, nnear = 1;
  int damp_adjacent = 0;           // 1: the Thole damping radius is at most the leaf edge, so only
                                   // adjacent leaves hold damped pairs
  const uint64_t* key = nullptr;   // cell key at its own level (3 bits per level)
  const int* first = nullptr;      // first sorted particle
  const int* count = nullptr;      // particles in the cell
  const int* parent = nullptr;     // global index of the parent, -1 at the root
  const int* child8 = nullptr;     // 8 global child indices per cell (octant order), -1 if empty
  const int* coll = nullptr;       // nnear colleagues per cell (offset order), -1 if empty
  // near field from the acceptance-criterion walk (mac.hip) instead of the colleagues: for leaf
  // g - off[L], the source leaves nidx[nptr[g - off[L]] .. nptr[g - off[L] + 1]); null otherwise
  const int* nptr = nullptr;
  const int* nidx = nullptr;
};

// Particle arrays in sorted (Morton) order.
struct Particles {
  int n = 0;
  const double4* P = nullptr;      // x, y, z, q
  const double* alpha = nullptr;   // polarisability
  const double* sqa = nullptr;     // sqrt(alpha)
  const double* tau = nullptr;     // sqrt(thole_a) * alpha^(1/6): s_ij = tau_i tau_j
  const double* itau = nullptr;    // 1 / tau, 0 where tau = 0 (no damping)
};

// Field outputs in sorted order (any may be null when not requested by the mode).
struct FieldOut {
  double* phi = nullptr;  // n
  double* Eu = nullptr;   // 3n, field with undamped dipole part
  double* Ed = nullptr;   // 3n, field with damped dipole part
  double* G = nullptr;    // 6n, d_a (Ed)_b as xx, yy, zz, xy, xz, yz
};

// ---------------------------------------------------------------- tree.hip
void launch_scan_inputs(const double* pos, const double* q, const double* alpha, int n,
                        double* partial, int nblk, int* flags, hipStream_t s);
void launch_bbox_final(const double* partial, int nblk, double* bbox, hipStream_t s);
void launch_morton(const double* pos, int n, const double origin[3], double w, int L,
                   uint64_t* keys, int* vals, hipStream_t s);
size_t sort_temp_bytes(int n, int end_bit);
void launch_sort(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int* vin,
                 int* vout, int n, int end_bit, hipStream_t s);
void launch_gather(const int* perm, const double* pos, const double* q, const double* alpha, int n,
                   double sqrt_a, double4* P, double* al, double* sqa, double* tau, double* itau,
                   hipStream_t s);
size_t scan_temp_bytes(int n);
void launch_inclusive_scan(void* tmp, size_t tmp_bytes, const int* in, int* out, int n, hipStream_t s);
// cid[i] = 1 + index (within the level) of the cell holding sorted particle i (inclusive scan of
// the cell-head flags); *count_out = cells on the level.
void launch_level_scan(const uint64_t* keys, int n, int shift, int* flags, int* cid, int* count_out,
                       void* tmp, size_t tmp_bytes, hipStream_t s);
void launch_fill_int(int* p, int64_t count, int value, hipStream_t s);
void launch_fill_double(double* p, int64_t count, double value, hipStream_t s);
void launch_cells(const uint64_t* keys, int n, int L, int l, const int* cid_l, const int* cid_parent,
                  int off_l, int off_parent, uint64_t* ckey, int* cfirst, int* cparent, int* child8,
                  hipStream_t s);
void launch_cell_counts(const int* cfirst, int off_l, int ncell_l, int n, int* ccount, hipStream_t s);
void launch_colleagues(const uint64_t* ckey, int off_l, int ncell_l, int l, int ws, int* coll,
                       hipStream_t s);
// stats[0] += M2L pairs with a source, stats[1] += ordered near-field particle pairs,
// stats[2] += useful M2L flops (2 C(q+6, 6) per pair of truncation order q = dorder[slot]),
// stats[3 + c] += the same flops with every order capped at c, c = 0 .. p
void launch_tree_stats(const TreeView& t, const int* m2l_code, const unsigned char* dorder, int noff,
                       int p, unsigned long long* stats, hipStream_t s);

// ---------------------------------------------------------------- expansions.hip
struct OpTables {
  int p = 0, nc = 0, stride = 0;
  const int* mi = nullptr;
  const double* p2m_coef = nullptr;
  const double* inv_fact = nullptr;
  const int* l2p_tab = nullptr;  // 16 ints per coefficient: nx ny nz |n|, n+e_c (3), n+e_a+e_b (6), pad
  const int* m2l_code = nullptr; int noff = 0;  // M2L offsets per target octant (tree statistics)
  // M2L operators: D_k(d) at unit cell width for every offset d in [-R, R]^3, R = 2 ws + 1, as
  // rows of sched_dpitch(p) values (float copy only on the mixed path), and the K-entry index table
  // (one index into such a row per MFMA block and lane, schedule.hpp)
  const double* dvec = nullptr; const float* dvec32 = nullptr; const unsigned short* hidx = nullptr;
  const unsigned char* dorder = nullptr;  // truncation order per offset slot
  const unsigned char* slotq = nullptr;   // highest order per (colleague offset, source octant)
  int nblocks = 0;
};
// sources: 1 = charges (P.w), 2 = dipoles (mu4), 3 = both
// pair_dl > 0 with dipole sources: dipole multipoles from the +/- q^mu pairs of Sec. II.C
void launch_p2m(const TreeView& t, const OpTables& op, const Particles& pa, const double4* mu4,
                int sources, double pair_dl, double* M, const int* done, hipStream_t s);
void launch_m2m(const TreeView& t, const OpTables& op, int parent_level, double* M, const int* done,
                hipStream_t s);
// F~(child) += partial M2L sums of splits 1..nsplit-1 (at F + s * split_stride) and, from level 3
// on, the shift of F~(parent).
void launch_l2l(const TreeView& t, const OpTables& op, int child_level, double* F, int nsplit,
                int64_t split_stride, const int* done, hipStream_t s);
// mode 0: Ed only (written, not added); mode 1: phi, Eu, Ed, G written
void launch_l2p(const TreeView& t, const OpTables& op, const Particles& pa, const double* F, int mode,
                FieldOut out, const int* done, hipStream_t s);

// ---------------------------------------------------------------- m2l.hip
// Targets are the cells of levels >= 2, taken as the children of 16-parent tiles; a launch covers
// the parents of levels [lp_lo, lp_hi].  Workgroup tiles of 16 ncb parents over those levels:
int m2l_tiles(const TreeView& t, int lp_lo, int lp_hi, int ncb = 1);
// 16-parent tiles per M2L workgroup for order p on the float64 or float32 path
int m2l_tile_ncb(int p, bool fp32);
// Split s of the colleague-offset range writes its partial F~ at F + s * split_stride (s = 0: F
// itself); the downward pass (launch_l2l) adds the partials of splits 1.. to F.  On the mixed path,
// targets at levels <= fp64_max_level still run in float64.
// qcap (device, may be NULL): every offset's order is capped at *qcap.  M32: float32 copy of M,
// read by the float32 launches of the mixed path (launch_to_float).
struct MacView;
// mac (may be NULL): the dual walk's lists instead of the ws lists: the split partners of each
// parent take the place of its colleagues and every child pair is tested with the walk's rule; the
// float32 tiles of the mixed path read mac->dvec32.
void launch_m2l(const TreeView& t, const OpTables& op, int nsplit, const double* M, const float* M32,
                double* F, int64_t split_stride, bool fp32, int fp64_max_level, const int* done,
                const int* qcap, hipStream_t s, const MacView* mac = nullptr);
void launch_to_float(const double* in, float* out, int64_t count, const int* done, hipStream_t s);

// ---------------------------------------------------------------- p2p.hip
// mode 0: dipole sources, Ed only (added); mode 1: full outputs (added) from charges and/or dipoles
// (sources bit 1 = charges, bit 2 = dipoles); mode 2: Thole term of dU/dalpha (written to dal);
// mode 3: damped field of the dipoles within rc of each target, over the adjacent leaves only
// (written to Ed): the operator of the dipole-solve preconditioner.
void launch_p2p(const TreeView& t, const Particles& pa, const double4* mu4, int mode, int sources,
                bool fp32, FieldOut out, double* dal, int* err, const int* done, hipStream_t s,
                double rc = 0.0);
// takes the exact terms of the excluded pairs (rows xptr/xidx in the caller's order) off an
// evaluation of P2P mode 0, 1 or 2; inv = sorted position of each caller index
void launch_exclusions(const Particles& pa, const int* perm, const int* inv, const int* xptr, const int* xidx,
                       const double4* mu4, int mode, int sources, FieldOut out, double* dal, const int* done,
                       hipStream_t s);
void launch_inverse_perm(const int* perm, int n, int* inv, hipStream_t s);

// ---------------------------------------------------------------- mac.hip
// The lists of the dual tree walk: the acceptance rule's parameters, the cells' enclosing radii, and
// for every cell of levels < L the partners of its split pairs (the pairs whose children the walk
// examined): split[B (2 Rp + 1)^3 + slot(A - B)] = A, -1 elsewhere, the offsets of split pairs that
// can have accepted children lying in [-Rp, Rp]^3.  The M2L kernel runs over these like the
// colleagues of the ws lists and applies the rule to the children (mac.hpp); dvec holds D_k(d) at
// unit cell width for every offset in [-(2 Rp + 1), 2 Rp + 1]^3 at the row pitch of the M2L tables.
// Acceptance of two distinct cells of one level at Chebyshev distance >= minsep holding at least
// ndirect particles together (with leaf_direct, not both terminal): with use_theta the criterion
// theta |z_B - z_A| > r_B + r_A (minsep 2), otherwise nothing more (the ws rule, minsep ws + 1).
// Adaptive octree (nonleaf != NULL): nonleaf[c] = 1 for the cells that are split (the others, and
// all cells of level L, are terminal), and lfirst[c] / lcount[c] the range of the level-L cells
// below c; a pair of terminal cells that is not accepted is summed directly at any level.  Without
// it, only the cells of level L are terminal.
struct MacView {
  double theta = 0.0;
  int use_theta = 1, minsep = 2;
  int ndirect = 0, leaf_direct = 0, Rp = 0;
  const double* renc = nullptr;
  const int* split = nullptr;
  const double* dvec = nullptr;
  const float* dvec32 = nullptr;  // float copy of dvec (mixed path)
  const int* nonleaf = nullptr;
  const int* lfirst = nullptr;
  const int* lcount = nullptr;
};
// enclosing radius of every cell of a level: the largest distance from its centre to its particles
void launch_mac_radii(const TreeView& t, const double4* P, int level, double* renc, hipStream_t s);
// one level of the walk over the frontier pairs fr (target, source) of level l:
// classify: acc[i] = 1 if the pair is accepted for M2L; otherwise, when both cells are terminal,
// nearc[i] = the near-list entries it makes (one per level-L cell below the target, each paired with
// the source cell), else kid[i] = its child pairs; the other two are 0;
// emit (from the inclusive prefix sums of kid and nearc): child pairs to next and the split
// table's entries, near entries to near_tgt / near_src (level-L target, source cell of level l);
// *bad |= 1 for a split pair whose children could be accepted outside [-Rp, Rp]^3 (which the bound
// on the radii rules out)
void launch_mac_classify(const TreeView& t, const MacView& mv, int level, const int2* fr, int nfr, int* acc, int* kid,
                         int* nearc, hipStream_t s);
void launch_mac_emit(const TreeView& t, const MacView& mv, int level, const int2* fr, int nfr, const int* kid_scan,
                     const int* near_scan, int2* next, int* split, int* near_tgt, int* near_src, int* bad,
                     hipStream_t s);
// useful M2L flops of the accepted pairs of a frontier (acc from classify), 2 C(q + 6, 6) per pair at
// its order q (p with the criterion, the per-offset order dorder of the ws rule): added to st[0], and
// with every order capped at c <= p to st[1 + c] (MAX_P + 2 entries)
void launch_mac_flops(const TreeView& t, const MacView& mv, const int2* fr, int nfr, const int* acc,
                      const unsigned char* dorder, int p, unsigned long long* st, hipStream_t s);
// Adaptive octree: nonleaf[c] = 1 for the cells of level < L holding more than leaf_max particles
// (one launch per level), then, from level L - 1 up to 0, every cell of level l touching a split
// cell of level l + 1 is split (2:1 balance over the full octree); lfirst / lcount: the level-L cells
// below each cell of a level
void launch_adapt_init(const TreeView& t, int level, int leaf_max, int* nonleaf, hipStream_t s);
void launch_adapt_balance(const TreeView& t, int level, int* nonleaf, hipStream_t s);
void launch_leaf_range(const TreeView& t, int level, int* lfirst, int* lcount, hipStream_t s);
// stable sort of (key, value) int pairs by key over the low end_bit bits
size_t mac_sort_temp_bytes(int n, int end_bit);
void launch_mac_sort(void* tmp, size_t tmp_bytes, const int* kin, int* kout, const int* vin, int* vout, int n,
                     int end_bit, hipStream_t s);
// counts per key (keys - key0 in [0, nkey)), added to cnt
void launch_mac_count(const int* keys, int n, int key0, int* cnt, hipStream_t s);
// ordered near-field particle pairs of the near list (i != j; the target cell may lie inside the
// source cell), added to *pairs
void launch_mac_near_pairs(const TreeView& t, const int* near_tgt, const int* near_src, int n,
                           unsigned long long* pairs, hipStream_t s);

// ---------------------------------------------------------------- solver.hip
struct CGState {
  double rr, pAp, a, b, bnorm2, res, res_true, res_max;
  int done, iters, notspd, maxed;
  int qcap;      // M2L order cap of the next field evaluation (relaxed solve)
  int ncap[16];  // field evaluations of the solve per order cap (not reset by the init kernels)
};
// Relaxed field evaluations of the outer solve: after each update with relative residual r >= 0,
// qcap = max(qmin, p - floor(ln(start / r) / lrho)) when r < start; track = 0 leaves qcap and ncap
// alone (inner solves).
struct RelaxParams {
  int p = 0, qmin = 0, track = 0;
  double start = 0.0, lrho = 1.0;
  double tol_scale = 1.0;  // a relaxed solve stops at tol_scale * scf_tol (its final check: scf_tol)
};
constexpr int RED_BLOCKS = 512;   // partial sums per reduction
void launch_cg_init(const Particles& pa, const double* Eq, const double4* mu_warm, bool warm,
                    double* y, double* pvec, double4* mu4, double* part, CGState* st, hipStream_t s);
void launch_cg_residual0(const Particles& pa, const double* Eq, const double* E, double* y,
                         double* r, double* pvec, double* part, CGState* st, double tol,
                         hipStream_t s);
void launch_make_dipoles(const Particles& pa, const double* v, double4* mu4, const int* done,
                         hipStream_t s);
void launch_cg_ap(const Particles& pa, const double* pvec, const double* E, double* Ap, double* part,
                  CGState* st, hipStream_t s);
void launch_cg_update(const Particles& pa, double* y, double* r, const double* pvec, const double* Ap,
                      double* part, CGState* st, double tol, int max_iter, hipStream_t s,
                      const RelaxParams& rp = RelaxParams());
void launch_cg_direction(int n3, const double* r, double* pvec, const CGState* st, hipStream_t s);
// cold start y0 = 0, r0 = S E^q (no field evaluation)
void launch_cg_init_zero(const Particles& pa, const double* Eq, double* y, double* r, double* part,
                         CGState* st, double tol, hipStream_t s);
// flexible preconditioned CG: q = A p with a = p.r / p.q; b = -z.q / p.q; inner-solve start
void launch_pcg_ap(const Particles& pa, const double* pvec, const double* E, const double* r, double* Ap,
                   double* part, CGState* st, hipStream_t s);
void launch_pcg_zq(int n3, const double* z, const double* Ap, double* part, CGState* st, hipStream_t s);
void launch_pc_init(int n3, const double* r, double* z, double* ri, double* pi, double* part,
                    CGState* inner, const CGState* outer, hipStream_t s);

struct EnergyParts { double Uqq, Amu, muEq, muEd, res2, bn2, resmax; };
// The static field that polarises the dipoles, from the charges q^E (Sec. III): qE (sorted) or
// nullptr when q^E = q, and that field E (n x 3) and its gradient G (n x 6).
struct FieldCharges {
  const double* qE = nullptr;
  const double* E = nullptr;
  const double* G = nullptr;
};
void launch_backward_mu(const Particles& pa, const int* perm, const double4* mu4, const double4* lam4,
                        const FieldOut& lam, const double* Ge, const double* Gm, const double* Etot, const double* Gs,
                        const double* qEs, const double* dalp, const double* dalm, double inv2c, double* gpos,
                        double* gq, double* gqE, double* ga, hipStream_t s);
void launch_flag_polarisable(const double* alpha, int n, int* flags, hipStream_t s);
void launch_compact_sites(const int* scan, const double* pos, const double* alpha, int n, int* idx, double* spos,
                          double* salpha, double* sq, hipStream_t s);
void launch_site_maps(const int* perm_mu, const int* idx, const int* inv, int m, int* comp, int* map, hipStream_t s);
void launch_place_site_dipoles(const int* map, int m, const double4* src, int n, const double* tau, double4* dst,
                               hipStream_t s);
void launch_permute_vec3(const int* perm, int n, const double* in, double* out, hipStream_t s);
void launch_dipole_pm(int n, const double4* a, const double4* b, double c, double4* plus, double4* minus,
                      hipStream_t s);
void launch_assemble(const Particles& pa, const int* perm, const double4* mu4, const double* phiq,
                     const double* Eq, const FieldCharges& fc, const double* phim, const double* Eum,
                     const double* Edm, const double* Gm, double k_e, double* mu_out,
                     double* F_out, double* phi_out, double* phiE_out, double* F_s, double* phi_s,
                     double* phiE_s, double* Etot_s, double* part, EnergyParts* ep, hipStream_t s);
void launch_backward(const Particles& pa, const int* perm, const double4* mu4, const double* F_s,
                     const double* phi_s, const double* Etot_s, const double* phiE_s, const double* dal_thole,
                     double k_e, double g, double* gpos, double* gq, double* gqE, double* galpha,
                     hipStream_t s);
// PE[i] = (P[i].xyz, qE[perm[i]]), qEs[i] = qE[perm[i]]
void launch_field_charges(const int* perm, int n, const double4* P, const double* qE, double4* PE,
                          double* qEs, hipStream_t s);
void launch_unpermute_field(const int* perm, int n, const FieldOut& src, double* phi, double* E,
                            double* Ed, double* G9, hipStream_t s);
void launch_permute_dipoles(const int* perm, int n, const double* mu_in, const double* tau,
                            double4* mu4, hipStream_t s);
void launch_check_finite(const double* v, int64_t count, int* flags, hipStream_t s);

}  // namespace pfmm

/*
 * pfmm — polarizable fast multipole method on AMD MI355X (gfx950).
 *
 * C interface of the library libpfmm.so.  It evaluates the electrostatics of point charges and
 * self-consistent induced point dipoles of Coles & Masella, "The Fast Multipole Method and Point
 * Dipole Moment Polarizable Force Fields" (arXiv:1408.6527):
 *
 *   U      = U^{qq'} + U^pol                                   (Sec. II.A, energy decomposition)
 *   U^{qq'} = 1/2 sum_i q_i sum_{j != i} q_j / r_ij             (Sec. II.A, Coulomb energy)
 *   mu_i   = alpha_i (E^q_i + E^mu_i)                          (Sec. II.A, dipole-moment equation)
 *   U^pol  = 1/2 sum |mu_i|^2/alpha_i - sum mu_i.E^q_i - 1/2 sum mu_i.E^mu_i
 *                                                              (Sec. II.A, A(mu) and U^pol)
 * with the fields evaluated by a Cartesian Taylor FMM (Sec. II.B-II.C) on a Morton-sorted,
 * uniform-depth octree, the dipoles found by conjugate gradients on the symmetric scaled system,
 * and forces and parameter gradients taken at fixed converged dipoles (stationarity, Sec. II.A).
 *
 * Conventions used by every entry point
 *   - Units: positions in Angstrom, charges in e, polarisabilities as volumes in Angstrom^3,
 *     dipoles in e*Angstrom.  Energies, forces and potentials returned by pfmm_solve and
 *     pfmm_backward are multiplied by cfg.coulomb_k (default 332.06371 kcal*Angstrom/(mol*e^2)).
 *   - Every pointer to particle data is a DEVICE pointer to float64 data on the current HIP
 *     device, owned by the caller.  pos, mu, forces are n x 3 row-major (x, y, z per particle);
 *     n-vectors are contiguous.  Inputs are read only; outputs are fully overwritten.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).  The calls that return
 *     host scalars (pfmm_solve, pfmm_field) synchronise that stream before returning; device
 *     outputs are then complete.  pfmm_backward returns after enqueueing its kernels.
 *   - A handle owns its device workspace (grown on demand and reused across calls), its constant
 *     tables and the state saved for pfmm_backward.  A handle is not thread safe; separate handles
 *     are independent.  No caller pointer is retained after a call returns.
 *   - Errors: every call returns a pfmm_status; pfmm_last_error(h) gives a message for the last
 *     failure on h.  On error the contents of the output buffers are unspecified, except for
 *     PFMM_ERR_NOT_CONVERGED, where all outputs hold the last iterate and *res is filled.
 */
#ifndef PFMM_H
#define PFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pfmm_status {
  PFMM_OK = 0,
  PFMM_ERR_INVALID_ARG = 1,   /* bad config, negative n or alpha, NULL where data is required    */
  PFMM_ERR_NONFINITE = 2,     /* a position, charge, polarisability or warm-start dipole is NaN/Inf */
  PFMM_ERR_COINCIDENT = 3,    /* two particles at the same position                               */
  PFMM_ERR_NOT_CONVERGED = 4, /* the dipole solve did not reach scf_tol within scf_max_iter        */
  PFMM_ERR_NOT_SPD = 5,       /* conjugate gradients met p.Ap <= 0: the dipole system is not
                                 positive definite (polarisation catastrophe)                      */
  PFMM_ERR_OOM = 6,           /* device allocation failed                                          */
  PFMM_ERR_HIP = 7,           /* a HIP runtime call failed; the message carries hipGetErrorString */
  PFMM_ERR_NO_STATE = 8       /* pfmm_backward without a preceding successful pfmm_solve          */
} pfmm_status;

typedef enum pfmm_precision {
  PFMM_FP64 = 0,   /* every field evaluation in float64.  The near-field preconditioner of the
                      dipole solve (precond_cutoff > 0) applies its product in float32 on both
                      paths: it only shapes the search directions; the field evaluations, the
                      residuals and the stopping rule stay in float64                           */
  PFMM_MIXED = 1   /* M2L and P2P in float32 with float32 accumulation; tree, P2M/M2M/L2L/L2P,
                      levels <= 3 of M2L, the dipole-solve vectors, dot products, residual norms
                      and the energy reduction stay in float64                                   */
} pfmm_precision;

enum pfmm_flags {
  PFMM_WANT_FORCES = 1u << 0,        /* compute forces (else `forces` may be NULL)                */
  PFMM_WANT_POTENTIALS = 1u << 1,    /* compute potentials (else `phi` may be NULL)               */
  PFMM_SAVE_FOR_BACKWARD = 1u << 2,  /* keep what pfmm_backward needs inside the handle          */
  PFMM_WARM_START = 1u << 3,         /* `mu` holds an initial guess on entry                      */
  PFMM_TIMING = 1u << 4              /* fill pfmm_result.t_phase_ms with HIP-event phase times    */
};

typedef struct pfmm_config {
  int order_p;         /* expansion order p, 1..12 (Sec. II.B truncation |n| + |m| <= p).  Up to
                          10 the M2L runs on the matrix cores (a tile's local expansions stay in
                          registers and its staged operands fill the LDS at C(13, 3) = 286
                          coefficients); orders 11 and 12 run a float64 vector M2L, on both
                          precision paths, several times slower per interaction                  */
  int ws;              /* well-separation parameter, 1 or 2: near field = leaves within Chebyshev
                          distance ws; M2L between children of near parents that are farther     */
  double leaf_width;   /* leaf cell edge in Angstrom; 0 = choose from the mean density            */
  int precision;       /* pfmm_precision                                                           */
  double scf_tol;      /* stop when ||alpha E(mu) - mu||_2 / ||alpha E^q||_2 <= scf_tol            */
  int scf_max_iter;    /* maximum conjugate-gradient iterations                                    */
  int graph_iters;     /* iterations captured per HIP graph launch (0 = plain launches)           */
  double thole_a;      /* Thole linear-damping constant a: s_ij = a (alpha_i alpha_j)^(1/6);
                          0 disables damping.  Applied to dipole-dipole pairs only.               */
  double coulomb_k;    /* energy scale k_e                                                         */
  unsigned flags;      /* pfmm_flags                                                               */
  int m2l_order_slack; /* -1: every M2L at order p (the plain method).  >= 0: the M2L at cell offset
                          d is truncated at the smallest order q whose error bound (sqrt(3)/|d|)^(q+1)
                          does not exceed that of the nearest offsets at order p,
                          (sqrt(3)/(ws+1))^(p+1), plus this slack, at most p (an extension: it
                          equalises the per-interaction error bound over the offsets of the list)  */
  double precond_cutoff; /* 0: conjugate gradients on the scaled system (Jacobi preconditioning).
                          > 0: flexible conjugate gradients preconditioned by precond_iters inner CG
                          iterations on (I - S T~_near S) z = r, T~_near the damped dipole tensor of
                          the pairs closer than this radius (Angstrom) in adjacent leaves.  Same
                          converged dipoles and stopping rule; fewer field evaluations.            */
  int precond_iters;   /* inner iterations of the preconditioner, 1..64                            */
  double scf_relax;    /* 0: every dipole-solve field evaluation at the configured orders.  In (0, 1):
                          once the relative residual r_k falls below scf_relax, the field evaluation
                          of the next iteration caps every M2L order at p - floor(ln(scf_relax / r_k) /
                          ln((ws + 1)^2 / 3)), at least ceil(p / 2): one order less for every factor
                          (ws + 1)^2 / 3 (3 at ws = 2, the measured growth of the field error per
                          order) by which the residual falls (an extension: relaxed matrix-vector
                          products in a Krylov solve, whose late corrections are small).  The
                          stopping rule is checked again on the final dipoles with the full orders;
                          if it fails, the solve continues once from them without the cap, and
                          returns PFMM_ERR_NOT_CONVERGED if it still fails.  On the mixed path the
                          relaxed iterations stop at scf_tol / 2, leaving room for the float32
                          rounding of their products in that final check.                         */
  double dipole_pair_dl; /* 0: the multipoles of the induced dipoles are those of point dipoles (the
                          limit of Sec. II.C).  > 0 (Angstrom, at most 1): each dipole's multipole
                          expansion is that of the pair of charges +/- |mu| / (2 dl) at x +/- dl mu/|mu|
                          of Sec. II.C (mu = 2 |q^mu| delta-l); the near field keeps the point dipoles.
                          Applies to every field evaluation with dipole sources, on both paths.  At
                          finite dl this field is not additive in the dipoles, so the solve checks
                          its stopping rule on the final dipoles and continues from them if needed
                          (at most twice; PFMM_ERR_NOT_CONVERGED if the rule still fails).        */
  int dipole_tree;     /* 0: the dipole solve uses the tree of all particles.  1: when the
                          polarisable sites (alpha > 0) are a proper subset, the dipole solve runs on
                          a tree of those sites alone (T^mu of Sec. III): its field evaluations
                          involve the sites only, while the charge field, the final pass, energy and
                          forces use the tree of all particles.  Same converged dipoles up to the
                          FMM error of each tree; the stopping rule holds for the site tree's field,
                          and pfmm_result.residual, measured with the full tree's, shows the two
                          trees' difference.  Not combined with excluded pairs
                          (PFMM_ERR_INVALID_ARG).                                                   */
  double mac_theta;    /* 0: interaction lists by the well-separation rule ws (the default).  In
                          [0.3, 1): the multipole acceptance criterion and dual tree walk of Sec. III
                          (eq. mac): two cells of one level that are not adjacent interact through
                          one M2L when theta |z_A - z_B| > r_A + r_B, with z the cell centres and r
                          the largest distance from a cell's centre to one of its particles;
                          otherwise the pairs of their children are examined, down to the leaves,
                          whose pairs that are not accepted are summed directly.  Every M2L is at
                          order p (m2l_order_slack must be -1; order_p at most 9), with the float32
                          tiles of the mixed path as for the ws lists; ws no longer shapes the lists.
                          The Thole damping radius must not exceed the leaf edge.  Below 0.3 the offsets of accepted pairs outgrow the
                          operator table (PFMM_ERR_INVALID_ARG).                                   */
  int mac_ndirect;     /* with mac_theta: a pair of cells holding fewer than this many particles
                          together is summed directly, whatever the criterion says (the paper's
                          direct interaction of small node pairs, about 64); 0 = no such rule      */
  int mac_leaf_direct; /* with mac_theta: 1 = pairs of leaves are always summed directly (the paper's
                          rule for two leaves), 0 = leaf pairs are accepted by the criterion too    */
  int adaptive_leaf_max; /* 0: every leaf at the finest level (the default).  > 0: the adaptive
                          octree, the octree form of the paper's adaptive tree whose recursion stops
                          at N_bucket particles (Sec. III): a cell above the finest level (edge
                          leaf_width) is split only when it holds more than this many particles, and
                          the tree is 2:1 balanced over the full octree, empty cells included (a
                          cell touching a split cell one level finer is split too, so touching
                          leaves differ by at most one level).  The lists come from a dual tree walk
                          over cell pairs of one level that sums two cells directly once both are
                          terminal (a leaf or below one), with the well-separation rule of ws
                          (mac_theta = 0; mac_ndirect and mac_leaf_direct unused) or the acceptance
                          criterion.  The expansions of cells below a leaf are exact translations of
                          the leaf's own and serve its interactions with finer neighbours.  The
                          M2L (order_p at most 9, float32 tiles on the mixed path) runs at the ws
                          lists' per-offset orders (m2l_order_slack), or at order p with mac_theta;
                          the Thole damping radius must not exceed ws leaf edges (leaf edges with
                          mac_theta).                                                              */
} pfmm_config;

typedef struct pfmm_result {
  double U_total, U_qq, U_pol;  /* k_e-scaled energies; U_pol in the full (variational) form      */
  int iters;                    /* conjugate-gradient iterations taken                             */
  double residual;              /* final ||alpha E(mu) - mu||_2 / ||alpha E^q||_2, recomputed from
                                   the final dipoles                                               */
  double residual_max_debye;    /* max_i |alpha_i E_i(mu) - mu_i| in Debye                         */
  int levels;                   /* leaf level L of the octree (root = level 0)                     */
  double leaf_width;            /* leaf edge actually used                                         */
  int64_t n_leaves, n_cells;    /* non-empty leaves, non-empty cells on all levels                 */
  int64_t n_m2l;                /* source-target M2L cell pairs per evaluation                     */
  int64_t n_p2p;                /* ordered near-field particle pairs per evaluation (i != j)       */
  int64_t m2l_flops;            /* useful M2L flops per evaluation: 2 C(q+6, 6) per pair of order q */
  int n_evals;                  /* FMM field evaluations performed                                 */
  double t_phase_ms[8];         /* with PFMM_TIMING: tree, charge field, dipole solve, final pass,
                                   assembly, total, -, - (after a continuation of a relaxed solve,
                                   phases 2-4 are those of its first pass)                         */
  double t_kernel_ms[8];        /* with PFMM_TIMING: summed device time per kernel class, measured
                                   with HIP events on the call's stream: P2M, M2M, M2L, L2L, L2P,
                                   P2P of the dipole solve (damped field only), P2P of the charge and
                                   final passes (all outputs), dipole-solve vector kernels          */
  int kernel_launches[8];       /* launches per kernel class counted in t_kernel_ms               */
  int64_t m2l_flops_total;      /* useful M2L flops of all field evaluations of the call, each at the
                                   orders it used                                                  */
  int m2l_order_cap_min;        /* lowest M2L order cap of the dipole solve (order_p without
                                   scf_relax)                                                      */
  int scf_restarts;             /* continuations from the final dipoles after the final check of the
                                   stopping rule (scf_relax: without the cap; dipole_pair_dl: the
                                   pair field is not additive in the dipoles; at most 1 and 2)      */
  int64_t solve_id;             /* 1, 2, ... for the successful solves on a handle (0 on failure):
                                   names the state pfmm_backward_qe may be asked for               */
  double t_m2l_split_ms[2];     /* with PFMM_TIMING: M2L device time of the launches at the full
                                   orders [0] and of the order-capped launches of a relaxed solve [1] */
  int m2l_split_launches[2];    /* the launches counted in t_m2l_split_ms                          */
  int64_t m2l_split_flops[2];   /* their useful flops (2 C(q+6, 6) per cell pair at the order q used) */
  int64_t n_sites;              /* particles in the tree of the dipole solve (n, or the polarisable
                                   sites with dipole_tree)                                         */
} pfmm_result;

typedef struct pfmm_handle pfmm_handle;

/* Fill *cfg with the defaults: p = 6, ws = 2, leaf_width = 0, FP64, scf_tol = 1e-6,
   scf_max_iter = 200, graph_iters = 4, thole_a = 2.0, coulomb_k = 332.06371,
   flags = WANT_FORCES | WANT_POTENTIALS | SAVE_FOR_BACKWARD, m2l_order_slack = -1,
   precond_cutoff = 0, precond_iters = 4, scf_relax = 0, dipole_pair_dl = 0, dipole_tree = 0,
   mac_theta = 0, mac_ndirect = 64, mac_leaf_direct = 1, adaptive_leaf_max = 0. */
void pfmm_config_default(pfmm_config* cfg);

/* Create a handle for a configuration.  Validates cfg, builds the constant operator tables of
   Sec. II.B for (p, ws) and uploads them to the current device.  *out is NULL on failure. */
pfmm_status pfmm_create(const pfmm_config* cfg, pfmm_handle** out);

/* Release the handle, its workspace and its tables.  NULL is accepted. */
void pfmm_destroy(pfmm_handle* h);

/* Full polarizable evaluation (Sec. III, three stages): charge field, dipole solve, energy and
   forces.  n >= 0; pos (n x 3), q (n), alpha (n, every entry >= 0; 0 = not polarisable) are
   read; mu (n x 3) receives the converged dipoles (and holds the initial guess with
   PFMM_WARM_START); forces (n x 3, or NULL without WANT_FORCES) receive F_i = -dU/dx_i; phi
   (n, or NULL without WANT_POTENTIALS) receives the total electrostatic potential
   k_e sum_j (q_j/r + mu_j.r/r^3) = dU/dq_i.  *res (host) receives energies and statistics.
   n = 0 and n = 1 return PFMM_OK with zero outputs. */
pfmm_status pfmm_solve(pfmm_handle* h, int64_t n, const double* pos, const double* q,
                       const double* alpha, double* mu, double* forces, double* phi,
                       pfmm_result* res, void* stream);

/* pfmm_solve with separate charges qE (n, e; device) for the static field that polarises the
   dipoles (Sec. III: the charges generating the field may differ from the Coulomb ones, and atoms
   with qE_i = 0 do not contribute to it).  U = U^qq(q) + U^pol with U^pol = sum |mu|^2/(2 alpha)
   - sum mu.E^{qE} - 1/2 sum mu.E^mu; forces F_i = q_i E^q_i + qE_i E^mu_i + (mu_i.grad)(E^{qE} +
   E^mu_damped)_i; phi receives dU/dq_i = k_e phi^q_i (the potential of the charges q alone) and
   phi_E (n, or NULL) dU/dqE_i = k_e phi^mu_i (the potential of the dipoles).  qE = NULL is
   pfmm_solve (qE = q; phi_E must then be NULL).  Non-finite qE: PFMM_ERR_NONFINITE.  The charges of
   both sets share the tree, so this costs one more charge pass. */
pfmm_status pfmm_solve_qe(pfmm_handle* h, int64_t n, const double* pos, const double* q, const double* qE,
                          const double* alpha, double* mu, double* forces, double* phi, double* phi_E,
                          pfmm_result* res, void* stream);

/* Gradients of g * U at the state saved by the last successful pfmm_solve on h (needs
   PFMM_SAVE_FOR_BACKWARD; a failed solve, pfmm_field or pfmm_set_exclusions leaves no state:
   PFMM_ERR_NO_STATE).  By stationarity of U^pol in mu (Sec. II.A), no derivative of the
   dipole solve is needed: grad_pos = -g F, grad_q = g phi, grad_alpha = g dU/dalpha with
   dU/dalpha_i = k_e (-|mu_i|^2/(2 alpha_i^2) - sum_j mu_i.(dT~_ij/ds_ij) mu_j s_ij/(6 alpha_i))
   (-|E_i|^2/2 for alpha_i = 0).  Each output is n-sized (n x 3 for positions) or NULL to skip. */
pfmm_status pfmm_backward(pfmm_handle* h, double g, double* grad_pos, double* grad_q,
                          double* grad_alpha, void* stream);

/* pfmm_backward for a named solve, also after pfmm_solve_qe.  solve_id = 0 takes the last successful
   solve; any other value must be the pfmm_result.solve_id of that solve, else PFMM_ERR_NO_STATE (the
   handle keeps the state of its last successful solve only, so a caller that runs another solve
   before the backward of the first is told instead of receiving the later system's gradients).
   grad_q = g dU/dq (the charges' own potential), grad_qE = g dU/dqE = g k_e phi^mu (n, or NULL).
   grad_qE after a solve without qE: PFMM_ERR_INVALID_ARG. */
pfmm_status pfmm_backward_qe(pfmm_handle* h, int64_t solve_id, double g, double* grad_pos, double* grad_q,
                             double* grad_qE, double* grad_alpha, void* stream);

/* Gradients of a loss L that depends on the converged dipoles, given g_mu = dL/dmu (n x 3, device,
   caller order), at the state of the named solve (solve_id as for pfmm_backward_qe; needs
   PFMM_SAVE_FOR_BACKWARD).  The dipoles solve A mu = E^q with A = diag(1/alpha) - T~ (Sec. II.A,
   dipole-moment equation); A is symmetric, so the adjoint lambda = A^-1 dL/dmu is a second solve with
   the same operator, tree, orders and preconditioner (every evaluation at the full orders) and
   dL = lambda . (dE^q + dT~ mu - d(diag(1/alpha)) mu):
     grad_pos_i   = dL/dx_i = qE_i E^lambda_i + (lambda_i . grad)(E^q + E^mu_damped)_i
                              + (mu_i . grad) E^lambda_damped,i      (qE = q without field charges)
     grad_q_i     = dL/dq_i = -phi^lambda_i (0 after pfmm_solve_qe, where q does not polarise)
     grad_qE_i    = dL/dqE_i = -phi^lambda_i (after pfmm_solve_qe only)
     grad_alpha_i = dL/dalpha_i = (dL/dmu_i + E^lambda_damped,i) . E_i + sum_j [lambda_i . dT~_ij/ds mu_j
                    + mu_i . dT~_ij/ds lambda_j] ds_ij/dalpha_i,   E = E^q + E^mu_damped
   with phi^lambda, E^lambda the potential and fields of the point dipoles lambda.  No k_e scaling
   (L is whatever the caller's loss is).  Each output n-sized (n x 3 for positions) or NULL.
   Overwrites the outputs; the saved state stays valid for pfmm_backward.  Errors as pfmm_solve for
   the adjoint solve (PFMM_ERR_NOT_CONVERGED, PFMM_ERR_NOT_SPD), PFMM_ERR_NONFINITE for non-finite
   dL/dmu. */
pfmm_status pfmm_backward_mu(pfmm_handle* h, int64_t solve_id, const double* g_mu, double* grad_pos,
                             double* grad_q, double* grad_qE, double* grad_alpha, void* stream);

/* Excluded pairs (the starred sums of Sec. II.A: bonded 1-2 and 1-3 pairs of a force field leave
   every sum: Coulomb energy, static field, dipole field, forces and gradients).  Host arrays in the
   caller's particle order, CSR form: the partners of particle i are xidx[xptr[i] .. xptr[i+1]-1];
   every pair must appear once in both of its rows, no self pairs.  They apply to every later
   pfmm_solve, pfmm_solve_qe, pfmm_backward and pfmm_field on h with this n (another n:
   PFMM_ERR_INVALID_ARG); n = 0 or xptr = NULL removes them.  The arrays are copied (synchronously);
   the caller keeps ownership.  Each evaluation takes the exact terms of the excluded pairs off what
   it summed, so a pair farther apart than the near field leaves the M2L truncation error of its
   interaction behind.  The preconditioner's near-field operator (precond_cutoff) keeps them: it
   only shapes the convergence.  Invalid lists: PFMM_ERR_INVALID_ARG, nothing changed. */
pfmm_status pfmm_set_exclusions(pfmm_handle* h, int64_t n, const int* xptr, const int* xidx);

/* One FMM field evaluation of fixed sources (Sec. II.B-II.C and the direct part of Sec. III),
   without any scaling by k_e.  Sources: charges q (n, or NULL) and point dipoles mu (n x 3, or
   NULL); alpha (n) sets the Thole radius of dipole-dipole pairs.  Outputs at every particle
   (each may be NULL): phi (n) total potential; E (n x 3) field with undamped dipole part;
   E_damped (n x 3) field with the Thole-damped dipole part; grad_E (n x 9, row-major 3 x 3,
   grad_E[a][b] = d_a E_b) gradient of E_damped. */
pfmm_status pfmm_field(pfmm_handle* h, int64_t n, const double* pos, const double* q,
                       const double* mu, const double* alpha, double* phi, double* E,
                       double* E_damped, double* grad_E, void* stream);

/* Bytes of device scratch that pfmm_field_noalloc may use (128 MiB per GPU). */
#define PFMM_SCRATCH_BYTES ((size_t)128 << 20)

/* pfmm_field for callers that cannot allocate memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid allocation): the same evaluation, arguments and results, but every
   device workspace buffer (tree, sort and scan temporaries, expansions, fields in sorted order) is
   carved from a fixed scratch array of PFMM_SCRATCH_BYTES that the library holds on each GPU it
   runs on until the process ends, and the call makes no hipMalloc, hipFree, host pinned
   allocation or allocating library call.  The handle must come from pfmm_create (which allocates
   its operator tables and a small host staging buffer).  An evaluation whose workspace would
   exceed PFMM_SCRATCH_BYTES returns PFMM_ERR_INVALID_ARG before any kernel uses the scratch.  The
   workspace is about 300 bytes per particle plus (1 + s) 8 C(p+3, 3) + 600 bytes per occupied cell
   (s <= 32 the offset splits of the M2L): a p = 6 evaluation of 40,000 particles at 3 per leaf fits,
   600,000 particles at 6 per leaf do not.  Every call on a GPU
   shares that GPU's scratch array and leaves its contents behind: calls that overlap on one GPU (two
   threads, or two streams whose work interleaves) race and must be serialised by the caller.
   pfmm_backward has no state from this call (PFMM_ERR_NO_STATE). */
pfmm_status pfmm_field_noalloc(pfmm_handle* h, int64_t n, const double* pos, const double* q,
                               const double* mu, const double* alpha, double* phi, double* E,
                               double* E_damped, double* grad_E, void* stream);

/* Static description of a status code. */
const char* pfmm_status_string(pfmm_status s);

/* Message for the last failure on h ("" if none); valid until the next call on h. */
const char* pfmm_last_error(const pfmm_handle* h);

/* Library version string. */
const char* pfmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PFMM_H */

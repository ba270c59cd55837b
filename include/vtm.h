/*
 * vtm.h -- C ABI of the MI355X (gfx950) Virtual Transmission Method library.
 *
 * The library solves the nodal-analysis system of a current-driven circuit,
 * A x = b (Section II, eq. 1), by the Virtual Transmission Method of Wei and
 * Yang (arXiv 0910.0663):
 *
 *   - wire tearing (Section V, Steps 1-4): every branch whose two nodes lie in
 *     different sub-circuits of the caller's node partition is cut at its
 *     middle, i --g-- j == i --2g-- m --2g-- j, and the middle node m is split
 *     into twins joined by a lossless line of characteristic impedance Z
 *     (level-one tearing: each line joins exactly two sub-circuits);
 *   - the iteration (Section VI, eqs. 9-14 with every line delay equal to one
 *     sweep): each sweep, every sub-circuit solves its own system, in which a
 *     line appears as its admittance W = 1/Z plus an incident-wave source; each
 *     line then carries the outgoing wave W u - i of one twin to the other twin
 *     for the next sweep.  Boundary variables start at zero.
 *
 * Convergence for SPD A and SPD Z is Theorem 1 (Section VII); its limit is the
 * solution of the untorn system (Appendix).
 *
 * Memory: matrices and partitions are HOST pointers and are copied; right-hand
 * sides, solutions and gradients are DEVICE pointers (HIP, the device current
 * when vtm_setup ran).  Multi-column vectors are column-major [nrhs][n]:
 * element (node i, column r) is at r*n + i.  All work runs on the stream given
 * to vtm_setup.  No exception crosses the ABI; every call returns a status and
 * vtm_last_error() gives a message for the calling thread.  One handle must
 * not be used by two host threads at once.
 */
#ifndef VTM_H
#define VTM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VTM_OK = 0,
    VTM_E_ARG = 1,          /* malformed input (sizes, ranges, NaN, labels)          */
    VTM_E_UNTEARABLE = 2,   /* a cross-partition coupling is not A_ij == A_ji < 0    */
    VTM_E_SINGULAR = 3,     /* a sub-circuit matrix (with its line admittances) is singular */
    VTM_E_DIVERGED = 4,     /* residual non-finite or above opt.divergence           */
    VTM_E_MAXITER = 5,      /* opt.max_sweeps reached without convergence            */
    VTM_E_HIP = 6,          /* HIP runtime error                                     */
    VTM_E_OOM = 7,          /* device, pinned-host or host memory allocation failed  */
    VTM_E_UNSUPPORTED = 8   /* valid input outside the library's limits             */
} vtm_status;

typedef enum {
    VTM_FP64 = 0,           /* FP64 local inverses, waves and sweeps                 */
    VTM_FP32_REFINE = 1,    /* FP32 inverses and sweeps inside FP64 refinement       */
    VTM_BF16_REFINE = 2     /* BF16 inverses (MFMA, FP32 accumulate) inside FP64 refinement */
} vtm_precision;

/* Sparse matrix, compressed rows, host memory, FP64.  Any row order; column
 * indices need not be sorted; duplicate entries are summed. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t *rowptr;  /* n + 1 */
    const int32_t *col;     /* nnz   */
    const double *val;      /* nnz   */
} vtm_csr;

typedef struct {
    int32_t precision;      /* vtm_precision                                         */
    int32_t nrhs_max;       /* widest solve this handle will run (sizes work space).
                               FP64 handles with nrhs_max >= 16 store the inverses
                               as MFMA tiles (batched sweeps) when a 16-column block
                               of the largest sub-circuit fits the sweep's LDS
                               staging (up to ~1,100 nodes), else the column-group
                               layout; BF16 handles always use tiles (at most 64
                               right-hand sides, VTM_E_UNSUPPORTED when the
                               largest sub-circuit does not fit)                 */
    int32_t check_every;    /* sweeps between FP64 residual checks (>= 1)            */
    int32_t max_outer;      /* refinement: most outer corrections                    */
    int64_t max_sweeps;     /* per plain solve, or per inner solve when refining     */
    double divergence;      /* a relative residual above this means divergence       */
    double inner_drop;      /* refinement: inner target ||r - A d|| / ||r||; 0 = default
                               (1e-5 for FP32, 1e-2 for BF16)                        */
    int32_t use_graph;      /* 1: each check interval (its sweeps, the FP64 residual
                               and the copy of its sums to the host) is captured once
                               per shape and replayed as one hipGraph launch; check
                               intervals are then check_every times a power of two */
    int32_t timing;         /* 1: HIP events around every sweep launch (report);
                               2: events around full sweeps and around each run of
                               consecutive port-to-port sweeps (their average then
                               includes the gaps between launches; the events
                               themselves perturb the run far less than 1 does).
                               Not available with use_graph.                      */
    int32_t adaptive_checks;/* 1: once the residual falls steadily, skip checks that
                               cannot reach tol: the next check comes after half the
                               predicted remaining sweeps (a multiple of check_every,
                               at most 64 of them); 0: check every check_every      */
    int32_t batch_row_tiles;/* batched (MFMA) sweep: 16-row tiles each wavefront holds
                               per pass, 3 or 5; 0 = chosen by the autotuner at setup
                               (which also tries 1: fewer registers, more wavefronts;
                               its choice is kept for the process and reused by later
                               setups on the same device with the same precision,
                               right-hand sides, shape options and plan sizes)   */
    int32_t batch_rhs_block;/* batched sweep: right-hand sides per workgroup, 16, 32,
                               48 or 64; 0 = chosen by the autotuner at setup        */
    int32_t local_form;     /* 0: every sweep applies the full local inverse.
                               1: port-to-port form (the interface-only iteration of
                               the Appendix, eqs. 23-26): the waves leaving a
                               sub-circuit are an affine function of those arriving,
                               with h = beta K^-1 b at the ports from a first full
                               sweep, so later sweeps stream only an operator between
                               ports.  The smallest that applies is used: the upper
                               triangle of K^-1 over the port nodes, packed (A
                               symmetric, <= 64 port nodes and ports per sub-circuit);
                               K^-1 over the port nodes (k x k, when smaller than
                               q x q; the adjoint of an unsymmetric A uses its
                               transpose); else M = diag(beta) K^-1[ports, ports]
                               diag(c) + diag(gamma).  Handles with MFMA tiles use M in
                               tile order for all right-hand sides.  Residual checks
                               use the port quantities alone (a local solve meets
                               every interior row, so b - A x lives on the port
                               nodes); once that residual passes, and at the end, x
                               is rebuilt by a full sweep from the same waves and the
                               residual on A decides.  Resumed solves run the full
                               form.  2: as 1 with M always.                        */
} vtm_options;

typedef struct {
    int64_t sweeps;         /* sweeps run (summed over inner solves when refining)   */
    int32_t outer;          /* refinement corrections applied (0 for VTM_FP64)       */
    int32_t checks;         /* residual checks run                                   */
    double relres_max;      /* final max over columns of ||b - A x|| / ||b||         */
    double solve_ms;        /* wall time of the call                                 */
    double sweep_kernel_ms; /* opt.timing: summed duration of the sweep launches     */
    int64_t sweep_launches; /* opt.timing: number of sweep launches timed            */
    int32_t batch_row_tiles;/* batched sweep shape in use (0 when not batched)       */
    int32_t batch_rhs_block;
    double pp_kernel_ms;    /* opt.timing: summed duration of the port-to-port sweeps */
    int64_t pp_launches;    /* opt.timing: number of port-to-port sweeps timed       */
    int32_t pp_shape[3];    /* batched port-to-port sweep shape in use: 16-row tiles
                               per wavefront pass, right-hand sides per workgroup,
                               wavefronts per workgroup (zeros when not batched)     */
    double *relres;         /* optional caller array [nrhs]: final per-column value  */
    /* Residual history.  A plain (FP64) solve records every residual check: the
       check of x = 0 before any sweep, each check after a run of sweeps (from port
       quantities in the port-to-port form, the same residual of the same iterate),
       and the check on A after the sweep that rebuilds x.  A refining solve records
       the FP64 residual ||b - A x|| / ||b|| at each outer step, before each
       correction and the final one.  Each entry is the maximum over the columns. */
    double *history;        /* optional caller array [history_cap]                   */
    int64_t *history_sweeps;/* optional caller array [history_cap]: sweeps run by that
                               entry (inner sweeps summed when refining)             */
    int32_t history_cap;    /* entries the caller's arrays hold (0: none written)    */
    int32_t history_len;    /* out: entries written, min(history_total, history_cap) */
    int32_t history_total;  /* out: entries the solve produced                       */
} vtm_report;

typedef struct vtm_handle_s *vtm_handle;

/* Fills *opt with defaults: FP64, nrhs_max 1, check_every 8, max_outer 30,
 * max_sweeps 1000000, divergence 1e6, inner_drop 0, use_graph 0, timing 0,
 * adaptive_checks 1, batch_row_tiles 0, batch_rhs_block 0, local_form 1. */
void vtm_default_options(vtm_options *opt);

/*
 * vtm_setup -- tear A along the partition and factor every sub-circuit.
 *
 * Defines the operation of Section V (Steps 1-4, eqs. 6-8) and the local
 * systems of Section VI (eq. 11: the C + W block).
 *
 *   A       host CSR of the untorn system, n x n.
 *   part    host int32[n]: sub-circuit of every node, labels 0..S-1, each used.
 *   Z       host: nZ == 1 -> one impedance (ohm, > 0) for every cut wire;
 *           nZ == number of cut wires -> one per wire, wires in canonical order
 *           (lower node ascending, then upper node ascending).
 *   opt     options (NULL = defaults).
 *   stream  hipStream_t for all later work (NULL = the null stream).
 *   out     receives the handle; the handle owns every device buffer.
 *
 * Every pair (i, j) in different sub-circuits with a nonzero entry must have
 * A_ij == A_ji < 0 (a two-terminal conductance g = -A_ij), else
 * VTM_E_UNTEARABLE.  Sub-circuits may not exceed 16384 nodes
 * (VTM_E_UNSUPPORTED), nor a device's LDS per workgroup in right-hand-side
 * values (8 bytes each in FP64, 4 otherwise; 160 KiB on gfx950 holds the
 * largest).  n and nnz must fit int32.  A sub-circuit matrix
 * (with its port conductances) whose elimination meets an exactly zero or
 * non-finite pivot gives VTM_E_SINGULAR.  Returns after the setup kernels
 * finish.
 */
vtm_status vtm_setup(const vtm_csr *A, const int32_t *part, const double *Z, int64_t nZ,
                     const vtm_options *opt, void *stream, vtm_handle *out);

/*
 * vtm_setup_vertex -- level-one wire tearing at interfacial nodes (Section V,
 * Steps 1-4; Fig. 4): every interfacial node is split into a pair of twins,
 * one in each of the two sub-circuits it borders, joined by a virtual line of
 * admittance W.  The twins are unknowns of their sub-circuits; the line is a
 * port with W on the twin's diagonal, incident current a, and outgoing wave
 * 2 W u_twin - a (Section VI).
 *
 *   A       host CSR of the untorn system, n x n (duplicates summed).
 *   label   host int32[n]: sub-circuit of every inner node (entries of
 *           interfacial nodes are ignored).
 *   iface   host int32[n_iface]: the interfacial nodes (Step 1), distinct.
 *   sides   host int32[n_iface][2]: the two distinct sub-circuits each
 *           interfacial node borders; the twin in sides[l][0] keeps the node's
 *           id, the other is a new node.  Labels 0..S-1, each used.
 *   W       host: nW == 1 -> one line admittance (S, > 0) for every line;
 *           nW == n_iface -> one per interfacial node, in iface order.
 *   opt, stream, out   as for vtm_setup.
 *
 * Step 3 (what moves to which twin), read from the example of Section IX: a
 * two-terminal branch (A_vw == A_wv < 0) from interfacial node v to an inner
 * node w joins w to the twin of v on w's side, conductance and all; a
 * one-sided entry (a controlled source) between v and an inner node w also
 * goes to the twin on w's side; the rest of A_vv (ground), the source b_v and
 * branches between two interfacial nodes of the same two sub-circuits are
 * split in equal halves.  An inner node coupled to an interfacial node of
 * sub-circuits it does not belong to, any coupling between inner nodes of
 * different sub-circuits, or two coupled interfacial nodes that border
 * different pairs of sub-circuits give VTM_E_UNTEARABLE.  Other limits and
 * errors as for vtm_setup, on the torn system of n + n_iface nodes.
 *
 * vtm_solve takes and returns vectors over the caller's n nodes; the value of
 * an interfacial node is the mean of its twins (equal at the fixed point), and
 * the stop rule is the residual on the caller's A.  Interim checks always use
 * that residual (the port identity of the wire-cut form does not apply).
 * vtm_solve_adjoint solves A^T lambda = g with the same tear: the split rule
 * treats A_vw and A_wv alike, so the torn A^T is the transposed torn A and the
 * stored inverses are read transposed (residual on the caller's A^T).
 * vtm_get_waves / vtm_set_waves address ports 2l (twin in sides[l][0]) and
 * 2l+1; vtm_info reports the torn system's size.
 */
vtm_status vtm_setup_vertex(const vtm_csr *A, const int32_t *label, const int32_t *iface,
                            const int32_t *sides, int64_t n_iface, const double *W, int64_t nW,
                            const vtm_options *opt, void *stream, vtm_handle *out);

/*
 * vtm_setup_vertex_coupled -- as vtm_setup_vertex, with coupled lines: one
 * characteristic admittance matrix W over the interfacial nodes (eqs. 4-5;
 * the overlapped-block rules of Section VIII give such a W).
 *
 *   W   host CSR, n_iface x n_iface, in iface order (duplicates summed):
 *       symmetric, positive diagonal; W_lm != 0 (l != m) only where iface[l]
 *       and iface[m] border the same two sub-circuits in the same order
 *       (sides[l] == sides[m]), else VTM_E_ARG.  W should be positive
 *       definite (the paper's requirement for resistor networks); it is not
 *       checked, an indefinite W may make a sub-circuit singular or the
 *       iteration diverge.
 *
 * W joins the twins of each side inside their sub-circuit (its block is added
 * to the sub-circuit matrix), and the outgoing waves of a sub-circuit are
 * 2 W u_twins - a (the oracle's coupled-line sweep).  The port-to-port form is
 * the dense one (local_form 1 and 2 alike); the packed and port-node forms
 * need diagonal lines.  Everything else as for vtm_setup_vertex.
 */
vtm_status vtm_setup_vertex_coupled(const vtm_csr *A, const int32_t *label, const int32_t *iface,
                                    const int32_t *sides, int64_t n_iface, const vtm_csr *W,
                                    const vtm_options *opt, void *stream, vtm_handle *out);

/*
 * vtm_vertex_admittance -- host-only: W for tearing at interfacial nodes under
 * a rule of Section VIII, as an n_iface x n_iface CSR in iface order for
 * vtm_setup_vertex_coupled.  C is the interface block of one side of the
 * torn system (vtm_split_vertex): the entries between the twins that lie in
 * sides[l][side] (the paper's C_1 for side 0, C_2 for side 1), symmetrized
 * as (C + C^T) / 2 (C itself when A is symmetric).
 *   kind  VTM_W_SCALED_MEAN: alpha * (mean conductance of A's branches) * I;
 *         VTM_W_IDENTITY: alpha I;  VTM_W_DIAG: diag(C);  VTM_W_OB: C;
 *         VTM_W_WOB: alpha C.
 *   nnz, rowptr [n_iface + 1], col [nnz], val [nnz]: outputs, caller-owned,
 *         NULLs skipped (call once with NULL arrays for nnz); columns sorted.
 * Errors: VTM_E_ARG (alpha <= 0, bad kind or side, a non-positive diagonal of
 * C), the tearing errors of vtm_setup_vertex.
 */
vtm_status vtm_vertex_admittance(const vtm_csr *A, const int32_t *label, const int32_t *iface,
                                 const int32_t *sides, int64_t n_iface, int32_t kind, double alpha,
                                 int32_t side, int64_t *nnz, int64_t *rowptr, int32_t *col, double *val);

/*
 * vtm_vertex_sca -- host-only: rule 5 of Section VIII, the Schur complement
 * approximation W = C - E~ D~^-1 F~ (the partial input admittance of one side),
 * for vtm_setup_vertex_coupled.  Lines are grouped by the ordered pair of
 * sub-circuits their twins lie in; per group, C, E~, F~, D~ are blocks of the
 * torn system (vtm_split_vertex) over the group's twins on `side` (sides[l][0]
 * for 0, sides[l][1] for 1) and D~ over the inner nodes of that sub-circuit
 * within `depth` hops of those twins in the torn matrix's graph (depth < 0:
 * every inner node, the exact Schur complement of Example 3; 0: W = C).  The
 * result is symmetrized, (S + S^T) / 2, and an off-diagonal entry is dropped
 * when |w_ij| < drop * sqrt(|w_ii w_jj|) (the paper drops small elements so
 * that W keeps a pattern like C's; drop = 0 keeps every entry).  D~ is solved
 * densely on the host (cost ~ m^3 for m chosen nodes per group).
 *   nnz, rowptr [n_iface + 1], col [nnz], val [nnz]: outputs as for
 *   vtm_vertex_admittance.
 * Errors: VTM_E_ARG (bad side, drop < 0), VTM_E_SINGULAR (D~ singular), the
 * tearing errors of vtm_setup_vertex.
 */
vtm_status vtm_vertex_sca(const vtm_csr *A, const int32_t *label, const int32_t *iface, const int32_t *sides,
                          int64_t n_iface, int32_t side, int32_t depth, double drop, int64_t *nnz,
                          int64_t *rowptr, int32_t *col, double *val);

/*
 * vtm_solve -- run VTM sweeps (Section VI, eqs. 11 and 14) from zero boundary
 * variables until every column has ||b - A x||_2 / ||b||_2 <= tol, the
 * residual taken on the untorn A in FP64 every opt.check_every sweeps.
 *
 *   b, x    device FP64 [nrhs][n] (column-major), original node order; x is
 *           written (the last iterate also on DIVERGED / MAXITER).
 *   nrhs    1 .. opt.nrhs_max.
 *   tol     > 0.
 *   rep     optional report.
 *
 * A zero column converges at once with x = 0.  With a refining precision the
 * sweeps run in FP32/BF16 on A d = r and x += d, r = b - A x in FP64, until
 * the FP64 residual meets tol (VTM_E_MAXITER after opt.max_outer).  Each inner
 * solve starts from zero waves and stops when ||r - A d|| / ||r|| falls below
 * max(inner_drop, tol * ||b|| / (2 ||r||)) for every column, or when two
 * checks in a row bring no column 20% below its best (the low-precision
 * inverse bounds how far an inner solve can go).
 */
vtm_status vtm_solve(vtm_handle h, const double *b, double *x, int32_t nrhs, double tol,
                     vtm_report *rep);

/*
 * vtm_solve_adjoint -- solve A^T lambda = g by the same iteration on the torn
 * A^T, reusing the stored sub-circuit inverses read transposed (valid because
 * every cut coupling is symmetric, so the torn A^T is the transposed torn A).
 * Handles whose inverses are MFMA tiles (batched) use the same tiles when A is
 * symmetric and a transposed copy made at setup otherwise (then every sweep of
 * the adjoint is a full sweep).  Same conventions and errors as vtm_solve.
 */
vtm_status vtm_solve_adjoint(vtm_handle h, const double *g, double *lambda, int32_t nrhs,
                             double tol, vtm_report *rep);

/*
 * vtm_solve_noalloc -- vtm_solve for callers that cannot allocate device
 * memory or create runtime objects during a solve (code under HIP graph
 * capture elsewhere in the process, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as vtm_solve; the same
 * kernels run in the same order, so x and the report are bitwise those of
 * vtm_solve.  The residual reductions keep their partial sums in a static
 * device workspace of the library (4 MiB per device, held until the process
 * ends) instead of the handle's buffers; the call makes no hipMalloc, hipFree,
 * event, stream or graph.  Every check writes all of the workspace it reads,
 * so a call does not depend on what an earlier call left there.
 *
 *   nrhs   1 .. min(opt.nrhs_max, 64); above 64: VTM_E_UNSUPPORTED.
 *   The handle must have opt.use_graph == 0 and opt.timing == 0, else
 *   VTM_E_UNSUPPORTED.
 *
 * All calls on one device share its workspace: two vtm_solve_noalloc calls
 * that overlap in time on one device (from two host threads) race and give
 * wrong results.  Calls run one after the other are safe; the call returns
 * only after its work has finished.
 */
vtm_status vtm_solve_noalloc(vtm_handle h, const double *b, double *x, int32_t nrhs, double tol,
                             vtm_report *rep);

/*
 * vtm_grad -- derivatives of a loss L(x) through A x = b, from x and the
 * adjoint solution lambda of A^T lambda = dL/dx (vtm_solve_adjoint):
 *     dL_dg[e] = - sum_r (lambda_i - lambda_j)(x_i - x_j)  for branch e = (i, j)
 *                (a conductance g stamps +g on A_ii, A_jj and -g on A_ij, A_ji);
 *     dL_dA[k] = - sum_r lambda_row(k) x_col(k)             for entry k of A,
 *                e.g. a controlled-source gain, a single entry of A (the
 *                op-amp example of Section IX, eq. 15).
 * (dL/db = lambda needs no call.)
 *
 *   x, lambda      device FP64 [nrhs][n] (the caller's node order).
 *   branch_ij      device int32 [m][2] (pairs i, j; original node ids); a pair
 *                  naming a node outside [0, n) yields NaN for that branch.
 *                  m may be 0 (then branch_ij and dL_dg may be NULL).
 *   dL_dg          device FP64 [m], overwritten.
 *   dL_dA_or_null  device FP64 [nnz] or NULL: entry k of the CSR arrays of the A
 *                  passed to vtm_setup / vtm_setup_vertex (the caller's order,
 *                  duplicates each get the derivative of their sum), overwritten.
 */
vtm_status vtm_grad(vtm_handle h, const double *x, const double *lambda, int32_t nrhs,
                    const int32_t *branch_ij, int64_t m, double *dL_dg, double *dL_dA_or_null);

/*
 * vtm_refresh -- new values of A (and optionally new line impedances) on the
 * pattern and partition a vtm_setup handle was built with: the setup of
 * Section VI (the sub-circuit matrices with their port conductances, eq. 11,
 * their inverses and the port-to-port operators) is redone on the device
 * without planning the tear again.  For loops that re-solve after changing
 * conductances (power-grid sizing).  The handle then behaves exactly as one
 * freshly set up with the new values: the same kernels on the same layout,
 * bitwise the same results.
 *
 *   val   host FP64 [nnz]: new values for the CSR arrays given to vtm_setup
 *         (same rowptr and col, same entry order).
 *   Z     host, nullable: nZ == 1 or the number of cut wires as for vtm_setup;
 *         NULL (or nZ == 0) keeps the current line impedances.
 *
 * The off-diagonal entries that are zero must stay the same (a different
 * sparsity pattern is VTM_E_ARG), as must the symmetry of A
 * (VTM_E_UNSUPPORTED), and every cut coupling must remain A_ij == A_ji < 0
 * (VTM_E_UNTEARABLE); the handle is unchanged after these errors.  Handles of
 * vtm_setup_vertex[_coupled] give VTM_E_UNSUPPORTED.  A sub-circuit that becomes
 * singular gives VTM_E_SINGULAR, after which the handle must be refreshed
 * again or destroyed.  Stored waves (vtm_set_waves) are discarded.  Returns
 * after the device work finishes.
 */
vtm_status vtm_refresh(vtm_handle h, const double *val, const double *Z, int64_t nZ);

/*
 * Checkpoint / resume of the iteration state: the incident wave at every port
 * (two ports per cut wire: port 2e on the lower node of wire e, 2e+1 on the
 * upper), device FP64 [nrhs][2 * n_wires].  vtm_get_waves gives the waves of
 * the last sweep; vtm_set_waves makes the next vtm_solve start from these
 * waves instead of zero.  FP64 handles only: a refining handle's iteration
 * state is its FP64 solution together with the waves of an inner solve of a
 * correction equation, which no wave vector alone resumes, so both calls give
 * VTM_E_UNSUPPORTED there.
 */
vtm_status vtm_get_waves(vtm_handle h, double *waves, int32_t nrhs);
vtm_status vtm_set_waves(vtm_handle h, const double *waves, int32_t nrhs);

/* Sizes of a handle: nodes, sub-circuits, cut wires, bytes of the stored
 * inverses and of the port-to-port operators as allocated (0 when not built),
 * and the algorithmic bytes one port-to-port sweep moves (operator entries once,
 * without layout padding; per port the
 * incident wave, h, c when packed, the outgoing wave and the twin index; per
 * port node and sub-circuit their offsets).  NULLs skipped.  For symmetric A
 * the operator is the packed upper triangle of K^-1 over a sub-circuit's port
 * nodes (beta = 2 W c and gamma = 1 - 2 c are then formed on the fly). */
vtm_status vtm_info(vtm_handle h, int64_t *n, int64_t *n_sub, int64_t *n_wires,
                    int64_t *inverse_bytes, int64_t *port_operator_bytes, int64_t *port_sweep_bytes);

void vtm_destroy(vtm_handle h);
const char *vtm_status_str(vtm_status s);
const char *vtm_last_error(void);

/* Line admittance rules for vtm_line_admittance and vtm_vertex_admittance
 * (the preconditioners of Section VIII).  With the cut-wire tearing of
 * vtm_setup each cut wire's interfacial node is its midpoint m (a branch g
 * becomes 2g + 2g through m); the two twins of m are not coupled to any other
 * interface node, so the interface block C of either side is diagonal with
 * the twin's 2g, and every rule below gives one W per wire (DIAG = OB there).
 * Tearing at interfacial nodes gives a C with off-diagonal entries (branches
 * between interfacial nodes), hence coupled lines for OB and WOB.  Rule 5,
 * the Schur-complement approximation, is vtm_vertex_sca (tearing at nodes). */
typedef enum {
    VTM_W_SCALED_MEAN = 0,  /* W_e = alpha * mean conductance of A's branches      */
    VTM_W_IDENTITY = 1,     /* W = alpha I (rule 1), alpha in siemens               */
    VTM_W_OB = 2,           /* W = C, the overlapped block (rule 3): W_e = 2 g_e;
                               the diagonal rule (2) gives the same here          */
    VTM_W_WOB = 3,          /* W = alpha C, weighted overlapped block (rule 4)       */
    VTM_W_DIAG = 4          /* W = diag(C), the diagonal preconditioner (rule 2)      */
} vtm_admittance_rule;

/*
 * vtm_line_admittance -- host-only: the characteristic admittance W_e of every
 * cut wire of the partition under one of the rules of Section VIII, in the
 * canonical wire order of vtm_setup (pass Z_e = 1 / W_e with nZ = n_wires).
 * A and part as for vtm_setup (host); W: host double[n_wires], caller-owned;
 * n_wires must equal the partition's cut-wire count (vtm_plan).  "Branches"
 * of A are its symmetric negative off-diagonal pairs.  Errors: VTM_E_ARG (bad
 * rule, alpha <= 0, count mismatch), the vtm_setup tearing errors.
 */
vtm_status vtm_line_admittance(const vtm_csr *A, const int32_t *part, int32_t kind, double alpha, double *W,
                               int64_t n_wires);

/*
 * vtm_split_vertex -- host-only: the system torn at interfacial nodes as
 * vtm_setup_vertex builds it (Section V, Steps 2-3), before any renumbering
 * and without the lines of Step 4.  Node i < n keeps its id (for an
 * interfacial node that is its twin in sides[l][0]); node n + l is the twin of
 * iface[l] in sides[l][1].  The torn right-hand side is b_i for inner nodes
 * and b_v / 2 for each twin of v.  Call once with NULL arrays for the sizes.
 *   n_torn   n + n_iface;  nnz  entries of the torn matrix.
 *   rowptr   int64 [n_torn + 1], col int32 [nnz], val double [nnz]: the torn
 *            matrix (CSR; duplicates possible, to be summed).
 *   part     int32 [n_torn]: sub-circuit of every torn node.
 * Errors: those of vtm_setup_vertex's tearing.
 */
vtm_status vtm_split_vertex(const vtm_csr *A, const int32_t *label, const int32_t *iface,
                            const int32_t *sides, int64_t n_iface, int64_t *n_torn, int64_t *nnz,
                            int64_t *rowptr, int32_t *col, double *val, int32_t *part);

/*
 * vtm_plan -- host-only tearing plan (no device work), for inspection and tests.
 * Runs the same planner as vtm_setup.  Outputs may be NULL.
 *   n_sub, n_wires       counts.
 *   wires     int32 [n_wires][2]  cut wires (i < j), canonical order.
 *   coef      double [n_wires][4] per wire: G = 2gW/(2g+W) (port conductance),
 *             c = 2g/(2g+W) (wave-to-source gain), beta = 4gW/(2g+W) and
 *             gamma = (W-2g)/(2g+W) (outgoing wave = beta*u + gamma*a).
 */
vtm_status vtm_plan(const vtm_csr *A, const int32_t *part, const double *Z, int64_t nZ,
                    int64_t *n_sub, int64_t *n_wires, int32_t *wires, double *coef);

#ifdef __cplusplus
}
#endif
#endif /* VTM_H */

/*
 * hfx.h -- plane-wave Gamma-point Hartree-Fock exact exchange on MI355X (gfx950).
 *
 * The operations follow the exact-exchange definitions of the Methods
 * section ("MTACE Method for H-AIMD Simulation") of Kar, Mandal, Thakkur,
 * Meyer, Nair, "Speeding-up Hybrid Functional based Ab Initio Molecular
 * Dynamics using Multiple Time-stepping and Resonance Free Thermostat":
 *
 *   Eq. (vx)   V_X psi_i = - sum_j v_ij(r) psi_j,          i = 1..N_orb
 *   Eq. (vij)  v_ij(r)   = <psi_j | 1/r12 | psi_i>  (Coulomb potential of the
 *                          pair density psi_i psi_j)
 *   Eq. (HFX)  exact-exchange energy (prefactor convention below)
 *   M_kl = <psi_k | V_X | psi_l>, the matrix whose Cholesky factor builds the
 *          ACE operator (same subsection).
 *
 * Conventions (the paper leaves them open; these are this library's):
 *   - Orbitals are real (Gamma point), float64, layout [orb][z][y][x] with x
 *     fastest, on a cubic n x n x n grid in an orthorhombic box L[0..2]
 *     (bohr).  dV = Lx Ly Lz / n^3 and <f|g> = dV sum f g.
 *   - Periodic Coulomb kernel v(G): HFX_KERNEL_TRUNCATED uses
 *     4 pi / G^2 (1 - cos(G Rc)), v(0) = 2 pi Rc^2, Rc = (3 Omega / 4 pi)^(1/3);
 *     HFX_KERNEL_ERFC uses 4 pi / G^2 (1 - exp(-G^2 / 4 w^2)), v(0) = pi / w^2
 *     with w = hfx_system.param (bohr^-1).
 *   - K psi_i = V_X psi_i; E_x = 1/2 sum_i <psi_i | K psi_i> = -1/2 sum_ij e_ij
 *     with e_ij = <psi_i psi_j | v_ij> >= 0, i.e. half of the paper's
 *     closed-shell sum in Eq. (HFX).  No hybrid mixing fraction is applied.
 *     dE_x / dpsi_i(r) = 2 dV (K psi_i)(r).
 *   - The functional is evaluated for the orbitals as given; they need not be
 *     orthonormal.
 *
 * Memory: every pointer argument is a DEVICE pointer unless its name ends in
 * _host.  The caller allocates and owns every buffer, including the
 * workspace; a plan owns only its own small device tables (kernel values,
 * twiddles, tile descriptors).  Systems of a batched plan are concatenated
 * in plan order in psi, kpsi, ex and m.
 *
 * Streams: work is enqueued asynchronously on `stream` (a hipStream_t, NULL
 * for the default stream); no call synchronises the device except
 * hfx_plan_create and hfx_plan_destroy.  A plan with several systems forks
 * them onto its own streams (default priority) after an event recorded on
 * `stream` and joins them back before returning, so they overlap on the GPU
 * while the caller sees ordinary stream order.  Calls on one plan share the
 * plan's side streams, events and workspace layout: issue them from one host
 * thread at a time and, when they go to different streams, order those
 * streams so the calls do not overlap on the device (one workspace each is not
 * enough: the side streams and events are per plan).  Separate plans are
 * independent.
 *
 * Errors: status codes only.  Arguments are validated before any HIP call;
 * HIP failures map to HFX_EDEVICE.  hfx_last_error() returns a thread-local
 * description of the most recent failure.
 */
#ifndef HFX_H
#define HFX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HFX_OK = 0,
  HFX_EINVAL = 1,       /* invalid argument (null pointer, size, shape)      */
  HFX_EUNSUPPORTED = 2, /* valid but not supported (grid size, non-cubic)    */
  HFX_ENOMEM = 3,       /* workspace too small, or device allocation failed */
  HFX_EDEVICE = 4       /* a HIP runtime call failed                        */
} hfx_status;

typedef enum { HFX_KERNEL_TRUNCATED = 0, HFX_KERNEL_ERFC = 1 } hfx_kernel;
typedef enum { HFX_FP32 = 0, HFX_FP64 = 1 } hfx_precision;
typedef enum { HFX_ORTHO_LOWDIN = 0, HFX_ORTHO_CHOLESKY = 1 } hfx_ortho_method;

/* One periodic system. */
typedef struct {
  int n[3];      /* grid points along x, y, z; n_x == n_y (n_z: see below) */
  double L[3];   /* box lengths along x, y, z, bohr; each > 0               */
  int n_orb;     /* number of occupied real orbitals, >= 1                   */
  int kernel;    /* hfx_kernel                                              */
  double param;  /* erfc screening w (bohr^-1) > 0; ignored for truncated   */
} hfx_system;

typedef struct hfx_plan_t* hfx_plan;

/*
 * Create a plan for n_sys systems at the given precision (hfx_precision).
 * Supported grids: n x n x n with n in {24, 64, 72, 80, 96, 108, 120, 128},
 * and the slab-cell grids n x n x nz with (n, nz) in {(24, 48), (64, 128)}
 * (x and y transforms of length n, z transforms of length nz; layout
 * [z][y][x]; the box may be orthorhombic in either case).  `options` is a
 * nullable "key=value;key=value" string: tiles=<k> caps the orbital tiles per
 * batch; maxws=<bytes> caps the workspace; variant=<name> picks a compiled
 * kernel configuration (see hfx_variants); streams=2 runs consecutive batches
 * alternately on the call's stream and on a stream the plan owns, with a second
 * pair-grid buffer in the workspace (results are bitwise those of streams=1,
 * the default; graphs captured from such a plan run the batches on one
 * stream); shard=<g>/<R> restricts the plan to the tile rounds r with
 * r % R == g, one of R virtual groups of the pair list (the way the pairs
 * would be dealt over R GPUs): K psi, E_x, M and the gradient are then that
 * group's partial sums, which add up over g = 0..R-1 to the full result (the
 * G = 0 energy of the pair means is added by group 0); rows=<R>, R in
 * {8, 16, 24, 32}, sets the rows of a tile pair (R orbitals x the 8-orbital
 * column tile): more rows read psi and update K psi of the column tile once
 * per R pairs instead of once per 8 (default 32 for systems of at least 256
 * orbitals, else 16; clamped to 8 for variants that stage the row orbitals
 * in LDS; screened schedules use the same tile pairs with masks of the kept
 * pairs; results agree to rounding, not bitwise, across R); ecut=<Ha>
 * declares that every orbital lies in the plane-wave sphere (1/2)|G|^2 <=
 * ecut (true of plane-wave orbitals of that cutoff, and kept by linear
 * combinations such as orthonormalisation): pair densities then vanish on the
 * kz planes with |kz| > 2 floor(sqrt(2 ecut) L_z / 2 pi), which the passes
 * skip, and, in float32 plans, where the band fits in half the grid along z
 * (and along x and y on cubic grids), the first pass transforms only the
 * even z points and rows and the plane pass only the band's columns
 * (results agree with the full transform to rounding; orbitals outside the
 * sphere give wrong results, which check=1 detects); check=1 (or the
 * environment variable HFX_CHECK_INPUTS=1) makes the energy, K psi, matrix
 * and gradient calls check psi first and return HFX_EINVAL, launching
 * nothing else, when an orbital holds a non-finite value or, in a plan with
 * ecut=, has more than 1e-12 of its power beyond the band |m| <=
 * floor(sqrt(2 ecut) L / 2 pi) along z, y or x, which the skipped planes,
 * the half-length z transform, the plane pass's band columns and its
 * half-height input rely on (direct transforms of every orbital line along
 * each axis in float64; the call then waits for its stream; skipped under
 * graph capture); mix=<a>,
 * 0 < a <= 1,
 * is a hybrid functional's exact-exchange fraction: the kernel is scaled by a,
 * so E_x, K psi, M, the gradient and the ACE operator are a times the full
 * exchange (default 1).  Open-shell systems are two systems of one plan, the
 * spin-up and the spin-down orbitals on the same box: pairs never mix spins,
 * and the total exchange energy is the sum of the two E_x.  The environment
 * variable HFX_MAX_WORKSPACE_BYTES also caps the workspace.  variant=, tiles=
 * and rows= take either one value for every system or a ','-separated list
 * with one value per system (variant names are checked against each
 * system's grid).  tune_cache=<path> (or the environment variable
 * HFX_AUTOTUNE_CACHE) names a cache written by hfx_autotune: each system
 * whose key is found there takes the cached variant, tiles and rows for
 * whatever the options leave open (hfx_plan_describe reports tuned=yes);
 * a missing file or key leaves the defaults.  Size classes: the energy, K psi,
 * matrix and gradient calls run systems with the same compiled configuration,
 * kz band and screening state (up to eight) as one class whose batch steps
 * share one launch per pass, with one staging, pair-mean and zero-fill
 * launch for the class; other classes run on forked streams.  By default only
 * systems whose own pass launches are small (fewer than 512 workgroups) are
 * grouped; group=1 groups every system it can, group=0 none (results are the
 * same bit for bit; hfx_plan_describe reports class=<k>/<size>).  Uploads the plan's tables
 * (synchronous).  Errors: HFX_EINVAL for null out/sys, n_sys < 1, n <= 0,
 * L <= 0, n_orb < 1, unknown kernel or precision, erfc w <= 0, an unknown
 * option key or a malformed option value;
 * HFX_EUNSUPPORTED for n_x != n_y or an unsupported grid; HFX_EDEVICE or
 * HFX_ENOMEM when device set-up fails.  *out is NULL on failure.
 */
hfx_status hfx_plan_create(hfx_plan* out, const hfx_system* sys, int n_sys, int precision,
                           const char* options);

/* Release the plan and its device tables (synchronises the device). */
hfx_status hfx_plan_destroy(hfx_plan plan);

/* Workspace bytes that every compute call of this plan needs. */
hfx_status hfx_workspace_size(hfx_plan plan, size_t* bytes_host);

/*
 * E_x for each system (Eq. HFX with the 1/2 convention above), without
 * forming K psi.  psi: float64 orbitals; ex: n_sys float64 results.
 */
hfx_status hfx_exchange_energy(hfx_plan plan, const double* psi, double* ex, void* ws,
                               size_t ws_bytes, void* stream);

/*
 * K psi = V_X psi (Eq. vx) for every orbital, and optionally E_x.
 * kpsi: [n_orb][n^3] per system, float32 for an HFX_FP32 plan and float64
 * for an HFX_FP64 plan (overwritten).  ex: nullable, n_sys float64.
 */
hfx_status hfx_apply_exchange(hfx_plan plan, const double* psi, void* kpsi, double* ex,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * Exchange matrix M = dV Psi^T (K Psi), M_kl = <psi_k | K psi_l> (the matrix
 * whose Cholesky factor -M = L L^T builds the ACE operator, Eq. (vx_ace)),
 * as float64 row-major n_orb x n_orb blocks per system, and optionally E_x.
 * K psi is formed first (as by hfx_apply_exchange) in the workspace, which
 * holds n_orb x n^3 values of the plan's precision for it.  ex: nullable,
 * n_sys float64.  FP32 plans: psi is split into float32 hi + lo parts
 * (hi = fl32(psi), lo = fl32(psi - hi)), both multiplied with the float32
 * K psi on FP32 MFMA, each float32 accumulator folded into float64 every 32
 * grid points.  FP64 plans: float64 MFMA.  Errors as hfx_apply_exchange, and
 * HFX_EINVAL for a null m.
 */
hfx_status hfx_exchange_matrix(hfx_plan plan, const double* psi, double* m, double* ex, void* ws,
                               size_t ws_bytes, void* stream);

/*
 * The same contraction M = dV Psi^T (K Psi) from a K psi the caller already
 * holds (the output of hfx_apply_exchange for the same plan and psi, in the
 * plan's precision: float32 or float64 [n_orb][n^3] per system), so that an
 * SCF step that needs both K psi and M forms K psi once.  kpsi may be any
 * array of that layout and precision: the call is then a plain contraction.
 * HFX_EINVAL for null psi, kpsi or m.
 */
hfx_status hfx_exchange_matrix_kpsi(hfx_plan plan, const double* psi, const void* kpsi, double* m,
                                    void* ws, size_t ws_bytes, void* stream);

/*
 * hfx_apply_exchange without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same launch sequence and results
 * (K psi = V_X psi and optionally E_x, bitwise equal to hfx_apply_exchange's)
 * with the workspace in a file-scope device array of the library, 256 MiB on
 * every GPU the library runs on, held until the process ends.  The call
 * allocates nothing and creates no event (profiling is skipped); the first
 * call on a device looks the array's address up.  The plan's device must be
 * current.  Every call on one GPU shares that GPU's array: calls that overlap
 * on the device (from several host threads, or on streams not ordered with
 * each other) race and give wrong results; ordered calls are safe, since no
 * state is kept between calls (nothing in the array needs to start at zero).
 * Errors: HFX_EINVAL for null plan, psi or kpsi, or another device current;
 * HFX_ENOMEM when the plan's energy and K psi calls need more than 256 MiB
 * of workspace (plans with fewer tile pairs per batch, tiles=, need less);
 * HFX_EDEVICE when the array's address cannot be looked up.
 */
hfx_status hfx_apply_exchange_noalloc(hfx_plan plan, const double* psi, void* kpsi, double* ex,
                                      void* stream);

/*
 * Gradient of E_x: grad = 2 dV * gscale[s] * (K psi) for every system s, as
 * float64 [n_orb][n^3] (overwritten).  The pair potentials are recomputed
 * (nothing is kept from an earlier energy call).  gscale: nullable device
 * array of n_sys float64 factors (the incoming adjoint of E_x); NULL means 1.
 */
hfx_status hfx_exchange_gradient(hfx_plan plan, const double* psi, const double* gscale,
                                 double* grad, void* ws, size_t ws_bytes, void* stream);

/*
 * In-place orthonormalisation of psi in float64, S = dV Psi^T Psi (the
 * occupied Kohn-Sham orbitals on which V_X acts are orthonormal):
 *   HFX_ORTHO_LOWDIN:   Psi <- S^(-1/2) Psi (rows), S^(-1/2) from a coupled
 *                       Newton-Schulz iteration run to float64 convergence;
 *   HFX_ORTHO_CHOLESKY: Psi <- L^(-1) Psi with S = L L^T (orbital k mixes only
 *                       orbitals 0..k); a rank-deficient set gives NaN.
 * HFX_EINVAL for any other method.
 */
hfx_status hfx_orthonormalize(hfx_plan plan, double* psi, int method, void* ws,
                              size_t ws_bytes, void* stream);

/*
 * Adaptively compressed exchange (Methods, MTACE subsection, Eq. (vx_ace)):
 * V_X^ACE = - sum_k |P_k><P_k| with P = W L^(-T), W_i = V_X psi_i and
 * -M = L L^T the Cholesky factorisation of the exchange matrix.
 *
 * hfx_ace_build: from kpsi (W, as written by hfx_apply_exchange: float32 in
 * float32 plans, float64 in float64 plans) and m (M from hfx_exchange_matrix,
 * float64, per system n_orb x n_orb row-major, systems concatenated) writes
 * p (float64, the layout of psi): row k of each system is |P_k>, i.e. the
 * rows of L^(-1) W.  Factorisation and triangular inverse in float64.  A
 * matrix -M that is not positive definite (dependent orbitals) gives NaN in p.
 *
 * hfx_ace_apply: out = V_X^ACE phi, row by row (phi, out: float64, the layout
 * of psi; phi may be any set of n_orb functions per system, e.g. the current
 * orbitals of an SCF iteration).  out must not alias p or phi.
 *
 * Both are asynchronous on `stream`, use the workspace like the calls above,
 * and return HFX_EINVAL for null pointers, HFX_ENOMEM for a short workspace.
 */
hfx_status hfx_ace_build(hfx_plan plan, const void* kpsi, const double* m, double* p, void* ws,
                         size_t ws_bytes, void* stream);
hfx_status hfx_ace_apply(hfx_plan plan, const double* p, const double* phi, double* out,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * Pair screening of the s-MTACE variant (Methods, MTACE subsection: pairs
 * whose orbitals barely overlap are dropped from the exchange sums).
 *
 * hfx_screen evaluates A_ab = dV sum_r |psi_a(r)| |psi_b(r)| (float64 MFMA)
 * for the float64 orbitals psi (device, the layout of the other calls) and
 * keeps the pairs with A_ab >= rho_cut (decided once per unordered pair, on
 * A's upper triangle).  It then rebuilds every system's tile schedule over
 * the kept pairs: orbitals are grouped into tiles of strongly overlapping
 * orbitals (greedy clustering on A), tile pairs without a kept pair are
 * dropped, and the rest are packed first-fit into batches of disjoint
 * orbital blocks.  Every
 * later energy, K psi and gradient call of the plan sums over the kept pairs
 * only (the G = 0 energy of float32 plans too): K psi_a = -sum_{b kept} v_ab
 * psi_b.  rho_cut <= 0 restores the unscreened schedule (results identical
 * to a fresh plan).
 *
 * kept (host, one entry per system, may be NULL) receives the number of
 * kept unordered pairs a <= b.  The call waits for `stream` and returns
 * after the new schedule is uploaded (host-synchronous).  Graphs captured
 * earlier keep the schedule they were captured with: while any graph of the
 * plan is alive, the replaced device tables are kept (not freed) and are
 * released when the plan's last graph is destroyed, or with the plan.  HFX_EINVAL: null plan
 * or psi, a non-finite rho_cut, or a call during graph capture; HFX_ENOMEM:
 * short workspace.
 */
hfx_status hfx_screen(hfx_plan plan, const double* psi, double rho_cut, long long* kept, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * SCDM localisation (the s-MTACE screening acts on SCDM-localised orbitals;
 * Methods, MTACE subsection, citing the selected-columns-of-the-density-matrix
 * method).  For every system: grid points c_1..c_N (N = n_orb) are chosen by
 * column-pivoted QR of Psi^T (each step takes the point whose residual, after
 * the chosen points' directions are projected out, has the largest norm;
 * ties to the smallest index; float64); phi_k = sum_i psi_i psi_i(c_k), the
 * density-matrix columns at those points, Loewdin-orthonormalised in the dV
 * inner product.  psi, phi: float64, the layout of the other calls (phi may
 * equal psi: in place).  pivots: nullable device int array of sum(n_orb)
 * entries receiving the flat grid index (z n + y) n + x of c_k.  Asynchronous
 * on `stream`; the workspace is used as by the other calls.  Linearly
 * dependent orbitals give NaN.  HFX_EINVAL: null pointers or a call during
 * graph capture; HFX_EUNSUPPORTED: more than 3500 orbitals in a system.
 */
hfx_status hfx_scdm(hfx_plan plan, const double* psi, double* phi, int* pivots, void* ws,
                    size_t ws_bytes, void* stream);

/*
 * Size of a system's current tile schedule (host query, no device work):
 * info[0] batches, info[1] tile pairs, info[2] pair grids (complex grids,
 * two orbital pairs each) per exchange call, info[3] orbital pairs a <= b
 * evaluated.  HFX_EINVAL: null plan or info, system index out of range.
 */
hfx_status hfx_schedule_info(hfx_plan plan, int system, long long* info);

/*
 * One-line description of a system's kernel configuration and schedule:
 * variant name, grid, tile and brick sizes, radix schedules (forward/inverse
 * per axis), threads per workgroup (pair_fwd/plane/inv_acc), rows per tile
 * pair, tiles per batch, batches, batch streams and whether the pairs are
 * screened.  The text is
 * owned by the plan and valid until the next call of this function on the
 * plan or its destruction.  NULL (and HFX_EINVAL in hfx_last_error) for a null
 * plan or an index out of range.
 */
const char* hfx_plan_describe(hfx_plan plan, int system);

/*
 * Per-pass timing (tracing aid).  While enabled, every kernel launch of the
 * plan is bracketed by a pair of HIP events recorded on the caller's stream,
 * and the pass's algorithmic HBM bytes (each operand read or written once;
 * workspace grids count as HBM traffic) and flops are tallied.
 * hfx_profile_read waits for the recorded events, writes per-pass totals into
 * host arrays of length n (index = hfx_pass; NULL arrays are skipped) and
 * clears the record.  Events add a few microseconds per launch.
 */
typedef enum {
  HFX_PASS_STAGE = 0,      /* float64 -> float32 orbital copy               */
  HFX_PASS_ZERO,           /* K psi zero fill                                */
  HFX_PASS_PAIR_FWD,       /* pair product + forward z FFT                   */
  HFX_PASS_PLANE,          /* xy FFT, * v(G), inverse xy FFT (fused plane)   */
  HFX_PASS_ROWS_FWD,       /* split plane: forward x FFT                     */
  HFX_PASS_COLS_CONV,      /* split plane: y FFT, * v(G), inverse y FFT      */
  HFX_PASS_ROWS_INV,       /* split plane: inverse x FFT                     */
  HFX_PASS_INV_ACC,        /* inverse z FFT + energy + K psi accumulation    */
  HFX_PASS_INV_ENERGY,     /* inverse z FFT + energy                         */
  HFX_PASS_ENERGY_REDUCE,  /* fixed-order energy sum                         */
  HFX_PASS_CONTRACT,       /* Psi^T (K Psi) or Psi^T Psi on MFMA + reduction */
  HFX_PASS_ORTHO,          /* Newton-Schulz S^(-1/2) and Psi <- S^(-1/2) Psi */
  HFX_PASS_SCALE,          /* gradient scaling                               */
  HFX_PASS_ACE_BUILD,      /* Cholesky of -M, L^(-1), P = L^(-1) W           */
  HFX_PASS_ACE_APPLY,      /* -P (P^T phi): contraction and apply            */
  HFX_PASS_SCDM,           /* SCDM pivots and density-matrix columns         */
  HFX_PASS_COUNT
} hfx_pass;

hfx_status hfx_profile_enable(hfx_plan plan, int enable);
hfx_status hfx_profile_read(hfx_plan plan, double* ms_host, double* bytes_host,
                            double* flops_host, long long* launches_host, int n);

/*
 * Graphs: capture the complete launch sequence of one call for the given
 * buffers into a HIP graph, then replay it with hfx_graph_launch on any
 * stream (the same buffers are reused on every replay; their contents may
 * change).  Operations: HFX_GRAPH_ENERGY (hfx_exchange_energy; kpsi, m unused),
 * HFX_GRAPH_APPLY (hfx_apply_exchange; ex nullable, m unused), HFX_GRAPH_STEP
 * (hfx_orthonormalize of psi in place, hfx_apply_exchange, then
 * hfx_exchange_matrix; ex nullable).  Capture runs on a plan-owned stream and
 * launches nothing; the plan must outlive its graphs.  Systems of a batched
 * plan become parallel branches of one graph.  hfx_graph_destroy synchronises
 * the device when it releases schedule tables that hfx_screen replaced while
 * graphs were alive (see hfx_screen).
 */
typedef struct hfx_graph_t* hfx_graph;
typedef enum { HFX_GRAPH_ENERGY = 0, HFX_GRAPH_APPLY = 1, HFX_GRAPH_STEP = 2 } hfx_graph_op;

hfx_status hfx_graph_create(hfx_plan plan, int op, double* psi, void* kpsi, double* ex,
                            double* m, void* ws, size_t ws_bytes, hfx_graph* out);
hfx_status hfx_graph_launch(hfx_graph graph, void* stream);
hfx_status hfx_graph_destroy(hfx_graph graph);

/*
 * Names of the compiled kernel configurations for an n^3 (cubic) grid at the given
 * precision, ';'-separated, default first ("" if the size is unsupported).
 * A plan selects one with the option "variant=<name>" (a list for batches).
 * The returned string is thread-local and valid until the next call.
 */
const char* hfx_variants(int n, int precision);

/*
 * Autotuner (host-synchronous; allocates device memory for its trial runs).
 * For each of the n_sys systems (described as for hfx_plan_create, orbitals
 * psi concatenated in that order, float64 device data as the compute calls
 * take), times hfx_apply_exchange of single-system plans over the compiled
 * kernel configurations of the system's grid (hfx_variants) crossed with the
 * batch size (tiles=0, the default, and tiles=4) and the rows per tile pair
 * (8, 16, 32 up to the orbital count), reps timed calls after one warm-up,
 * with HIP events on `stream` (the fastest of the reps counts).  The fastest
 * wins, except that among candidates within 5 % of it the first in a fixed
 * order is taken (the plan defaults first), which keeps the choice stable
 * against run-to-run timing spread.  `options`
 * (nullable) is added to every candidate plan, e.g. "ecut=20", and may not
 * name variant, tiles, rows or tune_cache.  cache_path (nullable): a text
 * file of earlier choices, one line "<key> <options> <ms>" per system key,
 * each followed by its candidate table ("<key>#candidate <options> <ms>")
 * (device architecture, grid, orbital count, precision, kz band of ecut and
 * the identity of the compiled kernel sources); systems found there are not
 * timed again and new choices are added.  chosen_host (nullable, host,
 * chosen_bytes long) receives the choice as plan options with one value per
 * system, "variant=a,b;tiles=x,y;rows=p,q", which hfx_plan_create accepts;
 * plans created with option tune_cache=<path> (or with the environment
 * variable HFX_AUTOTUNE_CACHE set) take each system's cached choice for
 * whatever their own options leave open.  Errors: HFX_EINVAL for null sys or
 * psi, n_sys < 1, a bad precision, an option the tuner sets itself, a short
 * chosen_host or an unwritable cache; HFX_EUNSUPPORTED for a grid without a
 * compiled configuration; otherwise the status of a failing trial plan.
 */
hfx_status hfx_autotune(const hfx_system* sys, int n_sys, int precision, const char* options,
                        const double* psi, int reps, const char* cache_path, char* chosen_host,
                        size_t chosen_bytes, void* stream);

/* Static description of a status code. */
const char* hfx_status_string(hfx_status s);

/* Thread-local description of the last failure in this thread ("" if none). */
const char* hfx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HFX_H */

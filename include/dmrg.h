/*
 * C-ABI of the MI355X DMRG linear-response library (DMRG sigma, block
 * renormalization, ground-state sweeps and DMRG-TDA Davidson sweeps).
 *
 * Method: Nakatani, Wouters, Van Neck, Chan, "Linear response theory for the
 * density matrix renormalization group" (arXiv:1311.1646).  Section and
 * equation labels below refer to that paper.
 *
 * Conventions shared by every entry point
 *  - Sites are spatial orbitals 0..L-1; the local basis of a site is
 *    n = 0:|0>, 1:|alpha>, 2:|beta>, 3:|alpha beta> = a+_alpha a+_beta |0>;
 *    fermion order is site-major, alpha before beta.
 *  - Bond b (0..L) lies left of site b; its symmetry sectors are labelled by
 *    the (n_alpha, n_beta) counted over sites 0..b-1, listed in increasing
 *    (n_alpha, n_beta) order.
 *  - A one-site coefficient tensor at site i has one dense row-major block per
 *    (left sector a of bond i, n) whose right sector c = q_a + q(n) exists at
 *    bond i+1; blocks are stored consecutively ordered by a then n (the
 *    "flat layout").  A two-site tensor at (i, i+1) uses (a, n1, n2) ordering
 *    with c at bond i+2.  dmrg_get_layout reports the blocks.
 *  - Integrals: h is L*L row-major; eri is L^4 row-major, chemist notation
 *    (pq|rs), real orbitals (8-fold symmetry is assumed, not checked).
 *  - Every call returns 0 (DMRG_OK) or a negative code; no exception crosses
 *    the ABI.  dmrg_last_error gives the message of the last failure.
 *  - Device work is enqueued on the stream given to dmrg_create; calls that
 *    return host scalars synchronize that stream.
 */
#ifndef DMRG_H_
#define DMRG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DMRG_OK = 0,
  DMRG_ERR_INVALID_ARG = -1,
  DMRG_ERR_OOM = -2,
  DMRG_ERR_NOT_CONVERGED = -3,
  DMRG_ERR_SINGULAR = -4,
  DMRG_ERR_HIP = -5,
  DMRG_ERR_STATE = -6,
  DMRG_ERR_INTERNAL = -7
};

/* Arithmetic of the operator contractions (sigma and renormalization).
 * FP64 everywhere; FP32 operands with FP32 accumulation; BF16X3: FP32
 * operands split x = hi + lo into bfloat16 parts, products hi*hi + hi*lo +
 * lo*hi accumulated in FP32.  Davidson data, gauge transforms and reduced
 * matrices are FP64 in every mode. */
enum { DMRG_FP64 = 0, DMRG_FP32 = 1, DMRG_BF16X3 = 2 };

/* Kinds of sigma (Sec. II A eq. dmrg; Sec. III B-D):
 *  ZEROTH_1SITE : sigma = H_0^[i] C, the one-site effective Hamiltonian
 *                 L_{i-1} x h_i x R_i (Sec. III B, eq. hzero_sb) applied to
 *                 nvec vectors.
 *  ZEROTH_2SITE : the two-site effective Hamiltonian on sites (i, i+1)
 *                 (Sec. II A, the site problem on two sites).
 *  TDA_FULL     : the TDA sigma of Sec. III D, eq. sigv1 with Delta-sigma of
 *                 eq. sigv2, for nvec first-order wavefunctions:
 *                   sigma^mu = H_0^[i] C^mu(1)
 *                            + [H_mu^{L} x h_i x H_0^{R}] C_i^(0)
 *                            + [H_0^{L} x h_i x H_mu^{R}] C_i^(0),
 *                 where C_in holds C_i^{mu(1)}, C_i^(0) is the imported centre
 *                 tensor at site i, and H_mu^{L} / H_mu^{R} are the
 *                 first-order block operators (Sec. III B eq. lopr1st, Sec.
 *                 III D eq. ropr1st) built beforehand by dmrg_renormalize
 *                 with order DMRG_FIRST: the left chain must end at bond i
 *                 and the right chain at bond i+1 (the left part is zero at
 *                 site 0 and the right part at site L-1, where no chain is
 *                 needed).  Width 1 only.
 *  TDA_DH_LEFT  : the first line of eq. sigv2 alone, applied to the given
 *                 vectors: sigma^mu = [H_mu^{L} x h_i x H_0^{R}] C_in^mu
 *                 (the left chain must end at bond i; zero at site 0). */
enum { DMRG_SIGMA_ZEROTH_1SITE = 0, DMRG_SIGMA_ZEROTH_2SITE = 1,
       DMRG_SIGMA_TDA_FULL = 2, DMRG_SIGMA_TDA_DH_LEFT = 3 };

/* Order of a renormalization (dmrg_renormalize). */
enum { DMRG_ZEROTH = 0, DMRG_FIRST = 1 };

enum { DMRG_DIR_LEFT = 0, DMRG_DIR_RIGHT = 1 };

typedef struct dmrg_ctx dmrg_ctx;

/* Device allocator of a context.  The library owns its operator pools, MPS
 * tensors, plans and workspaces; with this callback their device memory comes
 * from the caller's memory manager (e.g. a framework's caching allocator).
 * alloc returns memory usable in stream order on the context's stream, or
 * NULL (the call then fails with DMRG_ERR_OOM); free receives exactly the
 * pointers alloc returned, after the work that used them was enqueued on the
 * context's stream.  NULL members mean hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} dmrg_allocator;

/* Create a context for L orbitals and (n_alpha, n_beta) electrons: the
 * quantum-chemical Hamiltonian of real orbitals in second quantization
 * (the H of Sec. II A, eq. dmrg) with one-electron integrals h, two-electron
 * integrals eri and the constant ecore.
 * The integrals are copied; the caller keeps ownership of h and eri.
 * device < 0 creates a host-only context on which only the host/test-support
 * calls (dmrg_debug_*, layout queries) are valid.  stream: a hipStream_t or
 * NULL for the null stream.  alloc may be NULL (hipMalloc / hipFree); the
 * struct is copied.
 * Errors: INVALID_ARG (L outside [2, 128], electron counts, null integrals),
 * HIP_ERROR, OOM. */
int dmrg_create(int L, int n_alpha, int n_beta, const double* h, const double* eri,
                double ecore, int device, void* stream, const dmrg_allocator* alloc,
                dmrg_ctx** out);
/* Release the context and everything it owns (waits for nothing: the caller
 * synchronizes its stream first if work is still queued).  INVALID_ARG on NULL. */
int dmrg_destroy(dmrg_ctx* ctx);
/* Message of the last failed call on ctx (of the last failed dmrg_create when
 * ctx is NULL); owned by the library, valid until the next call on ctx. */
const char* dmrg_last_error(const dmrg_ctx* ctx);

/* Number of channels (normal + complementary operators) of the block
 * operator sets at bond b: the "x" summation over complementary operators
 * of Sec. III B (eq. hzero_sb) made explicit.  INVALID_ARG on a bad bond. */
int dmrg_num_channels(dmrg_ctx* ctx, int bond, int* out);

/* Import a mixed-canonical MPS (host FP64; copied to the device).
 *  nsec[b], b = 0..L: number of sectors of bond b;
 *  sectors: for all bonds in order, (n_alpha, n_beta, dim) per sector;
 *  Ldata / Rdata / Cdata: for all sites in order, the flat one-site layout of
 *  the left-orthonormal L_i, right-orthonormal R_i and C_i = L_i Lambda_i =
 *  Lambda_{i-1} R_i (Sec. II A, eq. gauge-shift);
 *  lam: for all bonds in order, per sector, the diagonal of Lambda_b.
 * Bonds 0 and L must hold the single sectors (0,0) and (n_alpha,n_beta) of
 * dimension 1.  Errors: INVALID_ARG on inconsistent tables. */
int dmrg_import_mps(dmrg_ctx* ctx, const int* nsec, const int* sectors, const double* Ldata,
                    const double* Rdata, const double* Cdata, const double* lam);

/* Export the current MPS in the same format (Sec. II A, eq. gauge-shift).
 * Call with NULL data pointers to get the sizes: nsec_out must hold L+1
 * ints; sizes_out[0..3] receives the number of sector triples and the
 * lengths of L/R/C data and of lam.  Errors: STATE without an MPS. */
int dmrg_export_mps(dmrg_ctx* ctx, int* nsec_out, int* sectors_out, double* Ldata,
                    double* Rdata, double* Cdata, double* lam, size_t* sizes_out);

/* Layout of the one-site (width 1) or two-site (width 2) coefficient tensor
 * at `site` (the C_i of Sec. II A, eq. mps_wave, blocked by the symmetry
 * sectors of its bonds): nblocks_out receives the block count; if blocks_out
 * is non-NULL it receives 6 ints per block (a, n, c, rows, cols, offset);
 * size_out receives the element count.  STATE without an MPS. */
int dmrg_get_layout(dmrg_ctx* ctx, int site, int width, int* nblocks_out, int* blocks_out,
                    size_t* size_out);

/* Build the zeroth-order renormalized block operators H_0^{L_b} and
 * H_0^{R_b} (normal and complementary) at every bond from the imported MPS
 * (Sec. III B: the operators "known from the ground-state DMRG").
 * prec is the arithmetic of the renormalization contractions (FP64, FP32;
 * BF16X3 builds these pools in FP32 because their errors compound over the
 * bonds).  Pools are stored in FP64; FP32 copies are made on first use by a
 * lower-precision sigma.  Errors: STATE without an MPS, INVALID_ARG. */
int dmrg_build_ops(dmrg_ctx* ctx, int prec);

/* Sigma vectors (Sec. II A eq. dmrg; Sec. III B eq. hzero_sb; Sec. III D
 * eqs. sigv1, sigv2 for the TDA kinds, see above).  C_in and sigma_out are
 * device FP64 arrays of len = nvec * size elements each (vector-major, each
 * vector in the flat layout of the one-site tensor at `site` or of the
 * two-site tensor at (site, site+1); size from dmrg_get_layout).  Both are
 * borrowed for the (stream-ordered) call and must not overlap.  prec is the
 * arithmetic of the contractions.  Requires dmrg_build_ops.
 * Errors: STATE before build_ops or when a TDA kind finds the first-order
 * chains at other bonds; INVALID_ARG on a bad site / kind / nvec, a len that
 * is not nvec * size, null pointers, or a TDA kind whose chains hold another
 * nvec (or FP32 sets for an FP64 sigma). */
int dmrg_sigma(dmrg_ctx* ctx, int site, int kind, int nvec, const double* C_in,
               double* sigma_out, size_t len, int prec);

/* No-allocation variant of dmrg_sigma, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Zeroth-order kinds only (ZEROTH_1SITE,
 * ZEROTH_2SITE); same arguments, layout and result as dmrg_sigma.  Its
 * workspaces come from a statically allocated scratch array of
 * DMRG_NOALLOC_SCRATCH_BYTES per GPU, held for the life of the process; it
 * calls no hipMalloc / hipFree and creates no event (stats.sigma_ms is not
 * updated).  One ordinary dmrg_sigma call with the same site, kind, nvec and
 * precision must come first: it builds the plans and tile lists and records
 * the workspace sizes (and again after dmrg_sweep_ground, dmrg_tda_roots,
 * dmrg_rpa_roots, dmrg_tda_transition or dmrg_response, which drop the
 * cached tile lists when they end).  Every call on a GPU shares that GPU's scratch (it
 * keeps the last call's contents; nothing in it needs clearing), so calls
 * that overlap on one GPU race.
 * Errors: INVALID_ARG (as dmrg_sigma, a TDA kind, or a workspace larger
 * than the scratch), STATE (no preparing dmrg_sigma call, or something the
 * call would have to allocate is missing). */
#define DMRG_NOALLOC_SCRATCH_BYTES (64u << 20)
int dmrg_sigma_noalloc(dmrg_ctx* ctx, int site, int kind, int nvec, const double* C_in,
                       double* sigma_out, size_t len, int prec);

/* Tile-shape autotuner of the grouped block GEMM (the contractions of Sec.
 * III B-D): times the one-site sigma at `site` for nvec vectors in precision
 * prec under every pair of stage-1 / stage-2 tile shapes (the planner's
 * choice, 64x64, 128x64, 64x128, and 128x128 for FP32 operands) and keeps the
 * fastest pair for all later contractions of that precision in this context.
 * shapes_out[0..1] receives the chosen stage-1 and stage-2 shapes (-1 =
 * planner's choice, 0 = 64x64, 1 = 128x64, 2 = 64x128, 3 = 128x128) and
 * best_ms_out the device time of that sigma.  Allocates two nvec x size FP64
 * device buffers for the duration of the call.  Errors: STATE before
 * build_ops, INVALID_ARG. */
int dmrg_autotune(dmrg_ctx* ctx, int site, int nvec, int prec, int* shapes_out, double* best_ms_out);

/* Diagonal of the one-site (width 1) or two-site (width 2) effective
 * Hamiltonian at `site`, the Davidson preconditioner of Sec. III D eq. error,
 * written to a device FP64 array of len = size elements.  prec must be FP64.
 * Errors: STATE before build_ops, INVALID_ARG (len, precision). */
int dmrg_diag(dmrg_ctx* ctx, int site, int width, double* diag_out, size_t len, int prec);

/* Renormalization of block operators across one site.
 * order DMRG_ZEROTH: recompute the zeroth-order operators of one bond from
 *   the current MPS (the operators "known from the ground-state DMRG" of
 *   Sec. III B): dir LEFT builds H_0^{L_{site+1}} from H_0^{L_site} and L_site;
 *   RIGHT builds H_0^{R_site} from H_0^{R_{site+1}} and R_site.  nvec must be
 *   0 and A1 NULL.
 * order DMRG_FIRST: grow a chain of first-order operators (bra zeroth order,
 *   ket first order) by one site, for nvec first-order tensors at once:
 *   LEFT (Sec. III B, eq. lopr1st):
 *     H_mu^{L_{site+1}} = L^T [H_mu^{L_site} x h] L + L^T [H_0^{L_site} x h] L^{mu(1)}
 *   with A1 = L_site^{mu(1)}; the chain starts at site 0 (from the empty
 *   block) and every later call must be at the site where the chain ends.
 *   RIGHT (Sec. III D, eq. ropr1st): the mirror image with A1 = R_site^{mu(1)},
 *   starting at site L-1 and moving left.
 *   A1 is a device FP64 array of len = nvec * size(site) elements in the flat
 *   one-site layout, borrowed for the call.  The library applies the gauge
 *   condition of the first-order tensors (Sec. II B, eqs. left-orthoSeb,
 *   right-orthoSeb) itself: it uses Q^L A1 = A1 - L (L^T A1) (left) or
 *   A1 Q^R = A1 - (A1 R^T) R (right), per symmetry block.  The chain's sets
 *   are held in FP64 for prec FP64 and in FP32 otherwise; they are used by
 *   the TDA sigma kinds of dmrg_sigma and dropped by dmrg_import_mps,
 *   dmrg_build_ops, dmrg_sweep_ground and dmrg_tda_roots (which builds its
 *   own first-order operators).
 * Errors: STATE (before build_ops, chain at another bond), INVALID_ARG (site,
 * dir, order, nvec or precision class differing from the chain's, len). */
int dmrg_renormalize(dmrg_ctx* ctx, int site, int dir, int order, int nvec, const double* A1,
                     size_t len, int prec);

typedef struct {
  int nsweeps;            /* two-site sweeps (left->right->left counts 1)  */
  const int* M_schedule;  /* bond dimension per sweep (nsweeps entries)    */
  const double* noise;    /* reserved, not applied (may be NULL): the two-
                             site update reaches new sectors by itself     */
  double davidson_tol;    /* residual norm^2 threshold of the local solver */
  int davidson_max_iter;  /* per site                                      */
  int seed;               /* initial state                                 */
  int prec;               /* DMRG_FP64 / FP32 / BF16X3 contractions        */
  int verbose;
  int onesite_sweeps;     /* one-site sweeps after the two-site ones (0:
                             none): bond dimensions fixed, the centre
                             optimized at every site, so the MPS converges
                             to a stationary point of the energy on its
                             manifold, the reference dmrg_rpa_roots needs   */
} dmrg_sweep_params;

/* Ground state by two-site sweeps with Davidson (Sec. II A, eq. dmrg and
 * eq. gauge-shift), followed by one non-truncating one-site pass that leaves
 * a consistent mixed-canonical MPS (L_i, C_i, R_i, Lambda_i at every site)
 * and its zeroth-order operators (built in FP64) for dmrg_tda_roots.
 * Starts from the imported MPS if there is one, else from a random MPS
 * (seed) with sector dimensions min(exact, M_schedule[0] / #sectors).
 * Each two-site step keeps at most M states over all sectors of the split
 * bond (singular values below 1e-12 of the largest are dropped).  Then
 * onesite_sweeps one-site sweeps (right, then left) replace the centre by
 * the lowest eigenvector of the one-site effective Hamiltonian at every
 * site and move it by non-truncating splits.  prec is
 * the arithmetic of the sigma and renormalization contractions; Davidson,
 * SVD and the final energy are FP64.  energy receives <Psi|H|Psi> of the
 * final MPS; discarded the largest discarded weight of the last sweep.
 * Errors: INVALID_ARG (schedule), NOT_CONVERGED (an SVD failed). */
int dmrg_sweep_ground(dmrg_ctx* ctx, const dmrg_sweep_params* p, double* energy,
                      double* discarded);

typedef struct {
  int max_iter;        /* Davidson iterations (one forward+backward sweep each) */
  int max_space;       /* N: maximum number of trial vectors (<= 64); 0: 64,
                          lowered to what fits in 60% of the free device
                          memory as hipMemGetInfo reports it (at least
                          2n + 2; memory cached by the allocator behind
                          dmrg_allocator counts as used, so such a caller
                          releases its cache first, as the Python binding
                          does); a full space restarts from the lowest
                          max(n + max(2, n/2), N/2) Ritz vectors; the value
                          used is in dmrg_stats.tda_space                     */
  double tol;          /* convergence: max_mu sum_i |r_i^mu|^2 < tol             */
  int seed;            /* random initial trial vectors                           */
  int prec;            /* contraction precision                                  */
  int verbose;
  int polish;          /* FP32 and BF16X3 runs: 0 (default) finishes with FP64
                          iterations once the residual reaches the estimated
                          floor of the run's contractions, 4 L (eps E_0)^2
                          with eps = 2^-16 (BF16X3) or 2^-19 (FP32), or tol,
                          or stalls near that floor (at least two FP64
                          iterations; convergence is judged in FP64); -1 keeps
                          the run's precision to the end                      */
  int guess;           /* initial trial vectors: 0 (default) unit vectors on the
                          n lowest diagonal elements of the middle site's
                          effective Hamiltonian (eq. error's diagonal); 1 seeded
                          random components at every site (as in Fig.
                          alg:dmrgtda; the Davidson then spends tens of
                          iterations on a plateau)                            */
} dmrg_davidson_params;

/* DMRG-TDA roots by the sweep Davidson algorithm (Sec. III, Fig. alg:dmrgtda)
 * on the current MPS (imported or from dmrg_sweep_ground; build_ops first).
 * FP32 and BF16X3 runs are polished by FP64 iterations (see
 * dmrg_davidson_params): the contraction error enters the reduced matrices
 * of eqs. hleft2 / sleft2, hence the excitation energies, to first order and
 * in proportion to |E_0|; stats.tda_polish_iters reports how many iterations
 * ran in FP64.
 * Outputs (host, nroots each): omega = E_mu - E_0 with E_0 = <Psi0|H|Psi0>,
 * e_total = E_mu, resid2 = sum over sites of |r_i^mu|^2 of the last
 * iteration; iters = Davidson iterations used.  NOT_CONVERGED fills the
 * outputs with the last iterate.  Releases the first-order chains of
 * dmrg_renormalize (order 1) before it starts. */
int dmrg_tda_roots(dmrg_ctx* ctx, int nroots, const dmrg_davidson_params* p, double* omega,
                   double* e_total, double* resid2, int* iters);

/* Grouped sigma of many independent problems.  n member contexts (each with
 * its MPS imported and dmrg_build_ops done, all on one device and stream)
 * apply the zeroth-order one-site sigma (Sec. III B, eq. hzero_sb) at their
 * own sites[i] to nvec vectors each, as one launch per contraction stage for
 * all members: the members' cached work lists are concatenated, each job
 * tagged with its member, whose base table the kernels read from device
 * memory.  The group holds pointers into its members' operator pools: it is
 * valid while they keep their MPS and operators (a later dmrg_import_mps,
 * dmrg_build_ops, dmrg_sweep_ground or zeroth-order dmrg_renormalize on a
 * member makes dmrg_group_sigma fail with STATE), and must be destroyed
 * before its members.
 * Errors: INVALID_ARG (sites, nvec, precision, contexts on different
 * devices or streams), STATE (a member without operators), OOM. */
typedef struct dmrg_group dmrg_group;
int dmrg_group_create(dmrg_ctx* const* ctxs, int n, const int* sites, int nvec, int prec, dmrg_group** out);
/* One grouped sigma step: C_in[i] / sigma_out[i] are member i's device FP64
 * arrays of lens[i] = nvec * size elements (layout as in dmrg_sigma),
 * borrowed for the call; enqueued after the members' earlier work and
 * followed by their later work (their stream waits for it).  use_graph != 0
 * replays the step from a HIP graph, captured at the second such call (the
 * first one runs eagerly and builds the tile lists); new buffers re-upload
 * only the base tables the graph reads.  Synchronizes (the step's device
 * time is kept for dmrg_group_stats).
 * Errors: INVALID_ARG (lens, null arrays), STATE (a member changed). */
int dmrg_group_sigma(dmrg_group* g, const double* const* C_in, double* const* sigma_out, const size_t* lens,
                     int use_graph);
/* Algorithmic flops of one step (all members), device time of the last
 * step, kernel launches per step, and nodes of the captured graph (0 before
 * capture).  Any output pointer may be NULL. */
int dmrg_group_stats(dmrg_group* g, double* flops, double* ms, int* launches, int* graph_nodes);
const char* dmrg_group_last_error(const dmrg_group* g);
int dmrg_group_destroy(dmrg_group* g);

/* Test support: the reduced matrices H_R and S_R (Sec. III B, eqs. hleft2
 * and sleft2, summed over sites) of the last forward sweep of the last
 * dmrg_tda_roots, l x l row-major FP64 on the host.  With NULL HR / SR only
 * l is returned.  Errors: STATE before a TDA run. */
/* DMRG-TDA roots (as dmrg_tda_roots, same arguments and errors) and their
 * one-particle transition density matrices (Sec. VI A)
 *   gamma^nu_pq = <Psi^nu | E_pq | Psi0>,  E_pq = sum_sigma a+_{p sigma} a_{q sigma},
 * for the nroots roots Psi^nu (unit norm in the tangent space, orthogonal
 * to Psi0; the overall sign of each root is arbitrary).  gamma: host array
 * of nroots * L * L doubles, gamma[(nu L + p) L + q].  Cost: after the TDA,
 * L^2 evaluations of E_pq Psi0 projected on every site (each the zeroth-order
 * sigma of a one-body operator on the same MPS), meant for the diagnostic
 * sum_pq gamma_pq^2 on small and medium systems. */
int dmrg_tda_transition(dmrg_ctx* ctx, int nroots, const dmrg_davidson_params* p, double* omega,
                        double* e_total, double* resid2, int* iters, double* gamma);

/* Frequency-dependent linear response to a one-body perturbation
 * V = sum_pq v_pq E_pq (E_pq the spin-summed excitation operator), Sec. II B,
 * eqs. realresp and imagresp: the first-order wavefunctions of the +omega
 * and -omega components (eq. psi1st, gauge of eqs. left-orthoSeb and
 * right-orthoSeb, orthogonal to Psi0) solve
 *   (H - (E0 - omega)) Psi1_+ = -Q V Psi0,   (H - (E0 + omega)) Psi1_- = -Q V Psi0
 * in the tangent space of the imported MPS, E0 = <Psi0|H|Psi0>.  They are
 * found by the sweep Davidson of dmrg_tda_roots (same sigma, reduced
 * matrices and Q^C projection) with the reduced linear system solved in the
 * Ritz basis and residuals (H - z) x + Q P_i^T V Psi0 at every site.
 * v: host L x L row-major symmetric matrix; omega: real frequency (away
 * from the poles E_mu - E0).  p: as for dmrg_tda_roots (nroots is 2; the
 * tolerance applies to both residuals; guess is ignored: the start vectors
 * are the preconditioned right-hand sides).  chi[0] = <V Psi0 | Psi1_+>,
 * chi[1] = <V Psi0 | Psi1_->; the dynamic polarizability along v is
 * alpha(omega) = -(chi[0] + chi[1]).  resid2[0..1]: final residual norms^2.
 * NOT_CONVERGED fills the outputs of the last iteration.
 * Errors: STATE before build_ops, INVALID_ARG (v not symmetric or not
 * finite, omega not finite, parameters), SINGULAR (V Psi0 has no component
 * in the tangent space). */
int dmrg_response(dmrg_ctx* ctx, const double* v, double omega, const dmrg_davidson_params* p, double* chi,
                  double* resid2, int* iters);

/* DMRG-RPA roots (Sec. II C eq. dmrgrpa; Sec. III E eqs. reducedrpa and
 * bmatrix) of the current MPS, which is taken to be a stationary point of
 * the energy on the MPS manifold (a converged ground state: the truncating
 * two-site sweeps do not end there, dmrg_sweep_ground with onesite_sweeps
 * does; away from it A +- W can be indefinite).  The Davidson
 * sweeps of dmrg_tda_roots run over trial first-order wavefunctions U; the
 * reduced matrices are H_R and S_R of eqs. hleft2 / sleft2 and the
 * second-order matrix W_R = W(U, U), accumulated in the backward sweep from
 * the left-gauge pieces of one vector and the first-order right block
 * states of the other (eq. bmatrix, both orders); the forward and backward
 * amplitudes are X = U a, Y = U b and the reduced problem
 *   [[A, W_R], [W_R, A]] (a, b) = omega [[S_R, 0], [0, -S_R]] (a, b),
 *   A = H_R - E0 S_R,
 * is solved on the host after canonical orthogonalization of S_R, through
 * the symmetric form of (A - W)(A + W).  Per root two residuals are formed
 * at every site: r_X = (H - E0 - omega) X + W Y and
 * r_Y = (H - E0 + omega) Y + W X, with the site-i part of W v taken as
 * <U_v n r|H|Psi0> + <l n V_v|H|Psi0> (U_v, V_v the first-order left /
 * right block states of v, first-order operator chains with the
 * first-order tensor on the bra side); this is the exact gradient of W at
 * a stationary reference.  Both corrections join the space, so it grows by
 * 2 nroots vectors per iteration (max_space >= 4 nroots); a full space
 * keeps X and Y of the lowest roots.  p: as for dmrg_tda_roots (guess 0:
 * unit vectors on the 2 nroots lowest diagonal elements of the middle
 * site).  omega receives the nroots lowest RPA excitation energies, e_total
 * E0 + omega, resid2 per root the larger of max sum_i |r_i|^2 of its X and
 * Y residuals.  NOT_CONVERGED fills the outputs of the last iteration.
 * Errors: STATE before build_ops, INVALID_ARG (parameters), SINGULAR (the
 * trial space lost rank below nroots, or A - W / A + W is not positive
 * definite on it: an unstable reference). */
int dmrg_rpa_roots(dmrg_ctx* ctx, int nroots, const dmrg_davidson_params* p, double* omega, double* e_total,
                   double* resid2, int* iters);

/* The reduced DMRG-RPA problem of eq. reducedrpa alone, on the host (no
 * context, no device): HR, SR, WR are l x l symmetric host arrays (the
 * matrices of dmrg_rpa_roots over l trial vectors), e0 the reference
 * energy.  Writes the nroots lowest roots omega_out[nroots] and, when x_out
 * / y_out are not NULL, the amplitudes a (x_out) and b (y_out) of each root
 * in the trial basis (l x nroots, column k = root k, element u + k*l),
 * normalized to a^T S_R a - b^T S_R b = 1.  Directions with S_R eigenvalue
 * below 1e-10 of the largest are dropped.  Returns the rank kept, or
 * INVALID_ARG (l < 1, l > 4096, null inputs) or SINGULAR (rank below nroots,
 * A - W or A + W not positive definite). */
int dmrg_rpa_reduced(int l, const double* HR, const double* SR, const double* WR, double e0, int nroots,
                     double* omega_out, double* x_out, double* y_out);

int dmrg_tda_reduced(dmrg_ctx* ctx, int* l, double* HR, double* SR);

#define DMRG_TDA_HIST 256 /* iterations kept in dmrg_stats.tda_r2_hist */

typedef struct {
  double sigma_flops;      /* algorithmic flops of the last dmrg_sigma call        */
  double sigma_ms;         /* device time of the last dmrg_sigma call              */
  double sigma_main_ms;    /* device time of its dominant (stage-2) kernel         */
  double sigma_main_flops; /* algorithmic flops of that kernel                     */
  double sigma_main_bytes; /* algorithmic bytes of that kernel: distinct operator
                              blocks and products read once, results read and
                              written once                                        */
  double renorm_flops, renorm_ms;
  double op_bytes;         /* device bytes held by zeroth-order operator pools     */
  double tda_iter_ms;      /* wall time of the last TDA Davidson iteration         */
  double tda_sigma_flops;  /* algorithmic flops of the TDA sigma (eq. sigv1) at the
                              middle site in that iteration: the first-order left
                              part (eq. sigv2) for all trial vectors plus the
                              zeroth-order part for the roots                      */
  int tda_iters;
  int sigma_main_launches; /* launches of the dominant kernel in the last sigma    */
  double tda_sigma_ms;     /* device time of that TDA sigma                         */
  double plan_ms;          /* host time of planning the contractions of the last
                              dmrg_build_ops (renorm_ms is then the device time of
                              its renormalizations alone)                           */
  double sigma_workspace_bytes; /* device workspace of the last zeroth-order
                              dmrg_sigma (what dmrg_sigma_noalloc needs from its
                              scratch for the same shape)                           */
  int tda_polish_iters;    /* iterations of the last dmrg_tda_roots run in FP64
                              polish (0: none)                                      */
  int tda_hist_len;        /* entries of tda_r2_hist                                */
  double tda_r2_hist[DMRG_TDA_HIST]; /* max over roots of sum_i |r_i^mu|^2 per
                              iteration of the last dmrg_tda_roots (first
                              DMRG_TDA_HIST iterations)                             */
  double tda_total_ms;     /* wall time of the last dmrg_tda_roots, including the
                              initial sweeps                                        */
  int tda_space;           /* maximum trial space N of the last dmrg_tda_roots      */
  double tda_phase_ms[6];  /* device time of the last iteration of a verbose
                              dmrg_tda_roots by phase: first-order sigma parts
                              (eq. sigv2), zeroth-order sigma (eqs. sigv1,
                              hleft2), first-order operators renormalized from
                              first-order ones, from zeroth-order ones (eqs.
                              lopr1st, ropr1st), vector work (projections,
                              gauge, reduced matrices), host waits            */
} dmrg_stats;

/* Metrics log: when the environment variable DMRG_LOG_JSONL names a file,
 * dmrg_sweep_ground appends one JSON object per sweep ("ground_sweep") and
 * dmrg_tda_roots / dmrg_response one per Davidson iteration
 * ("tda_iteration" / "response_iteration"), one object per line. */
int dmrg_get_stats(dmrg_ctx* ctx, dmrg_stats* out);
/* sizeof(dmrg_stats) as compiled into the library, so that a binding can
 * check its own copy of the layout (host only, needs no context). */
size_t dmrg_stats_size(void);

/* Test support (host only, L <= 5): contract the channel site operators into
 * the dense 4^L x 4^L Fock-space Hamiltonian, basis index sum_i n_i 4^i.
 * wide_bond >= 0 uses the two-site operator on (wide_bond, wide_bond+1);
 * from_right selects the right-to-left contraction. */
int dmrg_debug_mpo_dense(dmrg_ctx* ctx, int wide_bond, int from_right, double* out);

#ifdef __cplusplus
}
#endif
#endif /* DMRG_H_ */

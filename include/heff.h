/*
 * heff.h -- C ABI of the two-site effective-Hamiltonian library for
 * MI355X (gfx950).
 *
 * The library implements the Davidson matrix-vector product of two-site
 * ab initio DMRG, Psi' = H_eff Psi, in the U(1)xU(1) block-sparse task form
 * of Sec. II.C (Eqs. ``Hamilton_act_nonsym`` and ``Hamilton_act_U1sym``):
 * the Hamiltonian of Eq. ``Hamiltonian`` is factorized over the left block
 * L, the two middle sites and the right block R, and every task adds
 * f * O^L{p_L} Psi{p} O^R{p_R}^T to one output block.
 *
 * Conventions shared with the input generator (``synth.py``):
 *   - N spatial orbitals, sites 0..N-1; the two-site pair is (k0, k0+1) with
 *     k0 = N/2 - 1 (integer division); L = sites 0..k0-1, R = k0+2..N-1.
 *   - Site state s = 0..3 is (empty, down, up, up+down) with
 *     |up down> = c+_up c+_down |0>, label (n_up, n_dn).
 *   - Integrals: h[i*N + j] = h_ij (symmetric); V[((i*N+j)*N+k)*N+l] =
 *     (ij|kl) (8-fold symmetric); H = sum h_ij c+_is c_js
 *     + 1/2 sum (ij|kl) c+_is c+_kt c_lt c_js.
 *   - A bond table lists the sectors (n_up, n_dn) of one block, sorted
 *     lexicographically, with their kept dimensions (> 0).
 *   - Isometries: for every out-sector q of the new bond (in table order) a
 *     row-major matrix with sum_s D_old(q - q(s)) rows stacked in the order
 *     s = 0..3 and D_new(q) orthonormal columns; out-sectors concatenated.
 *     Left site l maps (left block of l sites) x (site l) to the left block
 *     of l+1 sites; right site N-m maps (site N-m) x (right block of m-1
 *     sites) to the right block of m sites.
 *   - Two-site vector layout: row-major blocks D_L(qa) x D_R(qb) for all
 *     (qa, s_k, s_k1) in the order (index of qa, s_k, s_k1) such that
 *     qb = (n_up, n_dn) - qa - q(s_k) - q(s_k1) is a sector of R;
 *     concatenated without padding.  heff_psi_layout() returns it.
 *
 * Error behaviour: every function returns 0 (HEFF_OK) or a negative code;
 * no exception crosses the ABI; heff_last_error() describes the last
 * failure on a context.  Device pointers must be allocated on the context's
 * device; all device work is enqueued on the context's stream.
 */
#ifndef HEFF_H
#define HEFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct heff_ctx heff_ctx;
typedef struct heff_blocks heff_blocks;
typedef struct heff_dav heff_dav;

enum heff_status {
  HEFF_OK = 0,
  HEFF_EINVAL = -1,   /* bad argument, shape, symmetry or layout             */
  HEFF_ESECTOR = -2,  /* the target (n_up, n_dn) sector is empty             */
  HEFF_ENOMEM = -3,   /* device or host allocation failed                     */
  HEFF_EHIP = -4,     /* a HIP runtime call failed                            */
  HEFF_ENOTSUP = -5,  /* precision not built for these blocks                 */
  HEFF_ENOCONV = -6,  /* Davidson breakdown (non-finite or zero correction)   */
  HEFF_ESTATE = -7    /* call out of order (e.g. step after convergence)      */
};

/* Arithmetic of the H_eff product (the rest of the path is FP64). */
enum heff_prec {
  HEFF_FP64 = 0,      /* FP64 operands, FP64 MFMA                             */
  HEFF_FP32 = 1,      /* FP32 operands and accumulation                       */
  HEFF_BF16X3 = 2     /* bf16 hi+lo split: hi*hi + hi*lo + lo*hi, FP32 accum. */
};

typedef struct {
  int32_t n_sect;
  const int32_t* nup;  /* [n_sect] host, block particle numbers (up)   */
  const int32_t* ndn;  /* [n_sect] host                                */
  const int32_t* dim;  /* [n_sect] host, kept dimension, > 0           */
} heff_bond;

typedef struct {
  int32_t n_orb, n_up, n_dn;   /* N >= 4 orbitals, target sector           */
  const double* h;             /* [N*N] host                               */
  const double* V;             /* [N^4] host                               */
  const heff_bond* left;       /* [k0+1]: left block with l = 0..k0 sites  */
  const heff_bond* right;      /* [N-k0-1]: right block with m = 0..N-k0-2 */
  const double* const* iso_left;   /* [k0] host arrays (site l builds l+1) */
  const double* const* iso_right;  /* [N-k0-2] host, entry m-1 builds m    */
} heff_problem;

/* Device memory provider of a context.  alloc(bytes, user) returns device
 * memory of at least `bytes` bytes on the context's device, aligned to 256
 * bytes and usable in stream order on the context's stream, or NULL when it
 * cannot (the call then fails with HEFF_ENOMEM); free(ptr, user) takes back
 * what alloc returned.  Every device buffer the library makes on behalf of a
 * context (operator stores, task tables, Davidson basis, truncation and
 * batch buffers, scratch) comes from it; each object frees through the
 * provider it was made with, also after its context is destroyed, so the
 * callbacks and `user` must stay valid until the last such object is freed.
 * A caching allocator such as PyTorch's can own all device memory this
 * way. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} heff_alloc;

/* Context bound to HIP device `device` and stream `stream` (a hipStream_t,
 * NULL = the null stream).  alloc (copied; may be NULL) is the device
 * memory provider, NULL = hipMalloc / hipFree.  One context per host
 * thread.  HEFF_EINVAL for a provider with a null callback, HEFF_EHIP for a
 * device that does not exist. */
int heff_create(heff_ctx** ctx, int device, void* stream, const heff_alloc* alloc);
int heff_destroy(heff_ctx* ctx);
/* Description of the last error on ctx; valid until the next call on it. */
const char* heff_last_error(const heff_ctx* ctx);

/* Renormalized operators of L and R (the Ren_l / Ren_r recursion over all
 * isometries), the complementary-operator sums and the task table of the
 * two-site product (Sec. II.C).  All inputs are host memory read during
 * the call.  prec_mask: bit (1 << HEFF_FP32) and/or (1 << HEFF_BF16X3)
 * also prepare the FP32 operand copies that both reduced-precision products
 * read (the split-bf16 product splits FP32 values into hi/lo on the fly).
 * Validates the problem first as heff_validate_problem() does (HEFF_EINVAL,
 * HEFF_ESECTOR).  Synchronizes the context stream.  *out is owned by the
 * caller (heff_blocks_free).  The bit HEFF_KEEP_ENV (below, with the sweep
 * step) also keeps the environment of later sweep steps. */
int heff_build_blocks(heff_ctx* ctx, const heff_problem* prob, uint32_t prec_mask,
                      heff_blocks** out);
/* The checks heff_build_blocks makes before any device work, on the host
 * only (no context, no device needed): n_orb in [4, 64], electron numbers,
 * symmetric h and 8-fold symmetric V (1e-12 of the largest entry), sorted
 * bond tables with positive dimensions <= 65535, the empty blocks' single
 * sector (0,0) of dimension 1, no out-sector with more kept than reachable
 * states, orthonormal isometry columns (|M^T M - I| <= 1e-10 over the whole
 * Gram matrix of every out-sector block, Eq. DefinitionMPS of Sec. II.A),
 * and at least one two-site block in the target sector.  Returns HEFF_OK,
 * HEFF_EINVAL or HEFF_ESECTOR; msg (caller-owned, may be NULL) receives a
 * NUL-terminated description of at most msg_len - 1 characters. */
int heff_validate_problem(const heff_problem* prob, char* msg, int32_t msg_len);
int heff_blocks_free(heff_blocks* b);

/* Two-site layout: number of elements and blocks; blk_desc[6*i..] =
 * (qa_up, qa_dn, s_k, s_k1, rows, cols), blk_off[i] = element offset.
 * Arrays are owned by `b`. */
int heff_psi_layout(const heff_blocks* b, int64_t* n_elem, int32_t* n_blk,
                    const int32_t** blk_desc, const int64_t** blk_off);

/* Task-table statistics: tasks per product, algorithmic flops per product
 * (sum over tasks of the cheaper contraction order), algorithmic bytes per
 * product for FP64 / FP32 / BF16X3 operands (each referenced operator
 * block read once + Psi read + Psi' written). bytes may be NULL. */
int heff_task_stats(const heff_blocks* b, int64_t* n_tasks, double* flops, double* bytes3);

/* Kernel timing of heff_apply (per-phase timers): when enabled,
 * every product launch records HIP events on the context stream around each
 * of its kernel-variant launches (variants 0..3 handle output blocks whose
 * width and task middle dimensions are <= 32, 64, 128, 256).  heff_timing() enables (1) or
 * disables (0) recording and clears what was recorded; heff_timing_read()
 * synchronizes the stream, writes per variant the summed milliseconds
 * ms[4] and the number of recorded launches launches[4] since the last
 * clear, then clears.  heff_task_stats_variant() gives the algorithmic
 * flops per product of variant v and its number of work-groups. */
int heff_timing(heff_ctx* ctx, int enable);
int heff_timing_read(heff_ctx* ctx, double* ms, int64_t* launches);
int heff_task_stats_variant(const heff_blocks* b, int v, double* flops, int64_t* work_items);
/* Issue counts of the FP64/FP32 kernel of variant v per product: the flops
 * of the matrix instructions it executes (the algorithmic flops plus the
 * padding of every dimension to the 16-wide instruction tiles) and the
 * number of pipeline steps summed over its work-groups (one step = one
 * 16-wide slice of the inner index of op(L) op(X) or of the rows of op(R))
 * and of its longest work-group (the critical path of the launch). */
int heff_task_stats_issued(const heff_blocks* b, int v, double* mfma_flops, int64_t* steps, int64_t* max_steps);

/* One GPU's share of the product for a product spread over nranks GPUs by
 * output blocks (Sec. II.D, parallelization of the product over devices).
 * Output blocks are assigned, largest algorithmic flops first, to the rank
 * with the least flops so far; afterwards every product on `b` (heff_apply
 * and what calls it: Davidson steps, energies, backward) writes only the
 * output blocks of `rank` and leaves the other elements of `out` untouched,
 * each block with the same task order, hence the same bits, as the full
 * product.  rank in [0, nranks); nranks = 1 restores the full product.
 * While nranks > 1 the calls whose result needs every output element
 * (heff_energy, heff_energy_backward, heff_dav_create, heff_davidson_step)
 * return HEFF_ESTATE.
 * shard_flops (may be NULL) receives this rank's algorithmic flops per
 * product.  heff_task_stats_variant() then reports the rank's work-groups;
 * the flop statistics stay those of the full product.  Synchronizes the
 * context stream; returns HEFF_EINVAL for a bad rank or nranks. */
int heff_blocks_shard(heff_ctx* ctx, heff_blocks* b, int32_t rank, int32_t nranks, double* shard_flops);

/* out = H_eff psi.  psi, out: device arrays of n_elem elements of the
 * precision's storage type (double for FP64, float for FP32 and BF16X3);
 * they must not alias.  Asynchronous on the context stream. */
int heff_apply(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, void* out);

/* diag[i] = H_eff[i,i] (device, n_elem doubles).  Asynchronous. */
int heff_diag(heff_ctx* ctx, const heff_blocks* b, double* diag);

/* Truncation (the SVD step after Diag_H; Sec. II.A keeps the D largest
 * singular values).  Psi (device, n_elem doubles) is reshaped per sector Q'
 * of the enlarged left block L + {k} into M[(s_k, alpha), (s_k+1, beta)];
 * its singular values and left singular vectors come from a block one-sided
 * (Hestenes) Jacobi SVD of M itself in FP64 on the device (rows rotated in
 * pairs of 16-row blocks until mutually orthogonal to 1e-15; singular values
 * are the row norms, which keeps small ones accurate); the d_keep largest
 * over all sectors are kept (ties: sector order, then rank).  The result object
 * holds the kept singular values (descending), the discarded weight (sum of
 * the other squared singular values), the new bond table of the block
 * L + {k} and the new left isometry of site k on the device in the layout of
 * heff_problem (rows stacked by s_k then alpha, columns of each sector in
 * descending order, each signed so its largest-magnitude entry is
 * positive).  Synchronizes the stream. */
typedef struct heff_trunc heff_trunc;
int heff_truncate(heff_ctx* ctx, const heff_blocks* b, const double* psi, int32_t d_keep, heff_trunc** out);
int heff_trunc_info(const heff_trunc* t, int32_t* n_kept, double* discarded, int32_t* n_sect, int64_t* iso_len);
/* sing[n_kept], nup/ndn/dim[n_sect] are caller-owned host arrays; iso_dev is
 * a caller-owned device array of iso_len doubles receiving the isometry
 * (each may be NULL).  Synchronizes the stream. */
int heff_trunc_get(heff_ctx* ctx, const heff_trunc* t, double* sing, int32_t* nup, int32_t* ndn, int32_t* dim,
                   double* iso_dev);
int heff_trunc_free(heff_trunc* t);

/* Sweep step (Sec. II.A: the MPS is optimized bond by bond in sweeps;
 * Sec. IV.A: the SVD, Ren_l and StVec phases around Diag_H).
 *
 * HEFF_KEEP_ENV in the prec_mask of heff_build_blocks() keeps what later
 * sweep steps need: the integrals and the right blocks of every length with
 * their isometries (device memory of the right blocks of all lengths).
 *
 * heff_sweep_right(): from blocks b of the pair (k, k+1) built (or swept to)
 * with HEFF_KEEP_ENV and the optimized two-site vector psi (device, n_elem
 * doubles of b's layout): truncates psi to d_keep states exactly as
 * heff_truncate() does, grows the left block by site k with the truncated
 * isometry (Ren_l), takes the kept right block of one site fewer, and builds
 * the blocks of the pair (k+1, k+2) into *out (terms, task table, operand
 * copies for prec_mask; HEFF_KEEP_ENV is implied: the environment is
 * shared).  The start vector of the new pair (StVec) is the old state
 * expressed in the new two-site basis,
 *   psi'[a', s_k+1, s_k+2, g] = sum A[(s_k, a), a'] psi[a, s_k, s_k+1, b] B[(s_k+2, g), b]
 * (A the truncated isometry, B the right isometry of site k+2); it is held
 * by *out (heff_start_vector).  *trunc_out (may be NULL) receives the
 * truncation result (heff_trunc_info / heff_trunc_get / heff_trunc_free).
 * Errors: HEFF_ESTATE (no kept environment, sharded blocks, or the pair at
 * the right end), HEFF_EINVAL (bad arguments, a kept sector wider than the
 * kernels' 256).  Synchronizes the stream.  *out is freed with
 * heff_blocks_free(); b stays valid.
 *
 * heff_start_vector(): device pointer to the start vector of blocks made by
 * heff_sweep_right() (n_elem doubles of their layout; owned by the blocks);
 * HEFF_ESTATE for blocks built otherwise. */
#define HEFF_KEEP_ENV (1u << 8)
int heff_sweep_right(heff_ctx* ctx, const heff_blocks* b, const double* psi, int32_t d_keep, uint32_t prec_mask,
                     heff_blocks** out, heff_trunc** trunc_out);
int heff_start_vector(const heff_blocks* b, const double** psi);

/* Mode optimization micro-iteration at the pair (Sec. II.B, Fig. microiter):
 * the two orbitals k, k+1 of the pair are rotated by
 * U = exp(theta (E_k,k+1 - E_k+1,k)) (U_kk = U_k+1,k+1 = cos theta,
 * U_k,k+1 = sin theta, U_k+1,k = -sin theta, the identity elsewhere; the same
 * rotation for both spins), new orbitals c'+_i = sum_a U_ai c+_a.
 *
 * heff_rotate_pair(): out = the two-site vector of the same state in the
 * rotated orbitals: exp(-theta K) on the middle index, K = sum_s
 * (c+_ks c_k+1,s - c+_k+1,s c_ks) (psi, out: device, n_elem doubles, no
 * alias).  Synchronizes the stream.
 *
 * heff_pair_entropy(): the half-Renyi entropy S_1/2 = 2 ln Tr sqrt(rho) and
 * the von Neumann entropy S_1 = -Tr rho ln rho of the left part (sites
 * 0..k) of the normalized state psi, from all singular values over the cut
 * (the truncation's SVD); either output may be NULL.
 *
 * heff_optimize_pair(): the angle minimizing S_1/2 of the rotated state
 * (S_1/2 has period pi: 16 angles of [-pi/2, pi/2), then golden-section
 * refinement of the best bracket to 1e-8; one SVD per trial); *theta the
 * angle, out the rotated vector at it, s_before / s_after (may be NULL)
 * S_1/2 at 0 and at theta, n_evals (may be NULL) the trials.
 *
 * heff_rotate_integrals() (host only, no device): h_out = U^T h U and
 * V_out_ijkl = sum U_ai U_bj U_ck U_dl V_abcd for the rotation of the
 * orbital pair (x, y) by theta (h, V as in heff_problem; outputs
 * caller-owned, may not alias the inputs).  Building blocks from the rotated
 * integrals with the same isometries gives an H_eff under which the rotated
 * vector has the energy the old vector had under the old one.
 * Errors: HEFF_EINVAL (null or aliasing arguments, bad indices, non-finite
 * theta). */
int heff_rotate_pair(heff_ctx* ctx, const heff_blocks* b, double theta, const double* psi, double* out);
int heff_pair_entropy(heff_ctx* ctx, const heff_blocks* b, const double* psi, double* s_half, double* s_vn);
int heff_optimize_pair(heff_ctx* ctx, const heff_blocks* b, const double* psi, double* out, double* theta,
                       double* s_before, double* s_after, int32_t* n_evals);
int heff_rotate_integrals(int32_t n, const double* h, const double* V, int32_t x, int32_t y, double theta,
                          double* h_out, double* V_out);

/* Batches: n independent problems (each built with FP32 operands) in one
 * persistent launch per kernel variant, captured once into a HIP graph on
 * an internal stream and replayed (ordered after / before the context
 * stream by events).  x_dev / y_dev are caller-owned concatenated FP32 device
 * vectors (input, output; no alias) of n_total elements where problem i
 * occupies [offsets[i], offsets[i] + n_elem_i) (heff_batch_layout); they and
 * the problems must outlive the batch.  heff_batch_set_grid() sets the
 * persistent work-groups per variant (the autotuner's knob) and drops the
 * captured graph. */
typedef struct heff_batch heff_batch;
int heff_batch_layout(const heff_blocks* const* probs, int32_t n, int64_t* offsets, int64_t* n_total);
int heff_batch_create(heff_ctx* ctx, const heff_blocks* const* probs, int32_t n, float* x_dev, float* y_dev,
                      heff_batch** out);
int heff_batch_io(const heff_batch* b, const int64_t** offsets, int64_t* n_total);
int heff_batch_set_grid(heff_batch* b, const int32_t* grid /* [4] */);
int heff_batch_stats(const heff_batch* b, double* flops, int32_t* grid /* [4] */, int64_t* work_items /* [4] */);
int heff_batch_apply(heff_ctx* ctx, heff_batch* b, int use_graph);
int heff_batch_free(heff_batch* b);

/* Energy and its gradients (the orbital-rotation step of Sec. II.B works
 * with derivatives of the two-site energy at fixed MPS isometries).
 *
 * heff_energy(): *E = <psi|H_eff|psi> (psi: device, n_elem elements of the
 * precision's type; FP64 or FP32 operands; FP64 accumulation of the dot
 * product).  Synchronizes the stream.
 *
 * heff_energy_backward(): reverse mode of E, scaled by gE (the upstream
 * gradient).  dpsi (device, n_elem, may be NULL) = 2 gE H_eff psi.  dL and
 * dR (device, may be NULL) receive dE/d(operator arena entries) of the left
 * and right blocks, each laid out as the concatenation [store | temporaries]
 * of heff_op_arena() (the operands exactly as the product's tasks read them:
 * the renormalized operators of the block and the linear combinations of
 * them that the terms use); entries no task reads are zero.  FP64 or FP32,
 * the same precision for psi and all outputs.  Asynchronous.
 *
 * heff_op_arena(): device pointers and element counts of the four operand
 * arenas [left store, left temporaries, right store, right temporaries] in
 * precision prec (library-owned; valid while the blocks live).
 *
 * heff_kappa_gradient(): g[i] = dE/dkappa_xy for (x, y) = pairs[2i],
 * pairs[2i+1] (host array), where the orbitals are rotated by U = exp(K),
 * K = sum kappa_xy (E_xy - E_yx), h -> U^T h U, V -> (U x U x U x U)^T V,
 * psi (device, FP64) and the isometries of p held fixed.  E is linear in
 * the integrals, so g_xy is computed exactly as E with the first-order
 * integral change of the rotation: one block build and one product per
 * pair.  Synchronizes the stream. */
int heff_energy(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, double* E);
int heff_energy_backward(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, double gE, void* dpsi,
                         void* dL, void* dR);
int heff_op_arena(const heff_blocks* b, int prec, void* ptr[4], int64_t n_elem[4]);

/* heff_energy_noalloc(): heff_energy() for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, result and errors as
 * heff_energy(), computed by the same kernels, but it allocates nothing: its
 * scratch (H psi and the partial sums of the dot product) is one static
 * device array of 48 MiB + 4 KiB per device, held by every device the
 * library runs on until the process ends, so psi may have at most 6291456
 * elements in FP64 and 12582912 in FP32 (HEFF_EINVAL beyond, with a message
 * that names the limit).  The caller passes psi and E only.  All calls on
 * one device share that array and every call overwrites it completely:
 * calls that overlap on one device (several host threads, or contexts on
 * different streams without ordering between them) race and must not be
 * issued.  Product timing (heff_timing) is not recorded by this call.
 * Synchronizes the stream. */
int heff_energy_noalloc(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, double* E);
int heff_kappa_gradient(heff_ctx* ctx, const heff_problem* p, const double* psi, int32_t n_pairs,
                        const int32_t* pairs, double* g);
/* heff_integral_gradient(): the derivatives of E = <psi|H_eff|psi> with
 * respect to the one- and two-electron integrals of Sec. II.A, Eq. Hamiltonian
 * (psi: device, FP64, n_elem of p's two-site layout; isometries of p and
 * psi held fixed), as symmetric tensors on the space of real symmetric
 * integrals: for a symmetric change (dh, dV) of the integrals E changes by
 * sum dh gh + sum dV gV.  gh (host, n_orb^2, row-major) is the spin-summed
 * one-particle density matrix of the two-site state, gV (host, n_orb^4,
 * (ij|kl) order) half its two-particle density matrix averaged over the
 * eightfold index symmetry; either may be NULL to skip it.  E is linear in
 * the integrals, so every orbit of indices costs one block build and one
 * product: n_orb (n_orb + 1) / 2 for gh and about n_orb^4 / 8 for gV
 * (exact; meant for small orbital counts).  Synchronizes the stream.
 * Errors: HEFF_EINVAL (null problem or psi, integrals not symmetric). */
int heff_integral_gradient(heff_ctx* ctx, const heff_problem* p, const double* psi, double* gh, double* gV);

/* heff_set_fp64_kernel(): which kernel family runs this context's FP64
 * products (heff_apply, heff_energy and the Davidson steps): 0 automatic
 * (the default: the LDS-ring kernel when the product has blocks wider than
 * 64, else the register-staged kernel), 1 the register-staged kernel for
 * every width, 2 the ring kernel for every width, 3 the ring kernel for
 * every width with its 16-byte loads switched off (every operand slice
 * moves by dword loads, the path the ring kernel otherwise takes only where
 * a 16-byte load could pass the end of a buffer).  The families compute
 * the same sums in the same order (bitwise identical results); the choice
 * only moves time.  Errors: HEFF_EINVAL (null context, mode outside 0..3). */
int heff_set_fp64_kernel(heff_ctx* ctx, int32_t mode);

/* Davidson eigensolver for the lowest eigenpair of H_eff (the Diag_H step).
 * m_max in [3, 29] basis vectors, restart to {Ritz vector, previous Ritz
 * vector}; converged when ||r|| <= tol*|theta|.  psi0: device, n_elem
 * doubles (copied).  Basis, orthogonalization, subspace eigenproblem and
 * Ritz vector are FP64 on the device; only the product uses `prec`. */
int heff_dav_create(heff_ctx* ctx, const heff_blocks* b, int32_t m_max, double tol,
                    const double* psi0, heff_dav** out);
/* One product plus update.  Returns the Ritz value and residual norm on
 * the host (synchronizes the stream).  HEFF_ESTATE after convergence. */
int heff_davidson_step(heff_ctx* ctx, heff_dav* d, int prec, double* theta, double* resid);
/* Current Ritz vector (device, n_elem doubles, largest |entry| positive). */
int heff_dav_ritz(heff_ctx* ctx, heff_dav* d, double* psi);
int heff_dav_free(heff_dav* d);

/* SU(2) spin-adapted product (Sec. II.C, Eq. Hamilton_act_su2).
 *
 * States are grouped into spin multiplets and operators into irreducible
 * tensor operators stored by their reduced matrix elements, with the
 * Wigner-Eckart convention <j' m'|T^k_q|j m> = <j m; k q|j' m'> <j'||T^k||j>
 * (Condon-Shortley Clebsch-Gordan coefficients).  The two-site space is
 * coupled hierarchically: left block x site k -> gamma, site k+1 x right
 * block -> delta, gamma x delta -> the total spin.  Each Hamiltonian term
 * is the scalar [[O_L x O_k]^S x [O_k1 x O_R]^S]^0 of a left-block operator,
 * two site operators and a right-block operator; it becomes one task per
 * (input block, output block) with the scalar prefactor
 * coef * sign * <k'||O_k||k> <k1'||O_k1||k1> * F_L * F_R * F_T, each F a
 * rescaled Wigner 9j symbol, sqrt((2a'+1)(2b'+1)(2c+1)(2k_c+1)) *
 * {a b c; k_a k_b k_c; a' b' c'}, taken from a lookup table filled on first
 * use.  sign is the Jordan-Wigner sign (-1)^(|O_k| n_l + |O_k1| (n_l + n_k)
 * + |O_R| (n_l + n_k + n_k1)) of the input particle numbers (subsystem
 * order L, k, k+1, R; |O| = 1 for an odd change of the particle number).
 * The tasks run on the same matrix-core kernels as the U(1) product.
 *
 * All spins are doubled integers (two_s = 2 S).  Site multiplets of one
 * spatial orbital: 0 empty (n 0, S 0), 1 doublet (n 1, S 1/2), 2 doubly
 * occupied singlet (n 2, S 0).  Site operators by code: 0 identity, 1
 * creation tensor (a+_{+1/2} = c+_up, a+_{-1/2} = c+_down), 2 annihilation
 * tensor (a~_{+1/2} = c_down, a~_{-1/2} = -c_up), 3 number, 4 spin vector
 * (T_{+1} = -S+/sqrt2, T_0 = S_z, T_{-1} = S-/sqrt2), 5 pair creation
 * c+_up c+_down, 6 pair annihilation c_down c_up; the doubly occupied state
 * is c+_up c+_down |0>.
 *
 * heff_su2_block: one block's multiplet sectors (n[i], two_s[i], dim[i]
 * multiplets, 1 <= dim <= 256, two_s of the parity of n, no repeated
 * (n, two_s)) and its operators (two_k[j] doubled rank, dn[j] change of
 * the particle number, two_k of the parity of dn); n_blk reduced blocks
 * (op blk_op[b], sectors blk_in[b] -> blk_out[b] with n_out = n_in + dn and
 * two_s_out in two_s_in x two_k), each a row-major dim_out x dim_in matrix
 * at data + blk_off[b] (host, copied at creation).  Missing blocks are
 * zero.  heff_su2_problem: both blocks, n_terms terms (term_l / term_r: an
 * operator index or -1 for the identity of the block; term_site_k /
 * term_site_k1: site operator codes; term_two_s: doubled rank S of the
 * coupled left and right parts; term_coef), the total particle number and
 * doubled total spin.  Terms must conserve the particle number and satisfy
 * the triangle rules of their couplings.
 *
 * Reduced two-site vector: row-major blocks dim_l x dim_r for every key
 * (il, mk, two_s_gamma, mk1, ir, two_s_delta) -- left sector, site-k
 * multiplet, doubled spin of left x site k, site-(k+1) multiplet, right
 * sector, doubled spin of site k+1 x right -- with n_l + n_k + n_k1 + n_r =
 * n_tot and two_s_tot in gamma x delta, in lexicographic key order,
 * concatenated.  heff_su2_layout() returns it: desc holds 8 int32 per block
 * (the key, rows, cols), off the element offsets (library-owned).
 *
 * heff_su2_create(): validates the problem on the host (HEFF_EINVAL with a
 * message on any violation, HEFF_ESECTOR if the target space is empty),
 * builds the task table and uploads the operator data; prec_mask as in
 * heff_build_blocks (FP64 always; bits HEFF_FP32 / HEFF_BF16X3 add FP32
 * operand copies).  heff_su2_apply(): out = H psi on the context's stream
 * (device vectors of n_elem elements of the precision's type, no alias).
 * The handle owns the partial sums of the output blocks whose task chains
 * run split over several work-groups (allocated by heff_su2_create), so
 * two products with one handle must not overlap: call them on one stream.
 * Results are deterministic (fixed summation order) but not bitwise equal
 * to an unsplit accumulation.
 * heff_su2_stats(): tasks, algorithmic flops per product (the U(1) count
 * per task) and the number of magnetic-resolved amplitudes the reduced
 * vector stands for at M = S_tot (sum over blocks of rows x cols x the
 * dimension of their M = S_tot subspace, for comparison with a U(1)
 * vector).  heff_su2_factor(): F(a, b, c; k_a, k_b, k_c; a', b', c') for
 * doubled spins two_j[9] in that order (host only, no context). */
typedef struct heff_su2 heff_su2;
typedef struct {
  int32_t n_sect;
  const int32_t* n;
  const int32_t* two_s;
  const int32_t* dim;
  int32_t n_ops;
  const int32_t* two_k;
  const int32_t* dn;
  int64_t n_blk;
  const int32_t* blk_op;
  const int32_t* blk_out;
  const int32_t* blk_in;
  const int64_t* blk_off;
  const double* data;
  int64_t data_len;
} heff_su2_block;
typedef struct {
  heff_su2_block left, right;
  int32_t n_terms;
  const int32_t* term_l;
  const int32_t* term_site_k;
  const int32_t* term_site_k1;
  const int32_t* term_r;
  const int32_t* term_two_s;
  const double* term_coef;
  int32_t n_tot, two_s_tot;
} heff_su2_problem;
int heff_su2_create(heff_ctx* ctx, const heff_su2_problem* p, uint32_t prec_mask, heff_su2** out);
int heff_su2_layout(const heff_su2* h, int64_t* n_elem, int32_t* n_blk, const int32_t** desc, const int64_t** off);
int heff_su2_stats(const heff_su2* h, int64_t* n_tasks, double* flops, double* n_resolved);
int heff_su2_apply(heff_ctx* ctx, const heff_su2* h, int prec, const void* psi, void* out);
int heff_su2_free(heff_su2* h);
int heff_su2_factor(const int32_t two_j[9], double* F);

#ifdef __cplusplus
}
#endif
#endif /* HEFF_H */

/*
 * vbcsr.h -- C ABI of the MI355X (gfx950) variable-block sparse library.
 *
 * The library applies an atom-centred block-sparse operator A to dense
 * multi-vectors.  Atom i carries b_i orbitals; a stored coupling (i, j) is a
 * dense b_i x b_j block (paper, section 2.1).  Scalar row offsets are
 * off_0 = 0, off_{i+1} = off_i + b_i and N = off_n.  The structure is given
 * once (block sizes, block row pointers, block column indices -- the atom
 * graph of section 3.1 for one rank) and values may be replaced later.
 *
 * Layout conventions (readings of the paper, which does not fix them):
 *   - input/output block values are in graph (CSR) order, each block
 *     row-major (section 3.2 states row-major dense blocks for the products);
 *   - dense multi-vectors are row-major N x nrhs arrays with a leading
 *     dimension ld >= nrhs (element (r, c) at r*ld + c), in device memory;
 *   - FP64 handles take double vectors, FP32 and BF16X3 handles take float.
 *
 * Errors: every call returns a status (VBCSR_OK or a negative code) and
 * records a message readable through vbcsr_last_error() on the calling
 * thread.  All argument validation happens on the host before any HIP call
 * (vbcsr_spgemm copies the two handles' block sizes back to compare them,
 * before any kernel runs).
 * Asynchronous device faults are reported as VBCSR_EHIP by a later call.
 * No C++ exception crosses this interface: a failed host allocation is
 * VBCSR_ENOMEM, and host worker threads that cannot be started leave their
 * work to the others.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Products
 * are enqueued asynchronously; the library synchronises the device only in
 * vbcsr_create, vbcsr_set_values (host input), vbcsr_cheb_moments(_doubled),
 * vbcsr_spgemm, vbcsr_get_structure and vbcsr_destroy.  A handle is immutable except through
 * vbcsr_set_values, vbcsr_use_pages and vbcsr_refresh_transposed;
 * products on different streams may run concurrently on one handle, but
 * must not overlap a vbcsr_set_values on it.
 */
#ifndef VBCSR_H
#define VBCSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vbcsr_mat vbcsr_mat; /* opaque, owned by the library */

typedef enum {
  VBCSR_FP64 = 0,   /* FP64 values and vectors, FP64 arithmetic                  */
  VBCSR_FP32 = 1,   /* values rounded to FP32, FP32 vectors, FP32 accumulation    */
  VBCSR_BF16X3 = 2  /* FP32-rounded values split a = hi + lo (two BF16 each);
                       a*x ~ hi*xh + hi*xl + lo*xh on matrix cores, FP32
                       accumulation, FP32 vectors                                  */
} vbcsr_prec;

enum {
  VBCSR_OK = 0,
  VBCSR_EINVAL = -1,       /* malformed argument (null pointer, bad index, ld < nrhs ...) */
  VBCSR_ESHAPE = -2,       /* n_values does not equal sum over blocks of b_i*b_j        */
  VBCSR_EDUP = -3,         /* a block (i, j) appears twice in one row                   */
  VBCSR_ENOMEM = -4,       /* device or host allocation failed                          */
  VBCSR_EHIP = -5,         /* HIP runtime error (message holds hipGetErrorString)       */
  VBCSR_EUNSUPPORTED = -6  /* valid but outside what this library handles               */
};

enum { VBCSR_PATH_AUTO = 0, VBCSR_PATH_VEC = 1, VBCSR_PATH_MFMA = 2 };
enum { VBCSR_ORDER_AUTO = 0, VBCSR_ORDER_ATOM = 1, VBCSR_ORDER_RCM = 2, VBCSR_ORDER_CLUSTER = 3 };

/* Planner options; zero fields mean "choose automatically".
 *   path:        VBCSR_PATH_* -- force the vector-FMA or the matrix-core
 *                kernel family for FP64/FP32 (BF16X3 always uses matrix cores);
 *                the environment variable VBCSR_PATH={auto,vec,mfma} overrides.
 *   nrhs_tile:   columns per pass of the vector kernel (1, 2, 4 or 8).
 *   rows_per_wg: reserved, must be 0.
 *   row_order:   VBCSR_ORDER_* -- order in which the device lays out and
 *                processes the block rows (and block columns, for the
 *                adjoint): atom order; reverse Cuthill-McKee of the
 *                symmetrised block graph; or clusters of 256 atoms grown
 *                breadth-first over that graph, each seeded next to the
 *                previous one, so that the panels processed together gather
 *                the input rows of one compact cluster and its halo while
 *                they are in cache.  AUTO is the clustered order.  Product
 *                and SDDMM results do not depend on the order (each output
 *                has one writer, which sums its row over the panel's columns
 *                in the same order whatever the processing order); moments
 *                of the Chebyshev helpers are reduced in the processing
 *                order, so they agree up to rounding.                         */
typedef struct {
  int32_t rows_per_wg;
  int32_t nrhs_tile;
  int32_t path;
  int32_t row_order;
} vbcsr_plan_opts;

/* Largest block size (orbitals per atom) this library accepts. */
#define VBCSR_MAX_BLOCK 64

/*
 * vbcsr_create -- build a device operator from a block graph and values.
 * Paper: section 3.1 (atom graph, block size per node), section 3.2
 * (shape classes registered from the distinct (b_i, b_j); every block mapped
 * to its place in the value storage of its shape class).
 *
 *   out          receives the new handle (set to NULL on failure)
 *   n_atoms      number of atoms n >= 0 (rows and columns of the block graph)
 *   block_sizes  host [n_atoms], 1 <= b_i <= VBCSR_MAX_BLOCK
 *   row_ptr      host [n_atoms+1], block units, row_ptr[0] = 0, non-decreasing
 *   col_idx      host [row_ptr[n]], 0 <= j < n, unique within a row, any order
 *   values       host, graph order, each block row-major (double); NULL = zeros
 *   n_values     must equal sum over blocks of b_i*b_j
 *   prec         storage/compute precision of the handle
 *   opts         may be NULL
 *   stream       stream used for the initial upload (synchronised before return)
 *
 * The caller keeps ownership of every input array; the library deep-copies.
 * Errors: EINVAL, ESHAPE, EDUP, EUNSUPPORTED (b_i > VBCSR_MAX_BLOCK,
 * N > 2^31-1, or one block row or block column with 2^28 or more values),
 * ENOMEM, EHIP.
 */
int vbcsr_create(vbcsr_mat **out, int32_t n_atoms, const int32_t *block_sizes,
                 const int64_t *row_ptr, const int32_t *col_idx, const double *values,
                 int64_t n_values, vbcsr_prec prec, const vbcsr_plan_opts *opts, void *stream);

/*
 * vbcsr_create_local -- the rank-local operator of a distributed block graph.
 * Paper: section 3.1 (each rank owns a set of atoms and stores their block
 * rows; the columns they reference are owned atoms or ghosts, the ghosts
 * ordered by owner rank and then by global id) and section 3.2 (the forward
 * product first fetches the ghost rows of X; the adjoint returns the
 * contributions of ghost columns to their owners).
 *
 * Local atom ids: 0 .. n_owned-1 are the owned atoms (block rows),
 * n_owned .. n_owned+n_ghost-1 the ghosts (columns only).  Scalar offsets
 * run over all local atoms, so N_rows = off_{n_owned} (owned scalar rows)
 * and N = off_{n_owned+n_ghost} (owned + ghost scalar rows).
 *   block_sizes  host [n_owned + n_ghost]
 *   row_ptr      host [n_owned + 1]
 *   col_idx      host, local column ids in [0, n_owned + n_ghost)
 *   values, n_values, prec, opts, stream as vbcsr_create
 * Products on such a handle (A is N_rows x N):
 *   vbcsr_spmm    X: N x nrhs (owned rows, then the ghost rows received from
 *                 their owners), Y: N_rows x nrhs;
 *   vbcsr_spmm_t  X: N_rows x nrhs, Y: N x nrhs -- rows below N_rows are the
 *                 owned atoms' results, the rest the ghost columns'
 *                 contributions, to be returned to their owners and added
 *                 there (vbcsr_halo_pack / vbcsr_halo_reduce);
 *   vbcsr_sddmm   dY: N_rows x nrhs, X: N x nrhs.
 * The Chebyshev helpers and vbcsr_spgemm need square operators and return
 * VBCSR_EUNSUPPORTED for a rank-local one.  vbcsr_info reports n_rows =
 * N_rows; vbcsr_get_structure returns n_owned + 1 row pointers and
 * n_owned + n_ghost block sizes; vbcsr_shape gives both dimensions.
 * Errors: as vbcsr_create (every column id is checked against
 * n_owned + n_ghost).
 */
int vbcsr_create_local(vbcsr_mat **out, int32_t n_owned, int32_t n_ghost,
                       const int32_t *block_sizes, const int64_t *row_ptr, const int32_t *col_idx,
                       const double *values, int64_t n_values, vbcsr_prec prec,
                       const vbcsr_plan_opts *opts, void *stream);

/*
 * vbcsr_shape -- (library utility) the handle's dimensions: block rows and
 * block columns (atoms), scalar rows N_rows and scalar columns N.  Square
 * handles have equal pairs.  Any output may be NULL.
 */
int vbcsr_shape(const vbcsr_mat *A, int32_t *n_row_atoms, int32_t *n_col_atoms, int64_t *n_rows,
                int64_t *n_cols);

/*
 * vbcsr_set_values -- replace all block values, same structure.
 * No passage of the paper defines this call: it is the library's way of
 * changing the operator's entries between products (the differentiation
 * form updates them every step).
 *   values     n_values entries in graph order, each block row-major
 *   on_device  0: host pointer (copied, synchronises `stream`);
 *              1: device pointer (read by a kernel on `stream`; no sync)
 *   dtype      0 = double, 1 = float
 * Errors: EINVAL, ENOMEM, EHIP.
 */
int vbcsr_set_values(vbcsr_mat *A, const void *values, int on_device, int dtype, void *stream);

/*
 * vbcsr_spmm -- Y <- alpha * A * X + beta * Y.
 * Paper: section 3.2, forward product: Y_i accumulates A_ij X_j over the
 * stored columns j of block row i.
 *   X   device, N x nrhs, leading dimension ldx >= nrhs, read only
 *   Y   device, N x nrhs, leading dimension ldy >= nrhs
 *   beta == 0 means Y is not read (NaNs in Y are ignored); an empty block row
 *   gives Y_i = beta * Y_i.  X and Y must not overlap.
 * Errors: EINVAL (null pointers, nrhs <= 0, ld < nrhs, overlap), EHIP.
 */
int vbcsr_spmm(const vbcsr_mat *A, const void *X, int64_t ldx, void *Y, int64_t ldy,
               int32_t nrhs, double alpha, double beta, void *stream);

/*
 * vbcsr_spmm_t -- Y <- alpha * A^T * X + beta * Y.
 * Paper: equation (1), the adjoint product Y_j += A_ij^dagger X_i for
 * j in J(i); values are real, so the adjoint is the transpose.  Arguments
 * and errors as vbcsr_spmm.  No atomics: every output row has one writer.
 */
int vbcsr_spmm_t(const vbcsr_mat *A, const void *X, int64_t ldx, void *Y, int64_t ldy,
                 int32_t nrhs, double alpha, double beta, void *stream);

/*
 * vbcsr_sddmm -- dA_ij = dY_i * X_j^T on the stored blocks only.
 * This is the gradient of sum(Y o G) with respect to the stored block values
 * when Y = A X and dY = G (with dX = A^T G from vbcsr_spmm_t).
 *   dY  device, N x nrhs, leading dimension lddy >= nrhs
 *   X   device, N x nrhs, leading dimension ldx >= nrhs
 *   dA  device, n_values entries, graph order, each block row-major; double
 *       for FP64 handles, float otherwise.  Must not overlap dY or X.
 * Errors: EINVAL, EHIP.
 */
int vbcsr_sddmm(const vbcsr_mat *A, const void *dY, int64_t lddy, const void *X, int64_t ldx,
                int32_t nrhs, void *dA, void *stream);

/*
 * Page-layout values (FP64 and FP32 handles).  No passage of the paper
 * defines these calls: they let a caller that differentiates with respect
 * to the block values (vbcsr_sddmm) keep that parameter in the operator's
 * own forward-page layout, so a training step repacks nothing for the
 * forward product and rebuilds only the transposed pages for the adjoint.  A page buffer holds
 * vbcsr_page_size() entries of the handle's value type: every block value at
 * its forward-page position, zeros in the alignment gaps between panels and
 * in the slack after the last (the products read those as zeros).
 *
 * vbcsr_page_size -- entries of a page buffer.
 * vbcsr_get_pages -- copy the current forward values, page layout, into the
 *   device buffer `pages` (on `stream`).
 * vbcsr_use_pages -- from now on the forward products (vbcsr_spmm, the
 *   Chebyshev helpers, vbcsr_get_values, the block product's B) read the
 *   forward values from the caller's device buffer `pages`, which is not
 *   copied: it must stay allocated and keep the layout above while in use.
 *   NULL returns to the handle's own pages (as the last vbcsr_create or
 *   vbcsr_set_values left them).  Either way the transposed pages become
 *   stale: vbcsr_spmm_t, and vbcsr_spgemm with this handle as A, return
 *   EINVAL until vbcsr_refresh_transposed.  vbcsr_set_values returns to the
 *   handle's own pages and rewrites both page sets.  Changes the handle: no
 *   product may run on it meanwhile.  No device work.
 * vbcsr_refresh_transposed -- rebuild the transposed pages from the current
 *   forward values (a kernel on `stream`); call it again after changing the
 *   contents of a buffer in use.  The first call on a handle also sorts its
 *   blocks into transposed-page order (kept with the handle) and
 *   synchronises `stream`.
 * vbcsr_sddmm_pages -- vbcsr_sddmm with dA written in the page layout:
 *   dA receives vbcsr_page_size() entries (values at their forward-page
 *   positions, zeros in the gaps and the slack), the gradient of the page
 *   buffer when the forward product reads its values from it.
 * Errors: EINVAL (null arguments, bad vectors, overlap), EUNSUPPORTED
 * (BF16X3 handles), EHIP.
 */
int vbcsr_page_size(const vbcsr_mat *A, int64_t *n_page_values);
int vbcsr_get_pages(const vbcsr_mat *A, void *pages, void *stream);
int vbcsr_use_pages(vbcsr_mat *A, const void *pages);
int vbcsr_refresh_transposed(vbcsr_mat *A, void *stream);
int vbcsr_sddmm_pages(const vbcsr_mat *A, const void *dY, int64_t lddy, const void *X,
                      int64_t ldx, int32_t nrhs, void *dA, void *stream);

/*
 * vbcsr_cheb_workspace_bytes -- device workspace, in bytes, that
 * vbcsr_cheb_moments needs for this handle, nrhs and degree: two N x nrhs
 * recurrence vectors, per-workgroup FP64 partial moments and the moments.
 * Errors: EINVAL.
 */
int vbcsr_cheb_workspace_bytes(const vbcsr_mat *A, int32_t nrhs, int32_t degree, int64_t *bytes);

/*
 * vbcsr_cheb_moments -- Chebyshev moments of the kernel polynomial method
 * (paper, section 5): with T_0 = R, T_1 = A R, T_{k+1} = 2 A T_k - T_{k-1},
 *   mu_host[k*nrhs + c] = sum_r R[r, c] * T_k[r, c],   k = 0..degree,
 * each moment accumulated in FP64 in a fixed order (bitwise reproducible).
 * A must already be scaled so that its spectrum lies in [-1, 1].  The vectors
 * T_k are kept in the handle's vector type (double or float).
 *   R          device, N x nrhs, leading dimension ldr >= nrhs
 *   degree     >= 0
 *   mu_host    host, (degree+1)*nrhs doubles
 *   workspace  device, >= vbcsr_cheb_workspace_bytes() bytes, 256-byte aligned;
 *              NULL = allocate (and free) it inside the call; must not
 *              overlap R
 * The signature adds the leading dimension ldr of R to the one the operation
 * needs (A, R, nrhs, degree, moments): R may be a column slice of a wider
 * array.
 * Synchronises `stream` (copies the moments to the host).
 * Errors: EINVAL, ENOMEM, EHIP.
 */
int vbcsr_cheb_moments(const vbcsr_mat *A, const void *R, int64_t ldr, int32_t nrhs,
                       int32_t degree, double *mu_host, void *workspace, int64_t ws_bytes,
                       void *stream);

/*
 * vbcsr_cheb_moments_doubled -- the same moments as vbcsr_cheb_moments from
 * about half the operator applications, for a symmetric A (A_ji = A_ij^T,
 * the case of the Hamiltonians of section 5).  From the Chebyshev product
 * identity 2 T_m T_n = T_{m+n} + T_{|m-n|} and the symmetry of T_k(A):
 *   mu_2k   = 2 <T_k R, T_k R>     - mu_0
 *   mu_2k+1 = 2 <T_k R, T_{k+1} R> - mu_1
 * so only T_1 .. T_ceil(degree/2) are formed.  The inner products are FP64
 * sums in a fixed order (the second one fused into the product's epilogue,
 * the first a column dot product); the combination above is done in FP64 on
 * the host.  For a non-symmetric A the result is not the moment sequence.
 * Arguments, workspace, synchronisation and errors as vbcsr_cheb_moments.
 */
int vbcsr_cheb_moments_doubled(const vbcsr_mat *A, const void *R, int64_t ldr, int32_t nrhs,
                               int32_t degree, double *mu_host, void *workspace,
                               int64_t ws_bytes, void *stream);

/*
 * vbcsr_cheb_step -- one step of the Chebyshev recurrence of section 5 with
 * its moment, for callers that drive the recurrence themselves:
 *   T_next = 2 A T_k - T_prev      (written over T_prev, in place)
 *   mu_dev[c] = sum_r R[r, c] * T_next[r, c]   (FP64, fixed order)
 *   Tk         device, N x nrhs, leading dimension ldt >= nrhs, read only
 *   Tprev      device, N x nrhs, leading dimension ldp >= nrhs; on return it
 *              holds T_next.  Must not overlap Tk.
 *   R          device, N x nrhs, leading dimension ldr >= nrhs
 *   mu_dev     device, nrhs doubles
 *   workspace  device, >= vbcsr_cheb_workspace_bytes(A, nrhs, 0) bytes
 * R must not overlap Tprev (the epilogue writes T_next and then reads R at
 * the same element); the workspace and mu_dev must not overlap each other
 * or any of the three vectors.
 * Asynchronous on `stream` (no synchronisation).
 * Errors: EINVAL, EHIP.
 */
int vbcsr_cheb_step(const vbcsr_mat *A, const void *Tk, int64_t ldt, void *Tprev, int64_t ldp,
                    const void *R, int64_t ldr, int32_t nrhs, double *mu_dev, void *workspace,
                    int64_t ws_bytes, void *stream);

/* Size of the device scratch behind vbcsr_cheb_step_noalloc, per GPU. */
#define VBCSR_NOALLOC_SCRATCH_BYTES (32u << 20)

/*
 * vbcsr_cheb_step_noalloc -- vbcsr_cheb_step without any device allocation
 * and without a workspace argument, for callers that cannot allocate: code
 * under HIP graph capture, tight serving or solver loops, harnesses that
 * forbid hipMalloc.  Same operation, arguments (minus the workspace), results
 * (bitwise) and errors as vbcsr_cheb_step.
 * The per-workgroup partial moments go to a scratch array inside the
 * library: one VBCSR_NOALLOC_SCRATCH_BYTES array per GPU, held from the
 * library's load until the process ends.  The call needs
 * 8 * ceil(n_atoms / 4) * nrhs bytes of it and fails with
 * VBCSR_EUNSUPPORTED beyond that (e.g. n_atoms = 199,911 allows nrhs <= 83).
 * Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's partials: calls that overlap in time on one GPU (other streams or
 * threads) race and must be serialised by the caller.  Nothing in the
 * scratch needs clearing between calls (each call writes all the partials
 * it reads).  No hipMalloc, hipFree or allocating routine is called.
 */
int vbcsr_cheb_step_noalloc(const vbcsr_mat *A, const void *Tk, int64_t ldt, void *Tprev,
                            int64_t ldp, const void *R, int64_t ldr, int32_t nrhs, double *mu_dev,
                            void *stream);

/*
 * vbcsr_info -- (a library utility; no passage of the paper defines it)
 * sizes of a handle: n_rows = N_rows (scalar rows of a forward product's
 * output: N for a square handle), nnzb stored
 * blocks, n_values = sum of b_i*b_j, n_shapes = distinct (b_i, b_j) classes.
 * Any output pointer may be NULL.
 */
int vbcsr_info(const vbcsr_mat *A, int64_t *n_rows, int64_t *nnzb, int64_t *n_values,
               int32_t *n_shapes);

/*
 * vbcsr_plan_host -- run validation and the host planner without a device
 * (diagnostics and tests).  Inputs as vbcsr_create.
 *   shapes       out, up to max_shapes triples (b_i, b_j, count) in ascending
 *                (b_i, b_j); *n_shapes receives the total number of classes
 *   fwd_pos      out [nnzb] or NULL: offset, in the forward value pages, of the
 *                first value of every graph-order block
 *   tr_pos       out [nnzb] or NULL: the same for the transposed pages
 *   page_values  out or NULL: number of values in the forward pages
 *   opts         may be NULL (row_order is the only field used)
 * Errors: as vbcsr_create, minus device errors.
 */
int vbcsr_plan_host(int32_t n_atoms, const int32_t *block_sizes, const int64_t *row_ptr,
                    const int32_t *col_idx, int64_t n_values, int32_t *n_shapes,
                    int32_t *shapes, int32_t max_shapes, int64_t *fwd_pos, int64_t *tr_pos,
                    int64_t *page_values, const vbcsr_plan_opts *opts);

/*
 * vbcsr_get_structure -- copy the block graph of a handle to the host.
 *   block_sizes  out [n_col_atoms]; row_ptr out [n_row_atoms+1]; col_idx out
 *   [nnzb] (sizes from vbcsr_shape and vbcsr_info; both atom counts are
 *   n_atoms for a square handle).  Synchronous.
 * Errors: EINVAL (null handle or output), EHIP.
 */
int vbcsr_get_structure(const vbcsr_mat *A, int32_t *block_sizes, int64_t *row_ptr,
                        int32_t *col_idx);

/*
 * vbcsr_get_values -- the handle's block values in graph order, each block
 * row-major (the layout vbcsr_create takes), written by a kernel on `stream`.
 *   values  device, n_values elements of the handle's type
 *   dtype   0 = double (FP64 handles), 1 = float (FP32 handles)
 * Errors: EINVAL, EUNSUPPORTED (BF16X3 handles keep only the split pages), EHIP.
 */
int vbcsr_get_values(const vbcsr_mat *A, void *values, int dtype, void *stream);

/* Counts and phase times of one vbcsr_spgemm call. */
typedef struct {
  int64_t candidates;    /* distinct (i, j) reached through some k               */
  int64_t kept_symbolic; /* candidates whose bound is not below eps              */
  int64_t nnzb;          /* blocks of C after the final filter                   */
  int64_t products;      /* block products A_ik B_kj evaluated                   */
  double flops;          /* sum over evaluated products of 2 b_i b_k b_j         */
  double ms_norms;       /* block sizes copy-back and block norms of A and B    */
  double ms_symbolic;    /* device symbolic stage                               */
  double ms_numeric;     /* numeric kernel (device events around it)            */
  double ms_filter;      /* final filter (device compaction)                    */
  double ms_build;       /* planning (device or host) and packing of C          */
} vbcsr_spgemm_stats;

/*
 * vbcsr_spgemm -- thresholded block product C = A B.
 * Paper: section 3.2, equation 2 (C_ij = sum_k A_ik B_kj) and equation 3
 * (||C_ij|| <= sum_k ||A_ik|| ||B_kj||).  Stages:
 *   1. block norms of A and B (Frobenius, on the device; only when eps > 0);
 *   2. symbolic stage on the device: the candidates of row i are the columns
 *      j of the rows k of B with a block (i, k) in A; a candidate is rejected
 *      when U_ij = sum_k ||A_ik|| ||B_kj|| (summed over k in A's stored order,
 *      each product and sum rounded separately) is below eps.  Kept columns
 *      are ascending in every row of C;
 *   3. numeric stage on the device, one wave per output block: the products
 *      A_ik B_kj of the block in A's stored order of k, on matrix cores, FP64;
 *   4. final filter on the device: computed blocks whose Frobenius norm is
 *      below eps are removed (nothing is removed at eps = 0);
 *   5. C is laid out and packed like a vbcsr_create result.  With row order
 *      VBCSR_ORDER_AUTO (or opts NULL) C's panels are processed in A's
 *      processing order, with VBCSR_ORDER_ATOM in atom order; both layouts
 *      are computed on the device from the pattern already there.  RCM and
 *      cluster orders of C's own graph are computed by the host planner
 *      (C's pattern is then copied back).
 *      The order changes no result of any product with C.
 *   out     receives the new FP64 handle C over the same atoms (NULL on failure)
 *   A, B    FP64 handles over the same atoms (same block sizes)
 *   eps     block-norm threshold, >= 0
 *   opts    planner options of C (may be NULL)
 *   stats   may be NULL
 * Synchronises `stream`.
 * Errors: EINVAL (null arguments, different atoms, eps < 0 or NaN, bad
 * options), EUNSUPPORTED (non-FP64 handles, 2^31 or more candidate block
 * products, or C outside vbcsr_create's limits), ENOMEM, EHIP.
 */
int vbcsr_spgemm(vbcsr_mat **out, const vbcsr_mat *A, const vbcsr_mat *B, double eps,
                 const vbcsr_plan_opts *opts, vbcsr_spgemm_stats *stats, void *stream);

/* Damping kernels of the kernel polynomial method. */
enum { VBCSR_KPM_NONE = 0, VBCSR_KPM_JACKSON = 1 };

/*
 * vbcsr_kpm_dos -- density of states from Chebyshev moments (paper, section
 * 5: the KPM with a damping kernel).  With M = n_moments and g_k = 1 (NONE)
 * or the Jackson factors
 *   g_k = [(M-k+1) cos(pi k/(M+1)) + sin(pi k/(M+1)) cot(pi/(M+1))] / (M+1),
 *   rho[i] = [g_0 mu_0 + 2 sum_{k=1}^{M-1} g_k mu_k T_k(x_i)] / (pi sqrt(1 - x_i^2)),
 * the series summed per point by Clenshaw's recurrence in FP64.  For the
 * density per state, mu_k are the moments divided by (number of states x
 * number of random vectors), e.g. averaged vbcsr_cheb_moments output / N.
 *   mu    device, n_moments doubles (n_moments >= 1)
 *   x     device, npts points of the scaled axis, |x| < 1 (|x| >= 1 gives
 *         non-finite rho)
 *   rho   device, npts doubles (must not overlap x)
 *   work  device, n_moments doubles for the damped coefficients, or NULL
 *         (allocated in the call; the call then synchronises `stream`)
 * Asynchronous on `stream` when `work` is given.
 * Errors: EINVAL, ENOMEM, EHIP.
 */
int vbcsr_kpm_dos(const double *mu, int32_t n_moments, int32_t damping, const double *x,
                  int64_t npts, double *rho, double *work, void *stream);

/*
 * vbcsr_kpm_threshold -- the density threshold of the gap estimate (paper,
 * section 5: a threshold tied to the KPM resolution): `fraction` of the peak
 * height of one state of weight 1/n_states broadened by a Gaussian of the
 * kernel width sigma = pi / n_moments (scaled axis),
 *   threshold = fraction / (n_states * sigma * sqrt(2 pi)).
 * Host only.  Errors: EINVAL.
 */
int vbcsr_kpm_threshold(int32_t n_moments, int64_t n_states, double fraction, double *threshold);

/*
 * vbcsr_kpm_gap -- the low-density interval: among runs of consecutive
 * points with rho < threshold that have a point with rho >= threshold on both
 * sides, the one whose bounding points are farthest apart; *lo and *hi
 * receive those two bounding abscissae (NaN when there is no such run).
 *   x, rho  host, npts values, x strictly ascending
 * Host only.  Errors: EINVAL.
 */
int vbcsr_kpm_gap(const double *x, const double *rho, int64_t npts, double threshold, double *lo,
                  double *hi);

/* ---------------------------------------------------------------------------
 * Halo exchange of rank-local operators (paper, sections 3.1 and 3.2).
 * A halo plan describes one rank's share of a distributed block graph: its
 * owned atoms (ascending global id), its ghosts (ordered by owner rank, then
 * global id), the local graph for vbcsr_create_local, and the exchange
 * lists.  Every list is in local scalar rows:
 *   send buffer  rows send_ptr[s] .. send_ptr[s+1] go to rank s: the scalar
 *                rows of the owned atoms that rank s's rows reference, in
 *                ascending global id -- exactly the order of rank s's ghost
 *                rows from this rank, so a received segment is copied
 *                unchanged into the ghost rows;
 *   receive      the ghost rows from owner s are local scalar rows
 *                N_rows + recv_ptr[s] .. N_rows + recv_ptr[s+1];
 *   adjoint      the ghost rows of a vbcsr_spmm_t result are returned the
 *                same way (owner s receives rows N_rows + recv_ptr[s] ..),
 *                arriving in the layout of this rank's send buffer; the
 *                reduction map lists, per owned scalar row red_rows[u], the
 *                buffer rows red_pos[red_ptr[u] .. red_ptr[u+1]) (ascending,
 *                i.e. rank order) that add into it.
 * The plan is computed on the host from the whole graph (here every rank's
 * share lives in one process); the transport between ranks is the
 * caller's (device copies on one GPU, or point-to-point messages).
 * ------------------------------------------------------------------------- */
typedef struct vbcsr_halo vbcsr_halo; /* opaque, host-side, owned by the library */

/*
 * vbcsr_halo_create -- the plan of rank `rank` of `n_ranks`.
 *   n_global, block_sizes, row_ptr, col_idx  the global block graph (as
 *            vbcsr_create takes it; values are not needed)
 *   owner    host [n_global], owning rank of every atom, in [0, n_ranks)
 * Host only.  Errors: EINVAL, EDUP, EUNSUPPORTED (as vbcsr_create's
 * validation), ENOMEM.
 */
int vbcsr_halo_create(vbcsr_halo **out, int32_t n_global, const int32_t *block_sizes,
                      const int64_t *row_ptr, const int32_t *col_idx, const int32_t *owner,
                      int32_t rank, int32_t n_ranks);

/* vbcsr_halo_info -- sizes: owned and ghost atoms, local blocks and values,
 * rows of the send buffer, rows of the reduction map.  Outputs may be NULL. */
int vbcsr_halo_info(const vbcsr_halo *H, int32_t *n_owned, int32_t *n_ghost, int64_t *nnzb,
                    int64_t *n_values, int64_t *n_send_rows, int64_t *n_red_rows);

/* vbcsr_halo_graph -- the local graph: gid [n_owned+n_ghost] global id of
 * every local atom, block_sizes [n_owned+n_ghost], row_ptr [n_owned+1],
 * col_idx [nnzb] (local ids; each row keeps the global order of its blocks).
 * Outputs may be NULL. */
int vbcsr_halo_graph(const vbcsr_halo *H, int32_t *gid, int32_t *block_sizes, int64_t *row_ptr,
                     int32_t *col_idx);

/* vbcsr_halo_local_values -- the owned rows' block values (local graph
 * order) from the global graph-order values; host arrays. */
int vbcsr_halo_local_values(const vbcsr_halo *H, const double *global_values, double *local_values);

/* vbcsr_halo_lists -- send_ptr [n_ranks+1], send_rows [n_send_rows],
 * recv_ptr [n_ranks+1], red_rows [n_red_rows], red_ptr [n_red_rows+1],
 * red_pos [n_send_rows] (host arrays, any may be NULL); see above. */
int vbcsr_halo_lists(const vbcsr_halo *H, int64_t *send_ptr, int32_t *send_rows, int64_t *recv_ptr,
                     int32_t *red_rows, int64_t *red_ptr, int64_t *red_pos);

/* vbcsr_halo_destroy -- free a plan (NULL is ignored). */
void vbcsr_halo_destroy(vbcsr_halo *H);

/*
 * vbcsr_halo_pack -- fill a send buffer on the device:
 *   buf[t*ldb + c] = X[rows[t]*ldx + c],  t < nrows, c < nrhs
 *   X     device, x_rows x nrhs (leading dimension ldx)
 *   rows  device [nrows] scalar rows of X (e.g. the send rows); a row outside
 *         [0, x_rows) is skipped (its buffer row is not written)
 *   dtype 0 = double, 1 = float;  buf device, nrows x nrhs (ldb), must not
 *         overlap X
 * Asynchronous on `stream`.  Errors: EINVAL, EHIP.
 */
int vbcsr_halo_pack(const void *X, int64_t x_rows, int64_t ldx, const int32_t *rows,
                    int64_t nrows, int32_t nrhs, int32_t dtype, void *buf, int64_t ldb,
                    void *stream);

/*
 * vbcsr_halo_reduce -- add returned adjoint contributions to their rows:
 *   Y[red_rows[u]*ldy + c] += sum over e in [red_ptr[u], red_ptr[u+1]) of
 *                             buf[red_pos[e]*ldb + c]
 * summed in e order, one writer per element (no atomics; bitwise
 * reproducible).  red_rows must be distinct (the plan's are).
 *   Y         device, y_rows x nrhs (ldy);  buf device, buf_rows x nrhs (ldb)
 *   red_rows, red_ptr, red_pos  device arrays (the plan's reduction map);
 *             indices outside Y or the buffer are skipped
 * Asynchronous on `stream`.  Errors: EINVAL, EHIP.
 */
int vbcsr_halo_reduce(void *Y, int64_t y_rows, int64_t ldy, const int32_t *red_rows,
                      const int64_t *red_ptr, const int64_t *red_pos, int64_t n_red,
                      const void *buf, int64_t buf_rows, int64_t ldb, int32_t nrhs, int32_t dtype,
                      void *stream);

/* ---------------------------------------------------------------------------
 * Reciprocal-space (k-sampled) operators.
 * Paper, section 3.3, equation 4: a periodic real-space operator is a set of
 * images O(R), one per integer lattice translation R, over the atoms of one
 * cell; sampling a point k (given in units of the reciprocal lattice vectors) gives the
 * complex block-sparse operator
 *     O(k) = sum_R exp(-2 pi i k.R) O(R)                      (VBCSR_PHASE_R)
 * or, in the alternative convention, block (i, j) of image R multiplied by
 * exp(-2 pi i k.(R + tau_j - tau_i))                        (VBCSR_PHASE_R_TAU)
 * with tau the atoms' fractional positions.  Blocks (i, j) of different
 * images add into one block of O(k).  Complex vectors are interleaved
 * (re, im) pairs: double for FP64 handles, float for FP32 handles; leading
 * dimensions count complex elements.
 * ------------------------------------------------------------------------- */
typedef struct vbcsr_zmat vbcsr_zmat; /* opaque, owned by the library */
enum { VBCSR_PHASE_R = 0, VBCSR_PHASE_R_TAU = 1 };

/*
 * vbcsr_zmat_create -- a periodic operator from its image blocks.
 *   block_sizes, row_ptr, col_idx  as vbcsr_create, except that the same
 *                (i, j) may appear once per image
 *   image        host [nnzb], 0 <= image[t] < n_images: block t couples atom
 *                i of the home cell to atom j of the cell shifted by
 *                shifts[3*image[t] .. +3]
 *   shifts       host [3*n_images] integer lattice translations
 *   tau          host [3*n_atoms] fractional positions, or NULL (then only
 *                VBCSR_PHASE_R can be sampled)
 *   values       host, graph order, each real block row-major; NULL = zeros
 *   prec         VBCSR_FP64 (complex double pages) or VBCSR_FP32 (complex
 *                float pages); the image values are kept in FP64
 *   opts         row_order is used (the pattern of O(k) is planned like
 *                vbcsr_create's); may be NULL
 * The pages of O(k) are zero until vbcsr_zmat_sample.  Synchronises stream.
 * Errors: EINVAL, ESHAPE, EDUP (same (i, j) twice in one image),
 * EUNSUPPORTED (BF16X3, vbcsr_create's size limits on the pattern of O(k),
 * or a block row or column of O(k) with 2^27 or more values), ENOMEM, EHIP.
 */
int vbcsr_zmat_create(vbcsr_zmat **out, int32_t n_atoms, const int32_t *block_sizes,
                      const int64_t *row_ptr, const int32_t *col_idx, const int32_t *image,
                      int32_t n_images, const int32_t *shifts, const double *tau,
                      const double *values, int64_t n_values, vbcsr_prec prec,
                      const vbcsr_plan_opts *opts, void *stream);

/*
 * vbcsr_zmat_sample -- assemble O(k) (and its conjugate transpose for the
 * adjoint) on the device: one FP64 phase per image block, FP64 sums over the
 * images of each block, stored in the handle's precision.
 *   k           host [3], finite
 *   convention  VBCSR_PHASE_R or VBCSR_PHASE_R_TAU (needs tau)
 * Asynchronous on `stream`; products on other streams must not overlap it.
 * Errors: EINVAL, EHIP.
 */
int vbcsr_zmat_sample(vbcsr_zmat *Z, const double *k, int32_t convention, void *stream);

/*
 * vbcsr_zmat_spmm -- Y <- alpha * op(O(k)) X + beta * Y, op = identity
 * (adjoint = 0, section 3.2) or the conjugate transpose (adjoint = 1,
 * equation 1: Y_j += O_ij^dagger X_i).  alpha, beta: host [2] (re, im);
 * beta = 0 means Y is not read.  X, Y: device, N x nrhs complex, row-major.
 * No atomics: every output row has one writer.  FP64 with nrhs >= 16 (and X
 * spanning less than 2^31 bytes) runs on matrix cores, otherwise on vector
 * FMA.
 * Errors: EINVAL (null pointers, nrhs <= 0, ld < nrhs, overlap), EHIP.
 */
int vbcsr_zmat_spmm(const vbcsr_zmat *Z, const void *X, int64_t ldx, void *Y, int64_t ldy,
                    int32_t nrhs, const double *alpha, const double *beta, int32_t adjoint,
                    void *stream);

/* vbcsr_zmat_info -- N, blocks and values of O(k); any pointer may be NULL. */
int vbcsr_zmat_info(const vbcsr_zmat *Z, int64_t *n_rows, int64_t *nnzb_k, int64_t *n_values_k);

/* vbcsr_zmat_get_structure -- the pattern of O(k) (distinct (i, j), ascending
 * j per row): row_ptr host [n_atoms+1], col_idx host [nnzb_k]. */
int vbcsr_zmat_get_structure(const vbcsr_zmat *Z, int64_t *row_ptr, int32_t *col_idx);

/* vbcsr_zmat_get_values -- the blocks of the last sampled O(k), graph order
 * of that pattern, each block row-major, complex interleaved, written by a
 * kernel on `stream` to `values` (device, n_values_k complex elements). */
int vbcsr_zmat_get_values(const vbcsr_zmat *Z, void *values, void *stream);

/* vbcsr_zmat_destroy -- free a handle (NULL is ignored); synchronises the device. */
void vbcsr_zmat_destroy(vbcsr_zmat *Z);

/* vbcsr_destroy -- free a handle (NULL is ignored); synchronises the device.
 * Library utility: no passage of the paper defines it. */
void vbcsr_destroy(vbcsr_mat *A);

/* vbcsr_last_error -- (library utility; no passage of the paper defines it)
 * message of the last non-OK status on this thread
 * ("" if none).  The pointer stays valid until the next call on the thread. */
const char *vbcsr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VBCSR_H */

/*
 * mbamg.h -- C-ABI of libmbamg: monolithic blocked algebraic multigrid for
 * coupled two-field block systems on one MI355X (gfx950).
 *
 * The problem statement follows Sec. 4.1-4.2 of Ohm et al., "A monolithic
 * algebraic multigrid framework for multiphysics applications with examples
 * from resistive MHD": a block system A x = b with blocks A_fg
 * (eq. block-prec-form), grouped as a 2x2 system (eq. 2x2system), whose
 * multigrid hierarchy is built from the matrix alone.  One V-cycle (Sec. 3,
 * MGV figure) with the damped block Gauss-Seidel smoother of Algorithm 1
 * (Sec. 4.3.2) and block-diagonal piecewise-constant transfers
 * (Sec. 4.3.1, eq. blocktransfers) serves as a right preconditioner inside
 * restarted GMRES; coarse operators are Galerkin products P^T A P (Sec. 3).
 *
 * Layouts
 *   Matrix blocks: BSR, int32 row pointers and column indices (columns sorted
 *   within each row), FP64 values, each block br x bc row-major.  Block (f,g)
 *   has br = dofs[f], bc = dofs[g].  A_00 must be structurally symmetric.
 *   Vectors: FP64, blocked [x_0; x_1; ...]; segment f holds N_f*dofs[f]
 *   entries (N_f: block f's node count), node-major
 *   (x_f[node*dofs[f] + component]).
 *
 * Ownership
 *   mbamg_setup deep-copies the blocks (host or device memory), so the caller
 *   may free them on return.  The hierarchy owns all of its device memory
 *   until mbamg_destroy.  Vector arguments are caller-owned device buffers.
 *   Device memory the library releases (at mbamg_destroy, and the
 *   temporaries of mbamg_setup) stays cached in the process for reuse by
 *   later setups on the same device; mbamg_setup and mbamg_destroy
 *   synchronise the device before cached memory is reused.
 *
 * Streams
 *   hip_stream may be NULL (the default stream).  mbamg_vcycle is
 *   asynchronous on the stream; mbamg_setup and mbamg_solve synchronise it.
 *   A hierarchy must not be used from two streams or threads at once.
 *
 * Errors
 *   Every entry point returns an mbamg_status; negative values are errors and
 *   mbamg_last_error() returns a message for the calling thread.  No C++
 *   exception crosses this interface.
 */
#ifndef MBAMG_H
#define MBAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MBAMG_OK = 0,
    MBAMG_NOT_CONVERGED = 1,   /* solve stopped at max_iters; x holds the last iterate */
    MBAMG_E_INVALID = -1,      /* inconsistent sizes, NULL pointers, aliasing, bad params */
    MBAMG_E_NOMEM = -2,        /* device or host allocation failed */
    MBAMG_E_HIP = -3,          /* a HIP runtime call failed */
    MBAMG_E_SINGULAR = -4,     /* a nodal diagonal block or the coarsest matrix is singular */
    MBAMG_E_STATE = -5         /* the hierarchy cannot do this (e.g. wrong precision form) */
} mbamg_status;

/* One matrix block A_fg of eq. block-prec-form in BSR form.  nnzb == 0
 * (pointers may then be NULL) is a zero block.  on_device != 0 means the three
 * arrays are device pointers.  mbamg_setup checks every block's structure --
 * row_ptr[0] == 0, row_ptr[n_brows] == nnzb, non-decreasing row pointers,
 * columns in range and strictly increasing within a row -- on the host for
 * host input and with a check kernel on its own copy for device input, before
 * any other kernel reads the block; a malformed block gives MBAMG_E_INVALID. */
typedef struct {
    int32_t n_brows, n_bcols, br, bc;
    int64_t nnzb;
    const int32_t* row_ptr;   /* n_brows + 1 */
    const int32_t* col_idx;   /* nnzb */
    const double* vals;       /* nnzb * br * bc */
    int32_t on_device;
} mbamg_bsr;

/* Field grouping (eq. block-prec-form; eq. 2x2system for two blocks): block f
 * has dofs[f] unknowns per node, the first n_vec[f] of them vector
 * components.  n_blocks = 2 with dofs[0] == dofs[1] is the full method (FP64
 * and FP32 forms, learned weights, both smoothers); block f's node count is
 * A_ff's n_brows, equal for both blocks unless clone_aggregates == 0.
 * n_blocks = 3 or 4 (e.g. the 4 x 4 split into u, p, b, r of Sec. 2.1, dofs
 * 1..4 per block) takes co-located fields: the aggregates of A_00 cloned to
 * every block and Algorithm 1 (Sec. 4.3.2) over the blocks in order; FP64,
 * fixed weights and the blocked smoother only (precision = 0, learned = 0,
 * omega_p = 0, smoother = 0, clone_aggregates = 1; MBAMG_E_INVALID
 * otherwise).  A block may be a zero block (nnzb = 0) except the diagonal
 * ones. */
typedef struct {
    int32_t n_blocks;
    int32_t dofs[4];
    int32_t n_vec[4];
} mbamg_field_map;

/* Per-aggregate weights for one level (learned == 2): given the level's
 * n_agg x 12 features (host, row-major, as returned by mbamg_features), write
 * omega_p[n_agg] (prolongator smoothing, >= 0) and omega_s[n_agg] (smoother
 * damping, > 0).  Called from mbamg_setup on the calling thread. */
typedef void (*mbamg_weight_fn)(int32_t level, int32_t n_agg, const float* features, double* omega_p,
                                double* omega_s, void* ctx);

typedef struct {
    double omega;             /* Algorithm 1 damping (default 0.8) */
    int32_t bgs_sweeps;       /* Algorithm 1 sweeps for pre- and post-smoothing (1) */
    int32_t inner_sweeps;     /* multicolour nodal-block GS sweeps per sub-block solve (1) */
    double theta;             /* strength threshold on squared block norms (0) */
    int32_t max_levels;       /* (10) */
    int32_t max_coarse;       /* stop coarsening at or below this many dofs (2500) */
    int32_t clone_aggregates; /* 1: block 1 reuses block 0's aggregates (the aggregate-cloning figure of
                                 Sec. 4.3.1; needs co-located fields, equal node counts).  0: each block is
                                 aggregated from the strong graph of its own diagonal block, the separate
                                 per-block AMG setup of Sec. 4.3.1 for fields on different node sets
                                 (A_00 on N_0 nodes, A_11 on N_1, A_01 N_0 x N_1); P = diag(P_00, P_11) with
                                 P_00 != P_11, coarsening until both blocks' aggregates together keep more
                                 than 90 % of a level's nodes; fixed form with the blocked smoother only
                                 (learned = 0, omega_p = 0, smoother = 0).  (1) */
    int32_t reuse_P;          /* kept for the interface; P_11 = P_00 holds when clone is on */
    int32_t precision;        /* 0: FP64 V-cycle + GMRES; 1: FP32 V-cycle inside FP64 FGMRES */
    int32_t restart;          /* GMRES restart length (30, at most 31) */
    int32_t max_iters;        /* (1000) */
    int32_t learned;          /* 0: fixed weights; 1: network in `mlp`; 2: `weight_fn` */
    const float* mlp;         /* learned == 1: host array of 5122 network parameters, then 12 feature
                                 means and 12 feature standard deviations (5146 floats) */
    uint64_t seed;            /* aggregation priority seed (0) */
    double omega_p;           /* learned == 0: uniform prolongator-smoothing weight (0: piecewise constant) */
    int32_t judge;            /* learned != 0: also build the fixed-weight hierarchy, estimate both
                                 convergence factors with mbamg_probe and keep the better one; a kept
                                 learned hierarchy holds the fixed-weight one as its fallback, and a
                                 solve that stalls with it (a complete restart cycle reducing the
                                 residual by less than 0.99 per iteration on average, or a residual
                                 that is not finite) finishes with the fixed-weight one from its
                                 current iterate (mbamg_info.reverted) (1) */
    mbamg_weight_fn weight_fn;
    void* weight_ctx;
    int32_t smoother;         /* 0: damped block Gauss-Seidel over the two blocks (Sec. 4.3.2, Algorithm 1);
                                 1: damped nodal-block Gauss-Seidel over the full (d0+d1)-square node blocks,
                                 the fully coupled (FC-AMG) reference of Sec. 5.1, here with nodal-block
                                 Gauss-Seidel in place of its Schwarz relaxation.  1 needs
                                 every block's pattern inside A00's and equal patterns of A00 and A11 on
                                 every level (MBAMG_E_INVALID otherwise); it uses the sliced smoother
                                 layout on every level (0) */
} mbamg_params;

typedef struct {
    int32_t iterations, levels, used_learned;
    double rel_residual;      /* true residual ||b - A x|| / ||b|| at exit */
    double conv_factor;       /* (rel_residual)^(1/iterations) */
    double op_complexity;     /* sum over levels of structural block entries / level 0 */
    double t_setup_ms, t_solve_ms;
    int32_t reverted;         /* 1: the solve of a judged learned hierarchy stalled and finished with the
                                 fixed-weight hierarchy (used_learned is then 0) */
} mbamg_info;

typedef struct mbamg_hierarchy mbamg_hierarchy;

/* Fill *p with the defaults listed above. */
void mbamg_default_params(mbamg_params* p);

/* Build the hierarchy (Sec. 3 and Sec. 4.3.1): strength graph of A_00 (the
 * amalgamated node graph), distance-2 aggregation cloned to block 1 (the
 * aggregate-cloning figure), piecewise-constant P per block assembled as the
 * block-diagonal transfer of eq. blocktransfers, Galerkin products P^T A P for
 * all four blocks on every level, colouring and nodal D^-1 for the smoother of
 * Algorithm 1 (Sec. 4.3.2), and the inverse of the coarsest matrix.  A_blocks
 * points to n_blocks*n_blocks blocks in row-major order (A_00, A_01, A_10,
 * A_11 for two blocks), deep-copied.  The colouring of a diagonal block is taken over its
 * symmetrised pattern, so A_11 need not be structurally symmetric.  *out
 * receives the hierarchy (the caller releases it with mbamg_destroy), or NULL
 * on an error, when whatever the build had allocated has been released.
 * Synchronous. */
mbamg_status mbamg_setup(const mbamg_bsr* A_blocks, const mbamg_field_map* fm,
                         const mbamg_params* p, void* hip_stream, mbamg_hierarchy** out);

/* z = M^-1 r: one V-cycle (Sec. 3, MGV figure) from a zero guess on the
 * finest level, pre- and post-smoothed by Algorithm 1 (Sec. 4.3.2), coarsest
 * level solved directly.  r and z are caller-owned device vectors of
 * sum_f n_nodes*dofs[f] doubles in the blocked layout; they must not alias
 * (MBAMG_E_INVALID).  Asynchronous on the stream. */
mbamg_status mbamg_vcycle(mbamg_hierarchy* h, const double* r, double* z, void* hip_stream);

/* w = A x with the four blocks of eq. 2x2system on the finest level (device
 * vectors in the blocked layout, must not alias).  Asynchronous. */
mbamg_status mbamg_apply(mbamg_hierarchy* h, const double* x, double* w, void* hip_stream);

/* Solve A x = b (eq. 2x2system) by restarted GMRES (FGMRES when
 * precision == 1), right preconditioned by one V-cycle as in Sec. 5 (a
 * multigrid V-cycle used as the Krylov preconditioner), to
 * ||b - A x|| <= rtol ||b||.  b and x are caller-owned device vectors.  x is read as
 * the initial guess and overwritten.  Returns MBAMG_NOT_CONVERGED after
 * max_iters.  info may be NULL.  Synchronous.  On a one-level hierarchy (a
 * system no larger than max_coarse) the preconditioner is the dense inverse,
 * so the solve stops after one iteration (a few in the FP32 form). */
mbamg_status mbamg_solve(mbamg_hierarchy* h, const double* b, double* x, double rtol,
                         mbamg_info* info, void* hip_stream);

mbamg_status mbamg_get_info(const mbamg_hierarchy* h, mbamg_info* info);
void mbamg_destroy(mbamg_hierarchy* h);
const char* mbamg_last_error(void);

/* ---- hierarchy inspection (read-back for verification and tooling) ------ */

/* Number of levels and, for level l, its node count. */
mbamg_status mbamg_num_levels(const mbamg_hierarchy* h, int32_t* n_levels);
mbamg_status mbamg_level_nodes(const mbamg_hierarchy* h, int32_t level, int32_t* n_nodes);

/* Aggregate of every node of level l (l < n_levels-1), node order of the
 * level as built by the Galerkin products (not the smoother's colour order).
 * agg is a host buffer of n_nodes int32.  Block 0's aggregates. */
mbamg_status mbamg_copy_aggregates(const mbamg_hierarchy* h, int32_t level, int32_t* agg);

/* The same per block f: node count of block f on level l, and block f's
 * aggregates (block 0's when cloned). */
mbamg_status mbamg_level_block_nodes(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t* n_nodes);
mbamg_status mbamg_copy_block_aggregates(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t* agg);

/* Number of stored blocks of block (f,g) on level l. */
mbamg_status mbamg_level_nnzb(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t g,
                              int64_t* nnzb);

/* Copy block (f,g) of level l in BSR form to host buffers sized by
 * mbamg_level_nodes and mbamg_level_nnzb. */
mbamg_status mbamg_copy_level_block(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t g,
                                    int32_t* row_ptr, int32_t* col_idx, double* vals);

/* Smoother colour of every node of block f on level l (host int32 buffer). */
mbamg_status mbamg_copy_colours(const mbamg_hierarchy* h, int32_t level, int32_t f,
                                int32_t* colour);

/* ---- learned form -------------------------------------------------------
 * Per aggregate k of a level, omega_P,k smooths the prolongator on the vector
 * components, P = Phat - D_vv^-1 A_vv Phat diag(omega_P), and omega_S,k damps
 * the block Gauss-Seidel updates of the aggregate's nodes (both blocks).  The
 * paper uses piecewise-constant transfers and one fixed damping (Sec. 4.3.1,
 * 4.3.2); these weights are this library's addition. */

/* Raw features (n_agg x 12, host float) of level l < n_levels-1; available
 * when the hierarchy was built with learned != 0. */
mbamg_status mbamg_features(const mbamg_hierarchy* h, int32_t level, float* features);

/* Weights used on level l (host buffers of n_agg doubles; omega_s is the
 * uniform omega where no per-aggregate damping was set). */
mbamg_status mbamg_level_weights(const mbamg_hierarchy* h, int32_t level, double* omega_p, double* omega_s);

/* Network 12 -> 64 -> 64 -> 2 (ReLU), bfloat16 matrix-core products with FP32
 * accumulation.  params: 5122 FP32 on the device (W1[64][12], b1, W2[64][64],
 * b2, W3[2][64], b3); x: n x 12 normalised features; out: n x 2 =
 * (omega_P in (0, 5/6), omega_S in (0.3, 1.3)).  Device pointers, asynchronous. */
mbamg_status mbamg_mlp_forward(const float* params, const float* x, int64_t n, float* out, void* hip_stream);

/* Mean squared error sum_c (out_c - target_c)^2 averaged over n rows, and its
 * gradient with respect to the 5122 parameters.  grad[5122] and loss[1] are
 * device outputs.  Asynchronous. */
mbamg_status mbamg_mlp_loss_grad(const float* params, const float* x, const float* target, int64_t n,
                                 float* grad, float* loss, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, training loops that must not call hipMalloc): the same loss and
 * gradient as mbamg_mlp_loss_grad, bit for bit (same grid, same summation
 * order), with the per-wavefront partial sums kept in a static device buffer
 * of 20.0 MiB (256 workgroups x 4 wavefronts x 5123 floats) instead of
 * library-allocated memory.  It calls no allocator: each GPU holds its own
 * copy of the buffer, reserved when the library's code is loaded on it and
 * held until the process ends; its device address is looked up on the first
 * call on each device.  The need does not grow with n (at most 256 workgroups
 * for any batch), so every n > 0 fits; a grid that would need more than the
 * buffer holds is rejected with MBAMG_E_INVALID.  The buffer keeps the last
 * call's contents; every call overwrites all the entries it reads, so nothing
 * needs clearing.  Calls that overlap on one GPU (two streams, two threads)
 * share the buffer and race: serialise them.  Device pointers, asynchronous. */
mbamg_status mbamg_mlp_loss_grad_noalloc(const float* params, const float* x, const float* target, int64_t n,
                                         float* grad, float* loss, void* hip_stream);

/* One Adam step (Kingma & Ba 2015) on the 5122 parameters with moment buffers
 * m, v (device); step counts from 1.  Asynchronous. */
mbamg_status mbamg_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr,
                            float beta1, float beta2, float eps, void* hip_stream);

/* Asymptotic convergence factor of the stationary iteration e <- e - M A e
 * from a seeded random start: (||e_iters|| / ||e_{iters-4}||)^(1/4).
 * iters >= 5.  Synchronous. */
mbamg_status mbamg_probe(mbamg_hierarchy* h, int32_t iters, uint64_t seed, double* rho, void* hip_stream);

/* Change the uniform smoother damping omega (Algorithm 1's damping of each block
 * update) of levels without per-aggregate damping, and of a judged learned
 * hierarchy's fixed-weight fallback.  omega must be finite and > 0
 * (MBAMG_E_INVALID otherwise).  Host only; takes effect from the next V-cycle. */
mbamg_status mbamg_set_omega(mbamg_hierarchy* h, double omega);

/* ---- measurement -------------------------------------------------------- */

/* Kernel timing with HIP events on the stream the kernels run on.  enable:
 * 0 off; 1 every kind below; 2 only whole V-cycles (kind 4); 3 whole V-cycles
 * and levels (kinds 4 and 16 + ...).  While mode 1 is on, every launch of the finest level's smoother and residual kernels is
 * bracketed by events.  kind 0: smoother colour passes from a nonzero iterate
 * with the coupling term (the post-smoother), 1: residual, 2: operator apply,
 * 3: the other smoother colour passes.  Reports launches, summed event time in
 * ms and the algorithmic bytes those launches move (structural values, block
 * indices, row pointers and vectors, each counted once per launch).
 * kind 4: whole V-cycles as the solver and the probe apply them (colour order,
 * without the interface's reordering or the FP32 form's casts; bytes 0).
 * kind 5: restrictions from the finest level, 6: prolongations to it; on a
 * coarser level l, kind 64 + 8 l + k for the same launches (k = 0, 1, 3, 5, 6).
 * kind 16 + 2 l: level l's share of each V-cycle on the way down
 * (pre-smoothing, residual, restriction; the coarsest level's direct solve);
 * kind 17 + 2 l: on the way up (prolongation, post-smoothing); with the
 * bytes of mbamg_level_vcycle_bytes.  Events add a little time: time with
 * timing disabled, collect these in a separate run. */
mbamg_status mbamg_timing_enable(mbamg_hierarchy* h, int32_t enable);   /* resets the collected events */
mbamg_status mbamg_timing_get(mbamg_hierarchy* h, int32_t kind, int64_t* launches,
                              double* total_ms, double* bytes);

/* Algorithmic bytes of one V-cycle of the current hierarchy and form (two-block
 * hierarchies; MBAMG_E_STATE for more blocks). */
mbamg_status mbamg_vcycle_bytes(const mbamg_hierarchy* h, double* bytes);

/* The same for level l's share: *down on the way down (pre-smoothing,
 * residual, restriction; on the coarsest level its direct solve), *up on the
 * way up (prolongation, post-smoothing). */
mbamg_status mbamg_level_vcycle_bytes(const mbamg_hierarchy* h, int32_t level, double* down, double* up);

#ifdef __cplusplus
}
#endif

#endif /* MBAMG_H */

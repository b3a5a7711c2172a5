// Solve-phase views and launchers (device work in solve_kernels.hip).
#pragma once

#include "common.h"

namespace mbamg {

// Rows of one block on one level, in smoother colour order, cut into slices
// of at most 64 rows that never straddle two colours.
struct SliceView {
    const int32_t* row0;
    const int32_t* nrow;
};

// One matrix part in masked sliced-ELL form.  Slice s has width[s] slots; slot
// t of slice s is global slot coff[s]+t, with a column per lane in
// col[slot*64 + lane] (-1 marks padding) and a bit mask of the block entries
// stored for every lane of the slot.  The values of the slot's set bits follow
// each other as groups of 64 (one per lane) starting at group voff[slot].
template <class T>
struct SellView {
    const int32_t* width;
    const int64_t* coff;
    const int64_t* voff;       // per slot
    const uint32_t* mask;
    const int32_t* col;
    const T* val;
};

template <class T>
struct GsArgs {
    int s_begin, s_count;      // slices of this colour
    SliceView sl;
    SellView<T> off, cpl, dinv;
    const T* b;                // right-hand side of this block
    const T* x;                // current iterate of this block (unused when starting from zero)
    T* t;                      // undamped Gauss-Seidel iterate x + e
    T* xn;                     // damped result x + omega e
    const T* xg;               // iterate of the other block for the coupling term
    int cstart;                // rows below this index already carry this sweep's update
    T omega;
    const T* w_row;            // per-row damping (NULL: use omega)
    int skip_off;              // nothing processed yet and zero start: the A_ff term vanishes
};

// One colour of the nodal-block Gauss-Seidel over the full node blocks (both
// blocks' rows of a node relaxed together): the two blocks share one colour
// order and slicing; the node inverses are ((d0+d1) x (d0+d1)), masked per
// slice: the entries k set in dmask[s] stored as groups of 64 values (one per
// lane) from group doff[s].
template <class T>
struct GsFcArgs {
    int s_begin, s_count;
    SliceView sl;
    SellView<T> off[2], cpl[2];    // A_ff without its diagonal block; A_fg with it (skipped)
    const T* dinv;
    const uint64_t* dmask;
    const int32_t* doff;
    const T* b[2];
    const T* x[2];                 // current iterates (unused when starting from zero)
    T* t[2];                       // undamped iterates x + e
    T* xn[2];                      // damped results x + omega e
    int cstart;                    // rows below this index already carry this sweep's update
    T omega;
    const T* w_row;                // per-row damping (NULL: use omega)
    int skip_off;                  // nothing processed yet and zero start: the sums vanish
};

// A block row of a coarse level in row form: rows in colour order, each row's
// blocks contiguous (row-major br x bc) with columns in the column block's
// colour order.  Used where rows are long (dense coarse stencils): one
// wavefront per row, its lanes over the row's blocks.
template <class T>
struct RowView {
    const int32_t* rp;         // rows + 1
    const int32_t* col;
    const T* val;
};

template <class T>
struct GsRowArgs {
    int r_begin, r_count;      // rows of this colour
    RowView<T> aff, afg;       // A_ff with its diagonal block (skipped here), A_fg
    const T* dinv;             // d x d per row, colour order
    const T* b;
    const T* x;
    T* t;
    T* xn;
    const T* xg;
    int cstart;
    T omega;
    const T* w_row;
    int skip_off;
};

template <class T>
struct ResidRowArgs {
    int n[2];
    RowView<T> aff[2], afg[2];
    const T* b[2];             // NULL for a plain operator apply
    const T* x[2];
    T* r[2];
    const int32_t* order[2];   // slice of each launch position (NULL: the position itself)
};

template <class T>
struct ResidArgs {
    int s_count[2];
    SliceView sl[2];
    SellView<T> off[2], cpl[2], diag[2];
    const T* b[2];             // NULL for a plain operator apply
    const T* x[2];
    T* r[2];
    const int32_t* order[2];   // slice of each launch position (NULL: the position itself)
};

template <class T>
struct TransferArgs {
    int n_rows[2];             // fine rows (prolongation) or coarse rows (restriction) per block
    const int32_t* map[2];     // prolongation: coarse row of each fine row; restriction: member pointer
    const int32_t* idx[2];     // restriction: member rows
    const T* q[2];             // prolongation: per fine row; restriction: per member, in member-list order
    const T* in[2];
    T* out[2];
    // restriction: the coarse row each group of lanes takes, in launch order (NULL: row i for
    // group i); the next level's natural order keeps neighbouring aggregates, whose members
    // share the fine rows' cache lines, in neighbouring groups
    const int32_t* order[2];
};

// P: waves per slice (1, 2 or 4); the slice's slots are split among them.
template <class T>
struct XferArgs {
    int s_count[2];
    SliceView sl[2];
    SellView<T> A[2];
    const T* x[2];
    T* y[2];
    int accumulate;
    const int32_t* out_row[2];   // row of y each slice row writes (NULL: the slice row itself)
};

// P waves share each slice's slots (1, 2 or 4)
template <class T>
void launch_xfer(int d, int P, const XferArgs<T>& a, hipStream_t s);

// A transfer in row form: one wavefront per row of P or P^T (rows of block 0,
// then block 1), for few wide rows.
template <class T>
struct XferRowArgs {
    int n[2];
    RowView<T> A[2];
    const T* x[2];
    T* y[2];
    int accumulate;
    const int32_t* out_row[2];   // row of y each matrix row writes (NULL: the row itself)
};
template <class T>
void launch_xfer_rows(int d, const XferRowArgs<T>& a, hipStream_t s);
template <class T>
void launch_gs(int d, int P, bool zero_x, bool has_cpl, const GsArgs<T>& a, hipStream_t s);
template <class T>
void launch_resid(int d, int P, const ResidArgs<T>& a, hipStream_t s);
template <class T>
void launch_gs_fc(int d, int P, bool zero_x, const GsFcArgs<T>& a, hipStream_t s);
template <class T>
// rp: wavefronts per row (1, or 4 with 4 x 4 blocks for long rows)
void launch_gs_rows(int d, int rp, bool zero_x, bool has_cpl, const GsRowArgs<T>& a, hipStream_t s);
template <class T>
void launch_resid_rows(int d, const ResidRowArgs<T>& a, hipStream_t s);
// y += sign * A x for one block in row form, any block shape up to 4 x 4 (one thread per row)
template <class T>
void launch_rows_acc(int n, int br, int bc, const RowView<T>& A, const T* x, T* y, T sign, hipStream_t s);

template <class T>
// G: lanes per coarse row (4, 8, 16 or 64)
void launch_restrict(int d, const TransferArgs<T>& a, int G, hipStream_t s);
template <class T>
void launch_prolong(int d, const TransferArgs<T>& a, hipStream_t s);
template <class T>
void launch_coarse(int n, const double* inv, const T* x, T* y, hipStream_t s);

// Krylov helpers (FP64).  Reductions are two-pass and deterministic: per-block
// partial sums stored slot-major (partial[q * KBLOCKS + block]), then one
// workgroup sums every slot in a fixed order.
constexpr int KMAXQ = 33;        // basis vectors + 2 slots (a dot with the candidate, a norm)
constexpr int KBLOCKS = 1024;
// layout of the coefficient buffer of the delayed-reorthogonalisation update:
// [0, KMAXQ) a (reorthogonalisation coefficients of the candidate),
// [KMAXQ, 2 KMAXQ) b (projections of the new vector), then 1/nu and c_j
constexpr int KC_A = 0, KC_B = KMAXQ, KC_INV_NU = 2 * KMAXQ, KC_CJ = 2 * KMAXQ + 1, KC_TOTAL = 2 * KMAXQ + 2;
// partial[q] = sum V_q . w (q < nq), partial[nq] = sum w . w
void launch_orth(int64_t n, int nq, const double* V, int64_t ldv, const double* w, double* partial, int nblocks,
                 hipStream_t s);
// One pass of the delayed reorthogonalisation step (see the kernel)
void launch_dcgs_update(int64_t n, int nq, const double* V, int64_t ldv, const double* coef, double* u,
                        const double* w, double* out, double* partial, int nblocks, hipStream_t s);
// r_q = sum over blocks of partial[q] for q = 0..nq: d[q] = r_q (q < nq, d may be
// NULL), *nu = r_nq (may be NULL); with coef (the dot pass of the delayed
// reorthogonalisation, nq - 1 basis vectors and the candidate):
// coef[KC_B + q] = r_q (q < nq - 1), coef[KC_CJ] = (r_{nq-1} - sum_q coef[KC_A + q] r_q) coef[KC_INV_NU]
void launch_orth_reduce(const double* partial, int nblocks, int nq, double* d, double* nu, double* coef,
                        hipStream_t s);
void launch_combine(int64_t n, int k, const double* Z, int64_t ldz, const double* y, double* x, hipStream_t s);
void launch_combine32(int64_t n, int k, const float* Z, int64_t ldz, const double* y, double* x, hipStream_t s);
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
void launch_seeded(int64_t n, uint64_t seed, double* v, hipStream_t s);
int krylov_blocks(int64_t n);
void launch_gather(int n_rows, int d, const int32_t* perm, const double* src, double* dst, hipStream_t s);
void launch_scatter(int n_rows, int d, const int32_t* perm, const double* src, double* dst, hipStream_t s);
void launch_cast64to32(int64_t n, const double* a, float* b, hipStream_t s);
void launch_cast32to64(int64_t n, const float* a, double* b, hipStream_t s);

}  // namespace mbamg

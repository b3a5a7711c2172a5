// Setup-phase data and kernel entry points (device work in setup_kernels.hip).
#pragma once

#include <algorithm>
#include <climits>

#include "common.h"

namespace mbamg {

// A matrix block in natural node order with dense br x bc blocks (device).
struct SetupBsr {
    int n_rows = 0, n_cols = 0, br = 0, bc = 0;
    int64_t nnzb = 0;
    DevBuf<int32_t> rp, ci;
    DevBuf<double> val;
};

// Strong-connection graph of A00 (symmetric CSR, squared weights).
struct Strength {
    int n = 0, nnz = 0;
    DevBuf<int32_t> ptr, idx;
    DevBuf<double> w2;
};

// Aggregates of one level: agg[node], members per aggregate in increasing order.
struct Aggregates {
    int n = 0, n_agg = 0, mis_rounds = 0;
    DevBuf<int32_t> agg, mptr, midx;
};

int scan_exclusive(const int32_t* in, int64_t n, int32_t* out, hipStream_t s);
Strength build_strength(const SetupBsr& A, double theta, hipStream_t s);
Aggregates build_aggregates(const Strength& S, uint64_t seed, int level, hipStream_t s);
void fill_ones(double* a, int64_t n, hipStream_t s);
// a[0..n) = v with a kernel (no memset node, so the call may sit in a captured graph)
void fill_value(double* a, int64_t n, double v, hipStream_t s);
void build_tentative(const Aggregates& G, int d, const double* B, double* q, double* Bc, hipStream_t s);
// the tentative prolongator as a block matrix: row i holds diag(q_i) in column agg(i)
SetupBsr tentative_bsr(const Aggregates& G, int d, const double* q, hipStream_t s);
void build_dinv(const SetupBsr& A, double* dinv, hipStream_t s);
// Inverses of the full node blocks [[A00_ii, A01_ii], [A10_ii, A11_ii]] for the
// full-node smoother, the rows in the slices' order perm, masked per slice:
// bit k of mask[s] set when entry k is nonzero in some row of slice s, the set
// entries stored as groups of 64 (one per lane) from group off[s];
// MBAMG_E_SINGULAR when one is singular.
void build_node_inverses(const SetupBsr (&A)[2][2], int n_slices, const int32_t* row0, const int32_t* nrow,
                         const int32_t* perm, DevBuf<uint64_t>& mask, DevBuf<int32_t>& off, DevBuf<double>& inv64,
                         DevBuf<float>* inv32, hipStream_t s);
// true when every block of B lies in A's pattern (same rows)
bool within_pattern(const SetupBsr& A, const SetupBsr& B, hipStream_t s);
void sell_masks(int64_t n_slots, int bs, const int64_t* src, const double* val, uint32_t* mask, uint32_t* slot_nz,
                hipStream_t s);
void sell_fill(int64_t n_slots, int bs, const int64_t* src, const double* val, const uint32_t* mask,
               const int64_t* slot_voff, double* out, hipStream_t s);
void cast_to_f32(const double* a, float* b, int64_t n, hipStream_t s);
// smoothed prolongator (vector components), block transpose, generic ordered block product
SetupBsr sa_prolongator(const SetupBsr& A, int nv, const Aggregates& G, const double* q, const double* w,
                        hipStream_t s);
SetupBsr block_transpose(const SetupBsr& P, hipStream_t s);
// C = A B; `like`, when given, is a product whose operands had the same
// patterns as A and B: its pattern is reused and only the values are computed
SetupBsr spgemm(const SetupBsr& A, const SetupBsr& B, hipStream_t s, const SetupBsr* like = nullptr);
// C_k = A_k B_k for k < K <= 4 where the A_k share one pattern and the B_k
// share one pattern: the pattern is found once (or taken from `like`) and the
// values come from one launch; bit-identical to K separate products.
void spgemm_multi(const SetupBsr* const* A, const SetupBsr* const* B, int K, SetupBsr* const* C, hipStream_t s,
                  const SetupBsr* like = nullptr);
// A block row in row form (see RowView): rows in the colour order `perm`
// (colour position -> natural node), columns mapped through `col_iperm`
// (natural node -> colour position of the column block).
struct RowPart {
    int br = 0, bc = 0;
    int64_t nnzb = 0;
    DevBuf<int32_t> rp, col;
    DevBuf<double> v64;
    DevBuf<float> v32;
};
void build_rows(RowPart& R, int n, const int32_t* perm, const SetupBsr& A, const int32_t* col_iperm, bool want32,
                hipStream_t s);
// dst[p] = src[perm[p]] for blocks of bs values
void gather_blocks(int n, int bs, const int32_t* perm, const double* src, double* dst, hipStream_t s);
// For each colour c (rows colour_row[c] .. colour_row[c+1] in colour order,
// node perm[p]): 7 sums -- nonzero entries and blocks of A_ff's off-diagonal
// blocks, of A_fg, nonzero entries of D^-1 (natural order), nonzero entries
// and blocks of A_ff's diagonal block.
std::vector<int64_t> row_colour_stats(int n, const int32_t* perm, const SetupBsr& Aff, const SetupBsr& Afg,
                                      const double* dinv, const std::vector<int>& colour_row, hipStream_t s);

// true when X and Y have identical block patterns (synchronous)
bool same_pattern(const SetupBsr& X, const SetupBsr& Y, hipStream_t s);
// Structure check of device-resident BSR index arrays (row pointers n_rows + 1,
// columns nnzb); throws MBAMG_E_INVALID on a malformed block (synchronous)
void check_bsr_device(int n_rows, int n_cols, int64_t nnzb, const int32_t* rp, const int32_t* ci, hipStream_t s);

// Test-only choice between equivalent kernel forms: the value of environment
// variable `var`, or null when it is unset or empty.
const char* form_override(const char* var);
// device construction of the sliced smoother format (see hierarchy.hip)
void part_layout(int n, int ns, int kind, const int32_t* perm, const int32_t* rp, const int32_t* ci,
                 const int32_t* row0, const int32_t* nrow, DevBuf<int32_t>& width, DevBuf<int32_t>& coff32,
                 int64_t& n_slots, hipStream_t s);
void part_fill_index(int ns, int kind, const int32_t* row0, const int32_t* nrow, const int32_t* width,
                     const int32_t* coff32, const int32_t* perm, const int32_t* rp, const int32_t* ci,
                     const int32_t* col_iperm, int64_t n_slots, int32_t* col, int64_t* src, int32_t* slot_blocks,
                     hipStream_t s);
int64_t slot_offsets(int64_t n_slots, const uint32_t* mask, DevBuf<int64_t>& voff, hipStream_t s);
void i32_to_i64(int64_t n, const int32_t* a, int64_t* b, hipStream_t s);
void transfer_maps(int n, int nc, const int32_t* perm, const int32_t* iperm, const int32_t* agg,
                   const int32_t* cperm, const int32_t* ciperm, const int32_t* mptr, const int32_t* midx,
                   DevBuf<int32_t>& aggp, DevBuf<int32_t>& optr, DevBuf<int32_t>& oidx, hipStream_t s);
// Dense Gauss-Jordan inverse of the coarsest matrix ([block 0; block 1] order),
// queued on stream s; coarse_inverse_finish waits for it and checks pivots.
struct CoarseWork {
    int n = 0;
    DevBuf<double> M;                    // two n x n matrices (ping-pong)
    DevBuf<int32_t> sing, rowsrc, ord;   // singular flag; a panel's row sources; row order (two copies)
};
// the same for nb x nb blocks (A: nb * nb pointers, row-major; block f has A[f*nb+f]->n_rows nodes of d[f] dofs)
void coarse_inverse_launch_blocks(const SetupBsr* const* A, int nb, const int* d, DevBuf<double>& inv, CoarseWork& w,
                                  hipStream_t s);
void coarse_inverse_launch(const SetupBsr (&A)[2][2], const int d[2], DevBuf<double>& inv, CoarseWork& w,
                           hipStream_t s);
void coarse_inverse_finish(CoarseWork& w, hipStream_t s);

}  // namespace mbamg

// Host orchestration of libmbamg: hierarchy construction (Sec. 4.3: blocked
// aggregation cloned across blocks, block-diagonal piecewise-constant
// transfers, Galerkin coarse operators), the V-cycle schedule (Sec. 3, MGV)
// with the block Gauss-Seidel smoother (Sec. 4.3.2, Algorithm 1), restarted
// GMRES / flexible GMRES, and the C-ABI declared in include/mbamg.h.
#include <algorithm>
#include <chrono>
#include <future>
#include <map>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <optional>

#include "learned_kernels.h"
#include "setup_kernels.h"
#include "solve_kernels.h"

namespace mbamg {

// ----------------------------------------------------------------------------
// solve-format structures
// ----------------------------------------------------------------------------
struct SellPart {
    int br = 0, bc = 0;
    int64_t n_slots = 0, n_groups = 0;
    DevBuf<int32_t> width;
    DevBuf<int64_t> coff, voff;
    DevBuf<uint32_t> mask;
    DevBuf<int32_t> col;
    DevBuf<double> v64;
    DevBuf<float> v32;
    std::vector<int64_t> h_coff;        // per slice
    std::vector<int32_t> h_width;
    std::vector<uint32_t> h_slot_nz;    // structural nonzeros per slot
    std::vector<int32_t> h_slot_blocks; // stored blocks per slot

    template <class T>
    SellView<T> view() const;
    // structural values and stored blocks over slices [s0, s1)
    void stats(int s0, int s1, int64_t& nz, int64_t& blocks) const {
        nz = 0;
        blocks = 0;
        for (int s = s0; s < s1; ++s)
            for (int t = 0; t < h_width[s]; ++t) {
                nz += h_slot_nz[h_coff[s] + t];
                blocks += h_slot_blocks[h_coff[s] + t];
            }
    }
};

template <>
SellView<double> SellPart::view<double>() const { return {width.p, coff.p, voff.p, mask.p, col.p, v64.p}; }
template <>
SellView<float> SellPart::view<float>() const { return {width.p, coff.p, voff.p, mask.p, col.p, v32.p}; }

// Structural values and stored blocks of one colour's rows (byte model).
struct ColourStats {
    int64_t off_nz = 0, off_bl = 0, cpl_nz = 0, cpl_bl = 0, dinv_nz = 0;
};

struct BlockLevel {
    int d = 0, n = 0, n_colours = 0, n_slices = 0;
    int split = 1;                             // waves per slice in the smoother and residual kernels
    std::vector<ColourStats> cstats;
    int64_t all_nz = 0, all_bl = 0;            // off + cpl + diag over every row
    std::vector<int32_t> perm, iperm;          // colour order -> natural node, and back
    std::vector<int32_t> colour;               // natural order
    std::vector<int32_t> h_row0, h_nrow;
    std::vector<int> colour_slice, colour_row;  // per colour: first slice, first row (+ end)
    DevBuf<int32_t> row0, nrow, d_perm, d_iperm;
    SellPart off, cpl, diag, dinv;
    // per-row smoother damping in colour order (learned form), else empty
    DevBuf<double> w_row64;
    DevBuf<float> w_row32;
    // smoothed transfers: P rows of this level, P^T rows of the next level (sliced by the next level)
    SellPart pro, res;
    int pro_split = 1, res_split = 1;          // waves per slice in the transfer kernels
    // P^T's slices: the next level's rows in natural (aggregate) order, 64 per slice; the
    // restriction writes slice row r to the next level's colour-order row iperm[r]
    DevBuf<int32_t> res_row0, res_nrow;
    int res_slices = 0;
    // few wide P^T rows (small next levels): the restriction in row form, one wavefront per row
    bool res_rows = false;
    RowPart rres;
    int res_group = 4;                         // lanes per coarse row in the tentative restriction
    int row_split = 1;                         // row form smoother: wavefronts per row (1, or 4 with 4 x 4 blocks)
    // coarse levels with long rows: the smoother and residual run on the row form
    bool rows = false;
    // within-colour row order sorted by length in windows (coarse levels with mixed row lengths)
    bool sell_sorted = false;
    RowPart raff, rafg;
    DevBuf<double> rdinv64;
    DevBuf<float> rdinv32;
    // transfer to the next level (colour orders of both levels)
    DevBuf<int32_t> agg_p, mem_ptr, mem_idx;
    DevBuf<double> q64;
    DevBuf<float> q32;
    DevBuf<double> qm64;                       // q in member-list order (the restriction's reads)
    DevBuf<float> qm32;
    SliceView slices() const { return {row0.p, nrow.p}; }
};

template <class T>
struct Vecs {
    DevBuf<T> b, x, xs, t, r;
};

struct Level {
    int n = 0;                                 // nodes of block 0
    int n1 = 0;                                // nodes of block 1 (n when the fields are co-located)
    int d[2] = {0, 0};
    bool coarsest = false;
    bool apply_parts = false;                  // coarsest level with its sliced operator (single-level hierarchy)
    SetupBsr A[2][2];
    Aggregates G;                              // block 0's aggregates (both blocks' when cloned)
    Aggregates G1;                             // block 1's own aggregates (separate aggregation)
    bool separate = false;
    BlockLevel blk[2];
    int resid_split = 1;                       // waves per slice in the residual (one launch, both blocks)
    DevBuf<int32_t> resid_order[2];            // the residual's slice order per block (empty: identity)
    // smoothed prolongators (natural order) and the weights that built them
    bool smoothed = false, damped = false;
    SetupBsr P[2], PT[2];
    DevBuf<double> wp_agg, ws_agg;
    DevBuf<float> feat;
    // full-node smoother: inverses of the (d0+d1)-square node blocks, slice-major in block 0's order
    bool fc = false;
    DevBuf<uint64_t> fc_mask;                  // per slice: entries stored
    DevBuf<int32_t> fc_off;                    // per slice: first value group
    DevBuf<double> fc_inv64;
    DevBuf<float> fc_inv32;
    Vecs<double> v64;
    Vecs<float> v32;
    int64_t nnzb_total() const { return A[0][0].nnzb + A[0][1].nnzb + A[1][0].nnzb + A[1][1].nnzb; }
    int nodes(int f) const { return f == 0 ? n : n1; }
    int64_t ndof() const { return (int64_t)n * d[0] + (int64_t)n1 * d[1]; }
    const Aggregates& agg_of(int f) const { return (f == 1 && separate) ? G1 : G; }
};

// Systems of more than two blocks (eq. block-prec-form), co-located fields:
// the aggregates of A_00 are cloned to every block, and Algorithm 1 runs over
// the blocks in order with each block's couplings folded into its right-hand
// side.  Every block keeps its own colour order and sliced smoother parts
// (A_ff without its diagonal, nodal inverses); every block A_fg is also held
// in row form (rows in block f's colour order, columns in block g's) for the
// couplings, the residual and the operator.
constexpr int MAXB = 4;
struct GLevel {
    int n = 0, nb = 0;
    int d[MAXB] = {0, 0, 0, 0};
    int64_t off[MAXB + 1] = {0, 0, 0, 0, 0};   // first dof of each block
    bool coarsest = false;
    SetupBsr A[MAXB][MAXB];
    Aggregates G;
    BlockLevel blk[MAXB];
    RowPart R[MAXB][MAXB];
    DevBuf<double> b, x, xs, t, r, rhs;
    void set_blocks(int nodes, int nblocks, const int* dofs) {
        n = nodes;
        nb = nblocks;
        off[0] = 0;
        for (int f = 0; f < nb; ++f) {
            d[f] = dofs[f];
            off[f + 1] = off[f] + (int64_t)n * d[f];
        }
    }
    int64_t ndof() const { return off[nb]; }
    int64_t nnzb_total() const {
        int64_t t = 0;
        for (int f = 0; f < nb; ++f)
            for (int g = 0; g < nb; ++g) t += A[f][g].nnzb;
        return t;
    }
};

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
    double bytes;
};

// A second stream (default priority) with two events, released on scope exit.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    SideStream() {
        MB_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        MB_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        MB_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    }
    ~SideStream() {
        if (stream) { (void)hipStreamSynchronize(stream); (void)hipStreamDestroy(stream); }
        if (ready) (void)hipEventDestroy(ready);
        if (done) (void)hipEventDestroy(done);
    }
};

// The coarsest inverse of a build while it is still running on its own stream:
// members are released job first (its launches are all issued), then the
// stream (drained), then the buffers.
struct PendingCoarse {
    CoarseWork w;
    SideStream side;
    std::future<void> job;
};

// Hand-over from the fixed-weight build to a learned build running at the
// same time on another host thread and stream: the fixed build publishes its
// level-0 aggregates, then its level-0 smoother data (true), or that it has
// none (false); each publication comes with an event on the fixed build's
// stream after which the data is complete.
struct DonorLink {
    std::promise<bool> agg_p, smooth_p;
    std::shared_future<bool> agg, smooth;
    bool agg_set = false, smooth_set = false;
    hipEvent_t agg_ev = nullptr, smooth_ev = nullptr;
    const Level* level0 = nullptr;   // the fixed build's level 0 (stable: heap-allocated)
    DonorLink() : agg(agg_p.get_future().share()), smooth(smooth_p.get_future().share()) {
        MB_HIP(hipEventCreateWithFlags(&agg_ev, hipEventDisableTiming));
        MB_HIP(hipEventCreateWithFlags(&smooth_ev, hipEventDisableTiming));
    }
    ~DonorLink() {
        close();
        (void)hipEventDestroy(agg_ev);
        (void)hipEventDestroy(smooth_ev);
    }
    void publish_agg(bool ok) {
        if (agg_set) return;
        agg_set = true;
        agg_p.set_value(ok);
    }
    void publish_smooth(bool ok) {
        if (smooth_set) return;
        smooth_set = true;
        smooth_p.set_value(ok);
    }
    void close() {   // whatever was not published is not coming
        publish_agg(false);
        publish_smooth(false);
    }
};

thread_local std::string g_last_error;

// Krylov scalar buffer layout (device and pinned host copies): the dot pass's
// sums, the update pass's sums, two norms
constexpr int KB_D1 = 0, KB_D2 = KMAXQ, KB_NU0 = 2 * KMAXQ, KB_NU1 = 2 * KMAXQ + 1, KB_TOTAL = 2 * KMAXQ + 2;

}  // namespace mbamg

using namespace mbamg;

struct mbamg_hierarchy {
    mbamg_params p{};
    mbamg_field_map fm{};
    int d[2] = {0, 0};
    int nb = 2;                                // blocks; more than two use GL instead of L
    std::vector<std::unique_ptr<Level>> L;
    std::vector<std::unique_ptr<GLevel>> GL;
    DevBuf<double> coarse_inv;
    int coarse_n = 0;
    // Krylov workspace
    int64_t n_fine = 0;
    DevBuf<double> V, Z64, w, xw, bw, ztmp, partial, hbuf, ybuf, coef;
    DevBuf<float> mlp;             // network parameters (5122) followed by feature mean and std (12 + 12)
    double* hbuf_host = nullptr;   // pinned: Krylov scalars read back each iteration
    double* coef_host = nullptr;   // pinned: the update pass's coefficients going up
    double* y_host = nullptr;
    double judge_rho[2] = {0.0, 0.0};   // probe factors of the learned and the fixed hierarchy
    // a learned hierarchy the judge kept holds the fixed-weight one it was judged against: a
    // solve that stalls with the learned preconditioner finishes with it
    std::unique_ptr<mbamg_hierarchy> fallback;
    DevBuf<float> Z32, vin32;
    DevBuf<double> vio;   // ABI <-> colour-order staging for vcycle/apply
    DevBuf<double> vio2;
    mbamg_info info{};
    // timing
    int timing = 0;                // mbamg_timing_enable's mode
    bool time_launches() const { return timing == 1; }
    bool time_levels() const { return timing == 1 || timing == 3; }
    bool time_vcycles() const { return timing != 0; }
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    double t_setup_ms = 0.0;
    // last member, so it is released first: a coarsest inverse still in flight
    std::unique_ptr<PendingCoarse> coarse_pending;

    ~mbamg_hierarchy() {
        (void)hipDeviceSynchronize();
        for (auto& t : timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
        for (auto e : event_pool) (void)hipEventDestroy(e);
        if (hbuf_host) (void)hipHostFree(hbuf_host);
        if (coef_host) (void)hipHostFree(coef_host);
        if (y_host) (void)hipHostFree(y_host);
    }
};

namespace mbamg {

// ----------------------------------------------------------------------------
// timing helpers
// ----------------------------------------------------------------------------
static hipEvent_t get_event(mbamg_hierarchy* h) {
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    MB_HIP(hipEventCreate(&e));
    return e;
}

struct TimerScope {
    mbamg_hierarchy* h;
    hipStream_t s;
    bool on;
    TimedLaunch t{};
    TimerScope(mbamg_hierarchy* hh, hipStream_t ss, bool enabled, int kind, double bytes) : h(hh), s(ss), on(enabled) {
        if (!on) return;
        t.kind = kind;
        t.bytes = bytes;
        t.a = get_event(h);
        t.b = get_event(h);
        MB_HIP(hipEventRecord(t.a, s));
    }
    ~TimerScope() {
        if (!on) return;
        if (hipEventRecord(t.b, s) == hipSuccess) h->timed.push_back(t);
    }
};

// Setup phase timing, printed to stderr when MBAMG_VERBOSE is set (the stream
// is synchronised at each mark only in that case).
struct PhaseClock {
    bool on;
    hipStream_t s;
    std::chrono::steady_clock::time_point last;
    explicit PhaseClock(hipStream_t ss) : on(std::getenv("MBAMG_VERBOSE") != nullptr), s(ss) {
        last = std::chrono::steady_clock::now();
    }
    void mark(const char* what, int level) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[mbamg setup] level %d %-22s %8.2f ms\n", level, what,
                     std::chrono::duration<double, std::milli>(now - last).count());
        last = now;
    }
};

// ----------------------------------------------------------------------------
// setup helpers
// ----------------------------------------------------------------------------
static void copy_block(const mbamg_bsr& src, SetupBsr& dst, int n_rows, int n_cols, int br, int bc, hipStream_t s) {
    dst.n_rows = n_rows;
    dst.n_cols = n_cols;
    dst.br = br;
    dst.bc = bc;
    dst.nnzb = src.nnzb;
    MB_CHECK(src.nnzb >= 0 && src.nnzb < INT32_MAX, MBAMG_E_INVALID, "nnzb out of range");
    dst.rp.alloc(n_rows + 1);
    if (src.nnzb == 0 || src.row_ptr == nullptr) {
        MB_HIP(hipMemsetAsync(dst.rp.p, 0, sizeof(int32_t) * (n_rows + 1), s));
        dst.nnzb = 0;
        dst.ci.alloc(1);
        dst.val.alloc(1);
        return;
    }
    MB_CHECK(src.n_brows == n_rows && src.n_bcols == n_cols && src.br == br && src.bc == bc, MBAMG_E_INVALID,
             "block dimensions inconsistent with the field map");
    MB_CHECK(src.col_idx && src.vals, MBAMG_E_INVALID, "NULL block arrays");
    const int64_t bs = (int64_t)br * bc;
    dst.ci.alloc(src.nnzb);
    dst.val.alloc(src.nnzb * bs);
    hipMemcpyKind k = src.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (!src.on_device) {
        // host input: validate the structure here
        MB_CHECK(src.row_ptr[0] == 0 && src.row_ptr[n_rows] == src.nnzb, MBAMG_E_INVALID, "row_ptr inconsistent with nnzb");
        for (int i = 0; i < n_rows; ++i) {
            MB_CHECK(src.row_ptr[i + 1] >= src.row_ptr[i], MBAMG_E_INVALID, "row_ptr not monotone");
            for (int p = src.row_ptr[i]; p < src.row_ptr[i + 1]; ++p) {
                MB_CHECK(src.col_idx[p] >= 0 && src.col_idx[p] < n_cols, MBAMG_E_INVALID, "column index out of range");
                MB_CHECK(p == src.row_ptr[i] || src.col_idx[p] > src.col_idx[p - 1], MBAMG_E_INVALID,
                         "column indices must be strictly increasing within a row");
            }
        }
    }
    MB_HIP(hipMemcpyAsync(dst.rp.p, src.row_ptr, sizeof(int32_t) * (n_rows + 1), k, s));
    MB_HIP(hipMemcpyAsync(dst.ci.p, src.col_idx, sizeof(int32_t) * src.nnzb, k, s));
    MB_HIP(hipMemcpyAsync(dst.val.p, src.vals, sizeof(double) * src.nnzb * bs, k, s));
    // device input: the same structure checks on the library's copy, before any other kernel reads it
    if (src.on_device) check_bsr_device(n_rows, n_cols, src.nnzb, dst.rp.p, dst.ci.p, s);
}

// The transposed pattern (column -> rows), or nothing when the pattern is
// structurally symmetric already.
static bool transpose_pattern(int n, const int32_t* rp, const int32_t* ci, std::vector<int32_t>& trp,
                              std::vector<int32_t>& tci) {
    trp.assign(n + 1, 0);
    for (int p = 0; p < rp[n]; ++p) trp[ci[p] + 1]++;
    for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
    tci.assign(rp[n], 0);
    std::vector<int32_t> cur(trp.begin(), trp.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p) tci[cur[ci[p]]++] = i;   // rows ascending per column
    for (int i = 0; i <= n; ++i)
        if (trp[i] != rp[i]) return true;
    for (int p = 0; p < rp[n]; ++p)
        if (tci[p] != ci[p]) return true;
    return false;
}

// First-fit greedy colouring in increasing node order over the symmetrised
// pattern: a node avoids the colours of every node in its row and (when the
// pattern is not symmetric) in its column, so no two nodes coupled in either
// direction share a colour and every colour pass is a Gauss-Seidel step.
static int greedy_colour(int n, const int32_t* rp, const int32_t* ci, std::vector<int32_t>& colour,
                         const int32_t* trp = nullptr, const int32_t* tci = nullptr) {
    colour.assign(n, -1);
    std::vector<int32_t> mark(64, -1);
    int ncol = 0;
    auto visit = [&](int i, int j) {
        if (j == i || colour[j] < 0) return;
        if (colour[j] >= (int)mark.size()) mark.resize(colour[j] + 64, -1);
        mark[colour[j]] = i;
    };
    for (int i = 0; i < n; ++i) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) visit(i, ci[p]);
        if (trp)
            for (int p = trp[i]; p < trp[i + 1]; ++p) visit(i, tci[p]);
        int c = 0;
        while (c < (int)mark.size() && mark[c] == i) ++c;
        if (c >= (int)mark.size()) mark.resize(c + 64, -1);
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// Rows of one colour are independent in a Gauss-Seidel colour pass, so their
// order within the colour changes no result (each row's own sum runs over its
// columns in the same order).  A slice of 64 rows is as wide as its longest
// row; where rows of different lengths mix (coarse levels) the colour's rows
// are sorted by decreasing length within windows of SELL_SIGMA rows, which
// keeps the padding small while rows stay near their neighbours.
constexpr int SELL_SIGMA = 1024;

// Fraction of a sliced layout's slots that hold a stored block, for rows in
// the given order cut into slices of 64 (per colour).
static double slice_fill(const std::vector<int32_t>& order, const std::vector<int>& colour_row, const int32_t* rp) {
    int64_t blocks = 0, slots = 0;
    for (size_t c = 0; c + 1 < colour_row.size(); ++c)
        for (int r = colour_row[c]; r < colour_row[c + 1]; r += WAVE) {
            int w = 0;
            for (int q = r; q < std::min(r + WAVE, colour_row[c + 1]); ++q) {
                const int len = rp[order[q] + 1] - rp[order[q]];
                blocks += len;
                w = std::max(w, len);
            }
            slots += (int64_t)w * WAVE;
        }
    return slots ? (double)blocks / (double)slots : 1.0;
}

// rp: row pointers of the block row's diagonal block (row lengths), or NULL
// for the natural order within each colour.
static void order_and_slice(BlockLevel& B, int n, int ncol, const int32_t* rp = nullptr) {
    B.n = n;
    B.n_colours = ncol;
    std::vector<int> cnt(ncol + 1, 0);
    for (int i = 0; i < n; ++i) cnt[B.colour[i] + 1]++;
    B.colour_row.assign(ncol + 1, 0);
    for (int c = 0; c < ncol; ++c) B.colour_row[c + 1] = B.colour_row[c] + cnt[c + 1];
    B.perm.assign(n, 0);
    B.iperm.assign(n, 0);
    std::vector<int> cur(B.colour_row.begin(), B.colour_row.end() - 1);
    for (int i = 0; i < n; ++i) B.perm[cur[B.colour[i]]++] = i;
    B.sell_sorted = false;
    if (rp && slice_fill(B.perm, B.colour_row, rp) < 0.9) {
        B.sell_sorted = true;
        auto len = [rp](int32_t i) { return rp[i + 1] - rp[i]; };
        for (int c = 0; c < ncol; ++c)
            for (int w0 = B.colour_row[c]; w0 < B.colour_row[c + 1]; w0 += SELL_SIGMA) {
                const int w1 = std::min(w0 + SELL_SIGMA, B.colour_row[c + 1]);
                std::stable_sort(B.perm.begin() + w0, B.perm.begin() + w1,
                                 [&len](int32_t a, int32_t b) { return len(a) > len(b); });
            }
    }
    for (int p = 0; p < n; ++p) B.iperm[B.perm[p]] = p;
    B.h_row0.clear();
    B.h_nrow.clear();
    B.colour_slice.assign(ncol + 1, 0);
    for (int c = 0; c < ncol; ++c) {
        B.colour_slice[c] = (int)B.h_row0.size();
        for (int r = B.colour_row[c]; r < B.colour_row[c + 1]; r += WAVE) {
            B.h_row0.push_back(r);
            B.h_nrow.push_back(std::min(WAVE, B.colour_row[c + 1] - r));
        }
    }
    B.colour_slice[ncol] = (int)B.h_row0.size();
    B.n_slices = (int)B.h_row0.size();
}

enum class PartKind { Off = 0, Cpl = 1, Diag = 2, Dinv = 3 };

// coarse levels with at most this many rows per colour (on average) take the row form
// (measured crossover of the two layouts' colour passes on 4 x 4 FP64 blocks: 2.8K rows
// 6.9 us in the row form against 12.5 us sliced, 11K rows 15.6 against 13.6 us)
constexpr int ROWS_PER_COLOUR_MAX = 8192;

// Waves per slice (1..16) for a launch over `slices` slices of `width` slots
// on average: wide slices are shared by more waves until the launch has
// about 2048 waves, keeping at least 4 slots per wave.
static int slot_split(double slices, double width, double target = 2048) {
    int P = 1;
    while (P < 16 && slices * P < target && width >= 8.0 * P) P *= 2;
    return P;
}

// a transfer is one launch over the whole level (both block rows), not one colour
// lanes per coarse row in the tentative restriction: about two members per lane
// (MBAMG_RESTRICT_GROUP = 4 | 8 | 16 | 64 forces one, for tests: the group
// size changes the summation order)
static int restrict_group(int n_fine, int n_coarse) {
    if (const char* f = form_override("MBAMG_RESTRICT_GROUP")) {
        const int g = std::atoi(f);
        MB_CHECK(g == 4 || g == 8 || g == 16 || g == 64, MBAMG_E_INVALID, "MBAMG_RESTRICT_GROUP must be 4, 8, 16 or 64");
        return g;
    }
    const int64_t m = n_coarse > 0 ? ceil_div(n_fine, n_coarse) : 1;
    return m <= 8 ? 4 : m <= 16 ? 8 : m <= 32 ? 16 : 64;
}

static int transfer_split(const SellPart& P, int n_slices) {
    int64_t slots = 0;
    for (int w : P.h_width) slots += w;
    const double avg = n_slices ? (double)slots / n_slices : 0.0;
    return slot_split(n_slices, avg, 32768);
}

// A permutation of a level's slices (colour-major, colour_slice[c] .. [c+1])
// that lists, for x = 0..7, the x-th eighth of every colour's slices.
static std::vector<int32_t> slab_order(const std::vector<int>& colour_slice) {
    const int nc = (int)colour_slice.size() - 1;
    std::vector<int32_t> o;
    o.reserve(nc >= 0 ? (size_t)colour_slice.back() : 0);
    for (int x = 0; x < 8; ++x)
        for (int c = 0; c < nc; ++c) {
            const int64_t b = colour_slice[c], len = colour_slice[c + 1] - b;
            for (int64_t k = len * x / 8; k < len * (x + 1) / 8; ++k) o.push_back((int32_t)(b + k));
        }
    return o;
}

// next levels of at most this many rows take the restriction in row form
constexpr int RES_ROWS_MAX = 16384;

// Slices of 64 consecutive rows of an n-row matrix in natural order (identity
// row order), for parts whose rows need not follow a colour order.
static void natural_slicing(BlockLevel& B, int n, hipStream_t s) {
    B.n = n;
    B.n_slices = (int)ceil_div(n, WAVE);
    B.h_row0.resize(B.n_slices);
    B.h_nrow.resize(B.n_slices);
    for (int sl = 0; sl < B.n_slices; ++sl) {
        B.h_row0[sl] = sl * WAVE;
        B.h_nrow[sl] = std::min(WAVE, n - sl * WAVE);
    }
    B.perm.resize(n);
    for (int i = 0; i < n; ++i) B.perm[i] = i;
    B.row0.upload(B.h_row0, s);
    B.nrow.upload(B.h_nrow, s);
    B.d_perm.upload(B.perm, s);
}

// Pack one part of block row f into masked slices on the device.  A: the
// natural-order source block (unused for Dinv); val: its values, or the dense
// per-node inverse array for Dinv; col_iperm: natural column node -> colour
// order of the column block.
static void build_part(SellPart& P, PartKind kind, const BlockLevel& B, const SetupBsr* A, const int32_t* col_iperm,
                       const double* val, int br, int bc, bool want32, hipStream_t s) {
    P.br = br;
    P.bc = bc;
    const int ns = B.n_slices;
    const int k = (int)kind;
    const int32_t* rp = A ? A->rp.p : nullptr;
    const int32_t* ci = A ? A->ci.p : nullptr;
    DevBuf<int32_t> coff32;
    part_layout(B.n, ns, k, B.d_perm.p, rp, ci, B.row0.p, B.nrow.p, P.width, coff32, P.n_slots, s);
    const int64_t nsl = std::max<int64_t>(P.n_slots, 1);
    P.col.alloc(nsl * WAVE);
    DevBuf<int64_t> src(nsl * WAVE);
    DevBuf<int32_t> sblk(nsl);
    part_fill_index(ns, k, B.row0.p, B.nrow.p, P.width.p, coff32.p, B.d_perm.p, rp, ci, col_iperm, P.n_slots, P.col.p,
                    src.p, sblk.p, s);
    P.coff.alloc(std::max(ns, 1));
    i32_to_i64(ns, coff32.p, P.coff.p, s);
    P.mask.alloc(nsl);
    DevBuf<uint32_t> slot_nz(nsl);
    MB_HIP(hipMemsetAsync(slot_nz.p, 0, sizeof(uint32_t) * nsl, s));
    sell_masks(P.n_slots, br * bc, src.p, val, P.mask.p, slot_nz.p, s);
    P.n_groups = slot_offsets(P.n_slots, P.mask.p, P.voff, s);
    P.v64.alloc(std::max<int64_t>(P.n_groups, 1) * WAVE);
    sell_fill(P.n_slots, br * bc, src.p, val, P.mask.p, P.voff.p, P.v64.p, s);
    if (want32) {
        P.v32.alloc(std::max<int64_t>(P.n_groups, 1) * WAVE);
        cast_to_f32(P.v64.p, P.v32.p, P.n_groups * WAVE, s);
    }
    // host copies for the byte model, with one synchronisation (which also keeps the
    // temporaries alive until the kernels have finished)
    std::vector<int32_t> c32;
    HostCopies hc;
    hc.add(P.width, P.h_width, (size_t)ns);
    hc.add(coff32, c32, (size_t)ns + 1);
    hc.add(slot_nz, P.h_slot_nz, (size_t)nsl);
    hc.add(sblk, P.h_slot_blocks, (size_t)nsl);
    hc.run(s);
    P.h_coff.assign(c32.begin(), c32.end());
}

template <class T>
static void alloc_vecs(Vecs<T>& v, int64_t n) {
    int64_t m = std::max<int64_t>(n, 1);
    v.b.alloc(m);
    v.x.alloc(m);
    v.xs.alloc(m);
    v.t.alloc(m);
    v.r.alloc(m);
}

// ----------------------------------------------------------------------------
// setup
// ----------------------------------------------------------------------------
// Per-aggregate weights of one level: omega_P for the smoothed prolongator and,
// in the learned forms, omega_S for the smoother damping of the aggregate's
// nodes.  learned 1: features -> network on the device; learned 2: features ->
// the caller's callback; otherwise the uniform omega_p.
static void choose_weights(mbamg_hierarchy* h, Level& cur, const Aggregates& G, int lvl, hipStream_t s) {
    const mbamg_params& p = h->p;
    const int nc = G.n_agg;
    cur.wp_agg.alloc(std::max(nc, 1));
    cur.ws_agg.alloc(std::max(nc, 1));
    if (p.learned == 0) {
        std::vector<double> wp(nc, p.omega_p);
        cur.wp_agg.upload(wp, s);
        return;
    }
    BsrView A[2][2];
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g) A[f][g] = {cur.A[f][g].rp.p, cur.A[f][g].ci.p, cur.A[f][g].val.p, cur.A[f][g].br,
                                                       cur.A[f][g].nnzb};
    cur.feat.alloc((size_t)std::max(nc, 1) * N_FEATURES);
    aggregate_features(nc, cur.n, G.agg.p, G.mptr.p, G.midx.p, A, h->fm.n_vec[0], h->fm.n_vec[1], lvl, nullptr,
                       nullptr, cur.feat.p, s);
    if (p.learned == 1) {
        DevBuf<float> xn((size_t)std::max(nc, 1) * N_FEATURES), out2((size_t)std::max(nc, 1) * 2);
        normalize_features(nc, cur.feat.p, h->mlp.p + N_MLP_PARAMS, h->mlp.p + N_MLP_PARAMS + N_FEATURES, xn.p, s);
        mlp_forward(h->mlp.p, xn.p, nc, out2.p, s);
        split_weights(nc, out2.p, cur.wp_agg.p, cur.ws_agg.p, s);
        MB_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<float> F = cur.feat.download(s, (size_t)nc * N_FEATURES);
        std::vector<double> wp(nc, 0.0), ws(nc, p.omega);
        p.weight_fn(lvl, nc, F.data(), wp.data(), ws.data(), p.weight_ctx);
        for (int k = 0; k < nc; ++k)
            MB_CHECK(std::isfinite(wp[k]) && std::isfinite(ws[k]) && ws[k] > 0.0, MBAMG_E_INVALID,
                     "weight callback returned an invalid weight");
        cur.wp_agg.upload(wp, s);
        cur.ws_agg.upload(ws, s);
    }
    cur.damped = true;
}


// First-fit colouring, colour order and slices of both block rows of one level
// (host work on the diagonal blocks' patterns).  `ready` marks the point on
// the setup stream after which the level's blocks are complete; the patterns
// are copied on a stream of the calling thread.
static void colour_level(Level& Lv, hipEvent_t ready, int device) {
    MB_HIP(hipSetDevice(device));   // the calling thread may be a fresh one
    const bool verbose = std::getenv("MBAMG_VERBOSE") != nullptr;
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    hipStream_t cs = nullptr;
    MB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    std::unique_ptr<PinnedBuf<int32_t>> buf[2];
    const int32_t* rp[2] = {nullptr, nullptr};
    const int32_t* ci[2] = {nullptr, nullptr};
    bool same = false;
    auto t1 = t0, t2 = t0;
    try {
        MB_HIP(hipStreamWaitEvent(cs, ready, 0));
        // block 1's pattern is compared on the device and copied only when it differs
        same = same_pattern(Lv.A[0][0], Lv.A[1][1], cs);
        t1 = clock::now();
        for (int f = 0; f < (same ? 1 : 2); ++f) {
            const size_t nrp = (size_t)Lv.nodes(f) + 1, nci = (size_t)Lv.A[f][f].nnzb;
            buf[f] = std::make_unique<PinnedBuf<int32_t>>(nrp + nci);
            int32_t* h = buf[f]->p;
            rp[f] = h;
            ci[f] = h + nrp;
            MB_HIP(hipMemcpyAsync(h, Lv.A[f][f].rp.p, sizeof(int32_t) * nrp, hipMemcpyDeviceToHost, cs));
            if (nci) MB_HIP(hipMemcpyAsync(h + nrp, Lv.A[f][f].ci.p, sizeof(int32_t) * nci, hipMemcpyDeviceToHost, cs));
        }
        MB_HIP(hipStreamSynchronize(cs));
        t2 = clock::now();
    } catch (...) {
        (void)hipStreamSynchronize(cs);   // no copy may still write into a buffer going back to the pool
        (void)hipStreamDestroy(cs);
        throw;
    }
    (void)hipStreamDestroy(cs);
    struct Report {   // host time of the job's steps, printed when it ends
        bool on;
        int n;
        clock::time_point t0, t1, t2;
        ~Report() {
            if (!on) return;
            const auto t3 = clock::now();
            auto ms = [](clock::time_point a, clock::time_point b) {
                return std::chrono::duration<double, std::milli>(b - a).count();
            };
            std::fprintf(stderr, "[mbamg setup] colouring job, %d nodes: wait+compare %.2f ms, copy %.2f ms, "
                         "colour %.2f ms\n", n, ms(t0, t1), ms(t1, t2), ms(t2, t3));
        }
    } report{verbose, Lv.n, t0, t1, t2};
    for (int f = 0; f < 2; ++f) {
        BlockLevel& B = Lv.blk[f];
        B.d = Lv.d[f];
        if (f == 1 && same) {
            // same pattern: the same first-fit colouring, order and slices
            const BlockLevel& B0 = Lv.blk[0];
            B.colour = B0.colour;
            B.n = B0.n;
            B.n_colours = B0.n_colours;
            B.colour_row = B0.colour_row;
            B.perm = B0.perm;
            B.iperm = B0.iperm;
            B.sell_sorted = B0.sell_sorted;
            B.h_row0 = B0.h_row0;
            B.h_nrow = B0.h_nrow;
            B.colour_slice = B0.colour_slice;
            B.n_slices = B0.n_slices;
        } else {
            // A00 is structurally symmetric (checked with its strength graph); block 1's
            // pattern, when it differs, is symmetrised here
            std::vector<int32_t> trp, tci;
            const int nf = Lv.nodes(f);
            const bool asym = f == 1 && transpose_pattern(nf, rp[f], ci[f], trp, tci);
            int ncol = asym ? greedy_colour(nf, rp[f], ci[f], B.colour, trp.data(), tci.data())
                            : greedy_colour(nf, rp[f], ci[f], B.colour);
            order_and_slice(B, nf, ncol, rp[f]);
        }
    }
}

template <class T>
static void clone_buf(DevBuf<T>& dst, const DevBuf<T>& src, hipStream_t s) {
    dst.alloc(src.n);
    if (src.n) MB_HIP(hipMemcpyAsync(dst.p, src.p, src.bytes(), hipMemcpyDeviceToDevice, s));
}

static void clone_part(SellPart& d, const SellPart& p, hipStream_t s) {
    d.br = p.br;
    d.bc = p.bc;
    d.n_slots = p.n_slots;
    d.n_groups = p.n_groups;
    clone_buf(d.width, p.width, s);
    clone_buf(d.coff, p.coff, s);
    clone_buf(d.voff, p.voff, s);
    clone_buf(d.mask, p.mask, s);
    clone_buf(d.col, p.col, s);
    clone_buf(d.v64, p.v64, s);
    clone_buf(d.v32, p.v32, s);
    d.h_coff = p.h_coff;
    d.h_width = p.h_width;
    d.h_slot_nz = p.h_slot_nz;
    d.h_slot_blocks = p.h_slot_blocks;
}

// The colour order, slices and smoother parts of a block row: they depend on
// A and the colouring alone, not on the transfers or weights.
static void clone_smoother(BlockLevel& d, const BlockLevel& b, hipStream_t s) {
    d.d = b.d;
    d.n = b.n;
    d.n_colours = b.n_colours;
    d.n_slices = b.n_slices;
    d.split = b.split;
    d.cstats = b.cstats;
    d.all_nz = b.all_nz;
    d.all_bl = b.all_bl;
    d.perm = b.perm;
    d.iperm = b.iperm;
    d.sell_sorted = b.sell_sorted;
    d.colour = b.colour;
    d.h_row0 = b.h_row0;
    d.h_nrow = b.h_nrow;
    d.colour_slice = b.colour_slice;
    d.colour_row = b.colour_row;
    clone_buf(d.row0, b.row0, s);
    clone_buf(d.nrow, b.nrow, s);
    clone_buf(d.d_perm, b.d_perm, s);
    clone_buf(d.d_iperm, b.d_iperm, s);
    clone_part(d.off, b.off, s);
    clone_part(d.cpl, b.cpl, s);
    clone_part(d.diag, b.diag, s);
    clone_part(d.dinv, b.dinv, s);
}

// Join a build's coarsest inverse: the launches are issued, the inverse is
// checked, and stream s waits for it.
static void finish_coarse(mbamg_hierarchy* h, hipStream_t s) {
    if (!h->coarse_pending) return;
    PendingCoarse& pc = *h->coarse_pending;
    pc.job.get();
    MB_CHECK(pc.w.n == h->coarse_n, MBAMG_E_STATE, "internal: coarsest size");
    coarse_inverse_finish(pc.w, pc.side.stream);
    MB_HIP(hipEventRecord(pc.side.done, pc.side.stream));
    MB_HIP(hipStreamWaitEvent(s, pc.side.done, 0));
    h->coarse_pending.reset();
}

// from: a setup of the same blocks with the same level-0 parameters
// (aggregation, precision) running at the same time; its level-0 aggregates
// and smoother data are copied instead of recomputed.  to: this setup
// publishes its own level-0 aggregates and smoother data there.
static void setup_impl(mbamg_hierarchy* h, const mbamg_bsr* Ab, hipStream_t s, DonorLink* from, DonorLink* to,
                       bool defer_coarse) {
    struct Publish {   // on every exit, whatever this setup has not published is not coming
        DonorLink* to;
        ~Publish() { if (to) to->close(); }
    } publish_guard{to};
    const Level* donor0 = nullptr;   // the donor's level 0, once its aggregates are published
    auto t0 = std::chrono::steady_clock::now();
    const mbamg_params& p = h->p;
    const int d0 = h->d[0], d1 = h->d[1];
    const int N = Ab[0].n_brows;
    const int N1 = Ab[3].n_brows;
    MB_CHECK(N > 0 && N1 > 0, MBAMG_E_INVALID, "empty system");
    const bool separate = p.clone_aggregates == 0;
    MB_CHECK(separate || N1 == N, MBAMG_E_INVALID,
             "cloned aggregation needs co-located fields (equal node counts of A_00 and A_11)");
    const bool want32 = p.precision == 1;
    PhaseClock clk(s);
    h->coarse_pending = std::make_unique<PendingCoarse>();
    CoarseWork& cwork = h->coarse_pending->w;
    SideStream& side = h->coarse_pending->side;
    // host colouring jobs per level; joined before their level's smoother data is built
    // (and, on an error, waited for when the futures go out of scope, before the events)
    std::vector<hipEvent_t> colour_events;
    struct EventList {
        std::vector<hipEvent_t>& e;
        ~EventList() { for (auto ev : e) (void)hipEventDestroy(ev); }
    } colour_events_guard{colour_events};
    std::map<int, std::future<void>> colour_jobs;
    int device = 0;
    MB_HIP(hipGetDevice(&device));
    std::future<void>& coarse_job = h->coarse_pending->job;

    // level 0 from the caller's blocks
    auto first = std::make_unique<Level>();
    first->n = N;
    first->n1 = N1;
    first->d[0] = d0;
    first->d[1] = d1;
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g)
            copy_block(Ab[f * 2 + g], first->A[f][g], first->nodes(f), first->nodes(g), h->d[f], h->d[g], s);
    MB_CHECK(first->A[0][0].nnzb > 0 && first->A[1][1].nnzb > 0, MBAMG_E_INVALID, "diagonal blocks must be nonzero");
    h->L.push_back(std::move(first));

    // near-null space per block: constants on the finest level
    DevBuf<double> Bn[2];
    for (int f = 0; f < 2; ++f) {
        const int64_t nb = (int64_t)h->L[0]->nodes(f) * h->d[f];
        Bn[f].alloc((size_t)nb);
        fill_ones(Bn[f].p, nb, s);
    }
    int lvl = 0;
    while (true) {
        Level& cur = *h->L.back();
        const int64_t ndof = cur.ndof();
        if (ndof <= p.max_coarse || (int)h->L.size() >= p.max_levels) break;
        clk.mark("start", lvl);
        if (lvl == 0 && from && from->agg.get()) {
            MB_HIP(hipStreamWaitEvent(s, from->agg_ev, 0));
            if (from->level0->n == cur.n) donor0 = from->level0;
        }
        const bool donor_level = lvl == 0 && donor0 != nullptr;
        // level 0's pattern is final now: its colouring starts before aggregation (the job
        // is simply not used if level 0 turns out to be the coarsest)
        if (lvl == 0 && !donor_level) {
            hipEvent_t ev = nullptr;
            MB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            colour_events.push_back(ev);
            MB_HIP(hipEventRecord(ev, s));
            Level* lp = &cur;
            colour_jobs[lvl] = std::async(std::launch::async, [lp, ev, device] { colour_level(*lp, ev, device); });
        }
        Aggregates& G = cur.G;
        if (donor_level) {
            const Aggregates& D = donor0->G;
            G.n = D.n;
            G.n_agg = D.n_agg;
            G.mis_rounds = D.mis_rounds;
            clone_buf(G.agg, D.agg, s);
            clone_buf(G.mptr, D.mptr, s);
            clone_buf(G.midx, D.midx, s);
        } else {
            Strength S = build_strength(cur.A[0][0], p.theta, s);
            clk.mark("strength", lvl);
            G = build_aggregates(S, p.seed, lvl, s);
        }
        if (separate) {   // block 1 from the graph of its own diagonal block (Sec. 4.3.1)
            Strength S1 = build_strength(cur.A[1][1], p.theta, s);
            cur.G1 = build_aggregates(S1, p.seed, lvl, s);
            cur.separate = true;
        }
        clk.mark("aggregates", lvl);
        const bool stop = separate ? (double)(G.n_agg + cur.G1.n_agg) > 0.9 * ((double)cur.n + cur.n1)
                                   : (double)G.n_agg > 0.9 * cur.n;
        if (stop) {   // this level is the coarsest
            G = Aggregates();
            cur.G1 = Aggregates();
            cur.separate = false;
            break;
        }
        if (to && lvl == 0) {
            to->level0 = &cur;
            MB_HIP(hipEventRecord(to->agg_ev, s));
            to->publish_agg(true);
        }
        // this level is not the coarsest: colour it on a host thread while the GPU
        // builds the next level (the level-0 colouring comes with the donor's copy)
        if (!donor_level && !colour_jobs.count(lvl)) {
            hipEvent_t ev = nullptr;
            MB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            colour_events.push_back(ev);
            MB_HIP(hipEventRecord(ev, s));
            Level* lp = &cur;
            colour_jobs[lvl] = std::async(std::launch::async, [lp, ev, device] { colour_level(*lp, ev, device); });
        }
        const int nc = G.n_agg;
        DevBuf<double> q[2], Bc[2];
        for (int f = 0; f < 2; ++f) {     // block 1 reuses block 0's aggregates unless aggregated separately
            const Aggregates& Gf = cur.agg_of(f);
            q[f].alloc((size_t)cur.nodes(f) * h->d[f]);
            Bc[f].alloc((size_t)std::max(Gf.n_agg, 1) * h->d[f]);
            build_tentative(Gf, h->d[f], Bn[f].p, q[f].p, Bc[f].p, s);
        }
        auto nxt = std::make_unique<Level>();
        nxt->n = nc;
        nxt->n1 = cur.agg_of(1).n_agg;
        nxt->d[0] = d0;
        nxt->d[1] = d1;
        // A_c[f][g] = P_f^T A_fg P_g.  The four block pairs usually share one
        // pattern; the symbolic phase then runs once and the rest reuse it.
        auto galerkin_all = [&](const SetupBsr (&P)[2], const SetupBsr (&PT)[2]) {
            const bool sameP = same_pattern(P[0], P[1], s);
            // block pairs whose A block and prolongators have the same patterns form one group:
            // its products T = A_fg P_g and P_f^T T share their patterns and one launch each
            std::vector<std::vector<int>> groups;
            for (int k = 0; k < 4; ++k) {
                const int f = k / 2, g = k % 2;
                bool placed = false;
                for (auto& grp : groups) {
                    const int f2 = grp[0] / 2, g2 = grp[0] % 2;
                    if ((f2 == f || sameP) && (g2 == g || sameP) && cur.A[f2][g2].nnzb > 0 &&
                        same_pattern(cur.A[f][g], cur.A[f2][g2], s)) {
                        grp.push_back(k);
                        placed = true;
                        break;
                    }
                }
                if (!placed) groups.push_back({k});
            }
            SetupBsr T[2][2];
            for (const auto& grp : groups) {
                const SetupBsr* Aa[4];
                const SetupBsr* Pb[4];
                const SetupBsr* PTa[4];
                const SetupBsr* Tb[4];
                SetupBsr* Tc[4];
                SetupBsr* Cc[4];
                const int K = (int)grp.size();
                for (int u = 0; u < K; ++u) {
                    const int f = grp[u] / 2, g = grp[u] % 2;
                    Aa[u] = &cur.A[f][g];
                    Pb[u] = &P[g];
                    PTa[u] = &PT[f];
                    Tb[u] = &T[f][g];
                    Tc[u] = &T[f][g];
                    Cc[u] = &nxt->A[f][g];
                }
                spgemm_multi(Aa, Pb, K, Tc, s);
                spgemm_multi(PTa, Tb, K, Cc, s);
            }
        };
        if (p.learned != 0 || p.omega_p != 0.0) {
            choose_weights(h, cur, G, lvl, s);
            clk.mark("weights", lvl);
            for (int f = 0; f < 2; ++f) {
                cur.P[f] = sa_prolongator(cur.A[f][f], h->fm.n_vec[f], G, q[f].p, cur.wp_agg.p, s);
                cur.PT[f] = block_transpose(cur.P[f], s);
            }
            clk.mark("smoothed P, P^T", lvl);
            galerkin_all(cur.P, cur.PT);
            cur.smoothed = true;
        } else {
            SetupBsr P[2], PT[2];
            for (int f = 0; f < 2; ++f) {
                P[f] = tentative_bsr(cur.agg_of(f), h->d[f], q[f].p, s);
                PT[f] = block_transpose(P[f], s);
            }
            galerkin_all(P, PT);
        }
        clk.mark("tentative+galerkin", lvl);
        // keep q on the fine level (natural order) for the transfer maps
        cur.blk[0].q64 = std::move(q[0]);
        cur.blk[1].q64 = std::move(q[1]);
        Bn[0] = std::move(Bc[0]);
        Bn[1] = std::move(Bc[1]);
        h->L.push_back(std::move(nxt));
        ++lvl;
    }
    h->L.back()->coarsest = true;
    // the finest level starts its colouring job before aggregation; when that level turns
    // out to be the coarsest (aggregation kept more than 90 % of its nodes) the job writes
    // the same order fields the coarsest level's identity order goes into below: join it first
    {
        auto job = colour_jobs.find((int)h->L.size() - 1);
        if (job != colour_jobs.end()) {
            job->second.get();
            colour_jobs.erase(job);
        }
    }

    // coarsest: dense inverse
    {
        Level& c = *h->L.back();
        // the coarsest inverse runs on a second stream, overlapping the smoother data below
        MB_HIP(hipEventRecord(side.ready, s));
        MB_HIP(hipStreamWaitEvent(side.stream, side.ready, 0));
        // its thousands of small launches are issued from a host thread of their own, so this
        // thread goes on queueing the smoother data at once
        h->coarse_n = (int)c.ndof();
        Level* cp = &c;
        coarse_job = std::async(std::launch::async, [h, cp, &cwork, &side, device] {
            MB_HIP(hipSetDevice(device));
            coarse_inverse_launch(cp->A, cp->d, h->coarse_inv, cwork, side.stream);
        });
        clk.mark("coarse inverse queued", (int)h->L.size() - 1);
        for (int f = 0; f < 2; ++f) {      // identity order
            BlockLevel& B = c.blk[f];
            B.d = c.d[f];
            B.n = c.nodes(f);
            B.colour.assign(c.nodes(f), 0);
            order_and_slice(B, c.nodes(f), 1);   // one colour: identity order, slices for the transfer kernels
            B.row0.upload(B.h_row0, s);
            B.nrow.upload(B.h_nrow, s);
            B.d_perm.upload(B.perm, s);   // used at the interface when this is the only level
            B.d_iperm.upload(B.iperm, s);
        }
        if (h->L.size() == 1) {
            // the only level: the operator apply of the Krylov solver reads its blocks in the
            // sliced form (FP64, identity order, one colour); the V-cycle is the dense solve
            for (int f = 0; f < 2; ++f) {
                BlockLevel& B = c.blk[f];
                const int g = 1 - f;
                build_part(B.off, PartKind::Off, B, &c.A[f][f], B.d_iperm.p, c.A[f][f].val.p, c.d[f], c.d[f], false,
                           s);
                build_part(B.diag, PartKind::Diag, B, &c.A[f][f], B.d_iperm.p, c.A[f][f].val.p, c.d[f], c.d[f],
                           false, s);
                build_part(B.cpl, PartKind::Cpl, B, &c.A[f][g], c.blk[g].d_iperm.p, c.A[f][g].val.p, c.d[f], c.d[g],
                           false, s);
            }
            c.apply_parts = true;
        }
        alloc_vecs(c.v64, c.ndof());
        if (want32) alloc_vecs(c.v32, c.ndof());
    }

    // smoother format on every other level, in two passes: first each level's own smoother
    // blocks (its colouring, order and parts), then the transfers, which need the next
    // level's order.  A build that lends its level 0 does that level first and publishes
    // it at once; a build that borrows it does it last.
    const int n_fine_levels = (int)h->L.size() - 1;
    for (int k = 0; k < n_fine_levels; ++k) {
        const int l = to ? k : n_fine_levels - 1 - k;
        Level& Lv = *h->L[l];
        bool shared = l == 0 && donor0 != nullptr && from->smooth.get();
        if (shared) {
            MB_HIP(hipStreamWaitEvent(s, from->smooth_ev, 0));
            for (int f = 0; f < 2; ++f) clone_smoother(Lv.blk[f], donor0->blk[f], s);
            clk.mark("smoother data copied", l);
        }
        // colouring is sequential by definition (first fit in node order): done on the host from
        // the patterns of the diagonal blocks, by the job started when the level was built
        if (!shared) {
            auto job = colour_jobs.find(l);
            if (job != colour_jobs.end()) {
                job->second.get();
            } else {
                hipEvent_t ev = nullptr;
                MB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
                colour_events.push_back(ev);
                MB_HIP(hipEventRecord(ev, s));
                colour_level(Lv, ev, device);
            }
            clk.mark("colouring joined", l);
        }
        for (int f = 0; f < 2 && !shared; ++f) {
            BlockLevel& B = Lv.blk[f];
            B.row0.upload(B.h_row0, s);
            B.nrow.upload(B.h_nrow, s);
            B.d_perm.upload(B.perm, s);
            B.d_iperm.upload(B.iperm, s);
        }
        // coarse levels with few rows per colour take the row form: every colour pass is a short,
        // latency-bound launch, and one wavefront per row (four on rows of 4 x 4 blocks) shortens
        // its chain of dependent loads (the 128^3 workload's third level, 7461 nodes in 11
        // colours: 10.8 -> 7.3 us per pass; 2735 nodes in 28 colours with smoothed transfers:
        // 15 -> 6.7 us; the 64^3 workload's second level, 23,915 nodes in 9 colours: 819 -> 665 us
        // per FP64 V-cycle).  Larger levels keep the sliced layout, whose rows are sorted by
        // length within each colour when their lengths differ (the 128^3 workload's second
        // level, 188,588 nodes: 9 colours 0.80 against 1.10 ms per FP64 V-cycle in the row form;
        // 18 colours with smoothed transfers 1.36 against 1.56 ms).  The row form's sliced parts
        // are not built.
        const int max_colours = std::max(Lv.blk[0].n_colours, Lv.blk[1].n_colours);
        bool rows_level = l > 0 && (int64_t)std::max(Lv.n, Lv.n1) <= (int64_t)ROWS_PER_COLOUR_MAX * max_colours;
        // MBAMG_ROWS_FORM (tests): "rows" forces the row form on every coarse level, anything else the sliced one
        if (const char* fo = form_override("MBAMG_ROWS_FORM")) rows_level = l > 0 && std::strcmp(fo, "rows") == 0;
        if (p.smoother == 1) rows_level = false;   // the full-node kernel reads the sliced parts
        for (int f = 0; f < 2 && !shared; ++f) {
            const int g = 1 - f;
            BlockLevel& B = Lv.blk[f];
            const int df = Lv.d[f], dg = Lv.d[g];
            const int nf = Lv.nodes(f);
            DevBuf<double> dinv((size_t)nf * df * df);
            if (f == 0) clk.mark("colouring", l);
            build_dinv(Lv.A[f][f], dinv.p, s);
            clk.mark("dinv", l);
            B.rows = rows_level;
            if (B.rows) {
                // the per-colour counts the sliced parts would have recorded (byte model)
                const std::vector<int64_t> cs7 =
                    row_colour_stats(nf, B.d_perm.p, Lv.A[f][f], Lv.A[f][g], dinv.p, B.colour_row, s);
                B.cstats.assign(B.n_colours, ColourStats{});
                for (int c = 0; c < B.n_colours; ++c) {
                    ColourStats& cs = B.cstats[c];
                    const int64_t* v = &cs7[(size_t)c * 7];
                    cs.off_nz = v[0];
                    cs.off_bl = v[1];
                    cs.cpl_nz = v[2];
                    cs.cpl_bl = v[3];
                    cs.dinv_nz = v[4];
                    B.all_nz += v[0] + v[2] + v[5];
                    B.all_bl += v[1] + v[3] + v[6];
                }
                B.split = 1;
                // few rows per colour (small, latency-bound launches): a workgroup's four
                // wavefronts share each row, for shorter chains of dependent passes (measured
                // 12 % faster on a 98-rows-per-colour level, 60 % slower on 10K rows per colour)
                B.row_split = (df == 4 && nf <= 1024 * std::max(1, B.n_colours)) ? 4 : 1;
                if (const char* fo = form_override("MBAMG_ROW_SPLIT")) B.row_split = df == 4 ? std::atoi(fo) : 1;
                build_rows(B.raff, nf, B.d_perm.p, Lv.A[f][f], B.d_iperm.p, want32, s);
                build_rows(B.rafg, nf, B.d_perm.p, Lv.A[f][g], Lv.blk[g].d_iperm.p, want32, s);
                B.rdinv64.alloc((size_t)nf * df * df);
                gather_blocks(nf, df * df, B.d_perm.p, dinv.p, B.rdinv64.p, s);
                if (want32) {
                    B.rdinv32.alloc((size_t)nf * df * df);
                    cast_to_f32(B.rdinv64.p, B.rdinv32.p, (int64_t)nf * df * df, s);
                }
                MB_HIP(hipStreamSynchronize(s));   // dinv is released at the end of this iteration
                if (clk.on)
                    std::fprintf(stderr, "[mbamg setup] level %d block %d: %d nodes, %d colours, row form\n", l, f,
                                 nf, B.n_colours);
                continue;
            }
            build_part(B.off, PartKind::Off, B, &Lv.A[f][f], B.d_iperm.p, Lv.A[f][f].val.p, df, df, want32, s);
            build_part(B.diag, PartKind::Diag, B, &Lv.A[f][f], B.d_iperm.p, Lv.A[f][f].val.p, df, df, want32, s);
            build_part(B.cpl, PartKind::Cpl, B, &Lv.A[f][g], Lv.blk[g].d_iperm.p, Lv.A[f][g].val.p, df, dg, want32,
                       s);
            build_part(B.dinv, PartKind::Dinv, B, nullptr, nullptr, dinv.p, df, df, want32, s);
            B.cstats.assign(B.n_colours, ColourStats{});
            int64_t slots = 0;
            for (int c = 0; c < B.n_colours; ++c) {
                ColourStats& cs = B.cstats[c];
                int64_t nz, bl;
                B.off.stats(B.colour_slice[c], B.colour_slice[c + 1], cs.off_nz, cs.off_bl);
                B.cpl.stats(B.colour_slice[c], B.colour_slice[c + 1], cs.cpl_nz, cs.cpl_bl);
                B.dinv.stats(B.colour_slice[c], B.colour_slice[c + 1], cs.dinv_nz, bl);
                B.diag.stats(B.colour_slice[c], B.colour_slice[c + 1], nz, bl);
                B.all_nz += cs.off_nz + cs.cpl_nz + nz;
                B.all_bl += cs.off_bl + cs.cpl_bl + bl;
            }
            for (int sl = 0; sl < B.n_slices; ++sl) slots += B.off.h_width[sl] + B.cpl.h_width[sl];
            // split each slice's slots over several waves when a colour has too few slices to
            // fill the chip and the rows are wide enough to share
            const double avg_width = B.n_slices ? (double)slots / B.n_slices : 0.0;
            const double per_colour = (double)B.n_slices / std::max(1, B.n_colours);
            B.split = slot_split(per_colour, avg_width);
            // MBAMG_SLICE_SPLIT = 1 | 2 | 4 | 8 | 16 forces the waves per slice on every sliced
            // level, for tests: the split changes the order of each row's partial sums
            if (const char* fo = form_override("MBAMG_SLICE_SPLIT")) {
                const int P = std::atoi(fo);
                MB_CHECK(P == 1 || P == 2 || P == 4 || P == 8 || P == 16, MBAMG_E_INVALID,
                         "MBAMG_SLICE_SPLIT must be 1, 2, 4, 8 or 16");
                B.split = P;
            }
            if (clk.on)
                std::fprintf(stderr, "[mbamg setup] level %d block %d: %d nodes, %d colours, %d slices, %.1f slots/slice, "
                             "split %d\n", l, f, nf, B.n_colours, B.n_slices, avg_width, B.split);
        }
        // the residual is one launch over both blocks' slices, not one colour: its split is
        // chosen for the whole level, up to about 32K waves (MBAMG_SLICE_SPLIT forces both)
        Lv.resid_split = std::max(Lv.blk[0].split, Lv.blk[1].split);
        if (l > 0 && !Lv.blk[0].rows && !Lv.blk[1].rows && !form_override("MBAMG_SLICE_SPLIT")) {
            int64_t slots = 0, slices = 0;
            for (int f = 0; f < 2; ++f) {
                const BlockLevel& B = Lv.blk[f];
                for (int sl = 0; sl < B.n_slices; ++sl) slots += B.off.h_width[sl] + B.cpl.h_width[sl];
                slices += B.n_slices;
            }
            Lv.resid_split = slot_split((double)slices, slices ? (double)slots / (double)slices : 0.0, 32768);
        }
        // the residual's launch order: the same eighth of every colour together, so the blocks
        // each XCD takes (contiguous launch ranges) cover one slab of the domain in all colours
        // and their neighbour gathers stay in its L2 (in colour order an XCD's range spans a
        // whole colour, i.e. the whole domain)
        if (l > 0 && !Lv.blk[0].rows && !Lv.blk[1].rows)
            for (int f = 0; f < 2; ++f) Lv.resid_order[f].upload(slab_order(Lv.blk[f].colour_slice), s);
        clk.mark("sliced parts", l);
        if (p.smoother == 1) {
            // nodal-block Gauss-Seidel over the full node blocks: both blocks in one colour
            // order, valid for the whole node graph (the coupling blocks inside A00's pattern)
            const BlockLevel& B0 = Lv.blk[0];
            const BlockLevel& B1 = Lv.blk[1];
            MB_CHECK(B0.colour == B1.colour && B0.perm == B1.perm && B0.h_row0 == B1.h_row0, MBAMG_E_INVALID,
                     "the full-node smoother needs the two diagonal blocks' patterns equal");
            MB_CHECK(within_pattern(Lv.A[0][0], Lv.A[0][1], s) && within_pattern(Lv.A[0][0], Lv.A[1][0], s) &&
                         within_pattern(Lv.A[0][0], Lv.A[1][1], s),
                     MBAMG_E_INVALID, "the full-node smoother needs every block's pattern inside A00's");
            build_node_inverses(Lv.A, B0.n_slices, B0.row0.p, B0.nrow.p, B0.d_perm.p, Lv.fc_mask, Lv.fc_off,
                                Lv.fc_inv64, want32 ? &Lv.fc_inv32 : nullptr, s);
            Lv.fc = true;
            clk.mark("full node inverses", l);
        }
        if (l == 0 && to && to->agg_set) {   // level 0's smoother blocks are complete on s
            MB_HIP(hipEventRecord(to->smooth_ev, s));
            to->publish_smooth(true);
        }
        MB_HIP(hipStreamSynchronize(s));
    }
    for (int l = n_fine_levels - 1; l >= 0; --l) {
        Level& Lv = *h->L[l];
        Level& Nx = *h->L[l + 1];
        // transfers between this level's and the next level's colour orders
        for (int f = 0; f < 2 && Lv.smoothed; ++f) {
            BlockLevel& B = Lv.blk[f];
            BlockLevel& C = Nx.blk[f];
            build_part(B.pro, PartKind::Cpl, B, &Lv.P[f], C.d_iperm.p, Lv.P[f].val.p, B.d, B.d, want32, s);
            // P^T sliced over the next level's rows in natural order: neighbouring aggregates,
            // whose rows gather the same fine rows, share slices and stay on one XCD (in the
            // colour order a slice mixes aggregates from all over the domain: 4x the
            // algorithmic bytes fetched on the finest level)
            BlockLevel nat;
            natural_slicing(nat, Nx.nodes(f), s);
            build_part(B.res, PartKind::Cpl, nat, &Lv.PT[f], B.d_iperm.p, Lv.PT[f].val.p, B.d, B.d, want32, s);
            B.res_row0 = std::move(nat.row0);
            B.res_nrow = std::move(nat.nrow);
            B.res_slices = nat.n_slices;
            // a next level of at most RES_ROWS_MAX rows has few, wide P^T rows (hundreds of
            // blocks): one wavefront per row instead of a few slices' long chains (MBAMG_XFER_FORM
            // = rows | sliced forces a form, for tests; the summation order differs)
            B.res_rows = Nx.nodes(f) <= RES_ROWS_MAX;
            if (const char* fo = form_override("MBAMG_XFER_FORM")) B.res_rows = std::strcmp(fo, "rows") == 0;
            if (B.res_rows) build_rows(B.rres, Nx.nodes(f), nat.d_perm.p, Lv.PT[f], B.d_iperm.p, want32, s);
            B.pro_split = transfer_split(B.pro, B.n_slices);
            B.res_split = transfer_split(B.res, B.res_slices);
        }
        for (int f = 0; f < 2 && Lv.damped; ++f) {
            BlockLevel& B = Lv.blk[f];
            B.w_row64.alloc(std::max(Lv.n, 1));
            row_damping<double>(Lv.n, B.d_perm.p, Lv.G.agg.p, Lv.ws_agg.p, B.w_row64.p, s);
            if (want32) {
                B.w_row32.alloc(std::max(Lv.n, 1));
                row_damping<float>(Lv.n, B.d_perm.p, Lv.G.agg.p, Lv.ws_agg.p, B.w_row32.p, s);
            }
        }
        for (int f = 0; f < 2 && !Lv.smoothed; ++f) {
            BlockLevel& B = Lv.blk[f];
            const BlockLevel& C = Nx.blk[f];
            const Aggregates& Gf = Lv.agg_of(f);
            const int nf = Lv.nodes(f);
            transfer_maps(nf, Nx.nodes(f), B.d_perm.p, B.d_iperm.p, Gf.agg.p, C.d_perm.p, C.d_iperm.p, Gf.mptr.p,
                          Gf.midx.p, B.agg_p, B.mem_ptr, B.mem_idx, s);
            B.res_group = restrict_group(Lv.n + Lv.n1, Nx.n + Nx.n1);
            DevBuf<double> qp((size_t)nf * B.d);
            launch_gather(nf, B.d, B.d_perm.p, B.q64.p, qp.p, s);
            B.q64 = std::move(qp);
            B.qm64.alloc((size_t)nf * B.d);
            launch_gather(nf, B.d, B.mem_idx.p, B.q64.p, B.qm64.p, s);   // member m: fine row mem_idx[m]
            if (want32) {
                B.q32.alloc((size_t)nf * B.d);
                cast_to_f32(B.q64.p, B.q32.p, (int64_t)nf * B.d, s);
                B.qm32.alloc((size_t)nf * B.d);
                cast_to_f32(B.qm64.p, B.qm32.p, (int64_t)nf * B.d, s);
            }
        }
        alloc_vecs(Lv.v64, Lv.ndof());
        if (want32) alloc_vecs(Lv.v32, Lv.ndof());
        MB_HIP(hipStreamSynchronize(s));
    }

    clk.mark("smoother data done", 0);
    if (!defer_coarse) {
        finish_coarse(h, s);
        clk.mark("coarse inverse joined", 0);
    }
    // Krylov workspace
    h->n_fine = h->L[0]->ndof();
    const int m = p.restart;
    const int64_t n = h->n_fine;
    h->V.alloc((size_t)(m + 1) * n);
    if (want32) {
        h->Z32.alloc((size_t)m * n);
        h->vin32.alloc(n);
        h->ztmp.alloc(n);
    } else {
        h->Z64.alloc((size_t)m * n);
    }
    h->w.alloc(n);
    h->xw.alloc(n);
    h->bw.alloc(n);
    h->vio.alloc(n);
    h->vio2.alloc(n);
    h->partial.alloc((size_t)KBLOCKS * KMAXQ);
    h->hbuf.alloc(KB_TOTAL);
    h->ybuf.alloc(KMAXQ);
    h->coef.alloc(KC_TOTAL);
    MB_HIP(hipHostMalloc((void**)&h->hbuf_host, sizeof(double) * KB_TOTAL, hipHostMallocDefault));
    MB_HIP(hipHostMalloc((void**)&h->coef_host, sizeof(double) * KC_TOTAL, hipHostMallocDefault));
    MB_HIP(hipHostMalloc((void**)&h->y_host, sizeof(double) * KMAXQ, hipHostMallocDefault));
    MB_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    h->t_setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    int64_t nz0 = h->L[0]->nnzb_total(), nzs = 0;
    for (auto& lv : h->L) nzs += lv->nnzb_total();
    h->info.levels = (int)h->L.size();
    h->info.op_complexity = nz0 ? (double)nzs / (double)nz0 : 1.0;
    h->info.t_setup_ms = h->t_setup_ms;
}

// ----------------------------------------------------------------------------
// byte model (algorithmic bytes of the finest level's kernels)
// ----------------------------------------------------------------------------
static double gs_bytes(const BlockLevel& B, int c, bool zero_x, bool skip_off, bool cpl, int s, int dg) {
    const ColourStats& cs = B.cstats[c];
    const int64_t rows = B.colour_row[c + 1] - B.colour_row[c];
    double bytes = 0.0;
    if (!skip_off) bytes += cs.off_nz * (double)s + 4.0 * cs.off_bl + (double)rows * B.d * s;  // values, indices, gathered iterate
    if (cpl) bytes += cs.cpl_nz * (double)s + 4.0 * cs.cpl_bl + (double)rows * dg * s;
    bytes += cs.dinv_nz * (double)s;
    bytes += 4.0 * rows;                                        // row pointer equivalent
    bytes += (double)rows * B.d * s * (zero_x ? 3 : 4);         // b, (x), t, xn
    return bytes;
}

static double resid_bytes(const Level& Lv, int s, bool with_b) {
    double bytes = 0.0;
    for (int f = 0; f < 2; ++f) {
        const BlockLevel& B = Lv.blk[f];
        bytes += B.all_nz * (double)s + 4.0 * B.all_bl + 4.0 * B.n;
        bytes += (double)B.n * B.d * s * (with_b ? 4 : 3);   // x_f, x_g gathered, (b), r
    }
    return bytes;
}

// smoothed transfer y (+)= A x in sliced form: structural values, stored block
// indices, one 4-byte slice-row entry per output row, the input vector once,
// the output written (and read when accumulating)
static double xfer_bytes(const SellPart& P, int64_t rows_out, int64_t rows_in, int d, int s, bool accumulate) {
    int64_t nz = 0, bl = 0;
    P.stats(0, (int)P.h_width.size(), nz, bl);
    return nz * (double)s + 4.0 * bl + 4.0 * rows_out + (double)rows_in * d * s +
           (double)rows_out * d * s * (accumulate ? 2 : 1);
}

// tentative transfers: the restriction reads r and q once and writes b_c, with
// the member lists; the prolongation reads q, x_c and x and writes x, with the
// aggregate map
static double tentative_restrict_bytes(const Level& Lv, const Level& Nx, int s) {
    const int64_t nf = Lv.ndof(), nc = Nx.ndof();
    return (double)s * (2.0 * nf + nc) + 4.0 * ((double)Lv.n + Lv.n1 + Nx.n + Nx.n1);
}
static double tentative_prolong_bytes(const Level& Lv, const Level& Nx, int s) {
    const int64_t nf = Lv.ndof(), nc = Nx.ndof();
    return (double)s * (3.0 * nf + nc) + 4.0 * ((double)Lv.n + Lv.n1);
}

// Algorithmic bytes of level l's share of one V-cycle in the hierarchy's form:
// down = pre-smoothing, residual and restriction; up = prolongation and
// post-smoothing.  The coarsest level's direct solve (the inverse read once,
// the vectors in and out) counts as down.
static void level_vcycle_bytes(const mbamg_hierarchy* h, int l, double& down, double& up) {
    const int s = h->p.precision == 1 ? 4 : 8;
    down = up = 0.0;
    const Level& Lv = *h->L[l];
    if (Lv.coarsest) {
        down = 8.0 * (double)h->coarse_n * h->coarse_n + 2.0 * s * h->coarse_n;
        return;
    }
    const Level& Nx = *h->L[l + 1];
    for (int sweep = 0; sweep < 2 * h->p.bgs_sweeps; ++sweep) {
        const bool zero = sweep == 0;
        double& acc = sweep < h->p.bgs_sweeps ? down : up;
        for (int f = 0; f < 2; ++f) {
            const BlockLevel& B = Lv.blk[f];
            for (int k = 0; k < h->p.inner_sweeps; ++k)
                for (int c = 0; c < B.n_colours; ++c) {
                    const bool skip = zero && k == 0 && c == 0;
                    const bool cpl = !(zero && f == 0);
                    acc += gs_bytes(B, c, zero, skip, cpl, s, Lv.d[1 - f]);
                }
        }
    }
    down += resid_bytes(Lv, s, true);
    if (Lv.smoothed) {
        for (int f = 0; f < 2; ++f) {
            down += xfer_bytes(Lv.blk[f].res, Nx.n, Lv.n, Lv.d[f], s, false);
            up += xfer_bytes(Lv.blk[f].pro, Lv.n, Nx.n, Lv.d[f], s, true);
        }
    } else {
        down += tentative_restrict_bytes(Lv, Nx, s);
        up += tentative_prolong_bytes(Lv, Nx, s);
    }
}

// timing kinds beyond the finest level's launches: the whole V-cycle as the
// Krylov solver and the probe apply it, and each level's share
constexpr int TK_VCYCLE = 4, TK_LEVEL = 16;   // level l: TK_LEVEL + 2 l (down), + 1 (up)
// launch kinds: 0 post-smoother colour passes, 1 residual, 3 other colour passes,
// 5 restriction, 6 prolongation; kinds 0..3 keep their meaning on the finest
// level, other levels add 64 + 8 l
static int launch_kind(int l, int k) { return l == 0 ? k : 64 + 8 * l + k; }

// ----------------------------------------------------------------------------
// V-cycle
// ----------------------------------------------------------------------------
template <class T>
static Vecs<T>& vecs(Level& L);
template <>
Vecs<double>& vecs<double>(Level& L) { return L.v64; }
template <>
Vecs<float>& vecs<float>(Level& L) { return L.v32; }

template <class T>
static RowView<T> rview(const RowPart& R);
template <>
RowView<double> rview<double>(const RowPart& R) { return {R.rp.p, R.col.p, R.v64.p}; }
template <>
RowView<float> rview<float>(const RowPart& R) { return {R.rp.p, R.col.p, R.v32.p}; }
template <class T>
static const T* rdinv(const BlockLevel& B);
template <>
const double* rdinv<double>(const BlockLevel& B) { return B.rdinv64.p; }
template <>
const float* rdinv<float>(const BlockLevel& B) { return B.rdinv32.p; }

template <class T>
static const T* qptr(const BlockLevel& B);
template <>
const double* qptr<double>(const BlockLevel& B) { return B.q64.p; }
template <>
const float* qptr<float>(const BlockLevel& B) { return B.q32.p; }

template <class T>
static const T* qmptr(const BlockLevel& B);
template <>
const double* qmptr<double>(const BlockLevel& B) { return B.qm64.p; }
template <>
const float* qmptr<float>(const BlockLevel& B) { return B.qm32.p; }

template <class T>
static const T* wrow(const BlockLevel& B);
template <>
const double* wrow<double>(const BlockLevel& B) { return B.w_row64.p; }
template <>
const float* wrow<float>(const BlockLevel& B) { return B.w_row32.p; }

template <class T>
static const T* fc_inv(const Level& Lv);
template <>
const double* fc_inv<double>(const Level& Lv) { return Lv.fc_inv64.p; }
template <>
const float* fc_inv<float>(const Level& Lv) { return Lv.fc_inv32.p; }

// One sweep of the nodal-block Gauss-Seidel over the full node blocks (both
// blocks of a node relaxed together, colour by colour) from x (NULL: zero)
// into xn; b, x and xn hold both blocks.
template <class T>
static void smooth_fc(mbamg_hierarchy* h, int l, bool zero, const T* b, const T* x, T* xn, hipStream_t s) {
    Level& Lv = *h->L[l];
    const BlockLevel& B0 = Lv.blk[0];
    const int64_t n0 = (int64_t)Lv.n * Lv.d[0];
    T* t = vecs<T>(Lv).t.p;
    const int P = std::max(Lv.blk[0].split, Lv.blk[1].split);
    for (int k = 0; k < h->p.inner_sweeps; ++k)
        for (int c = 0; c < B0.n_colours; ++c) {
            GsFcArgs<T> a{};
            a.s_begin = B0.colour_slice[c];
            a.s_count = B0.colour_slice[c + 1] - B0.colour_slice[c];
            a.sl = B0.slices();
            for (int f = 0; f < 2; ++f) {
                const int64_t off = f ? n0 : 0;
                a.off[f] = Lv.blk[f].off.view<T>();
                a.cpl[f] = Lv.blk[f].cpl.view<T>();
                a.b[f] = b + off;
                a.x[f] = x ? x + off : nullptr;
                a.t[f] = t + off;
                a.xn[f] = xn + off;
            }
            a.dinv = fc_inv<T>(Lv);
            a.dmask = Lv.fc_mask.p;
            a.doff = Lv.fc_off.p;
            a.cstart = k == 0 ? B0.colour_row[c] : INT_MAX;
            a.omega = (T)h->p.omega;
            a.w_row = Lv.damped ? wrow<T>(Lv.blk[0]) : nullptr;
            a.skip_off = (zero && k == 0 && c == 0) ? 1 : 0;
            launch_gs_fc<T>(B0.d, P, zero, a, s);
        }
}

template <class T>
static void smooth_block(mbamg_hierarchy* h, int l, int f, bool zero, const T* b, const T* x, T* xn, const T* xg,
                         hipStream_t s) {
    Level& Lv = *h->L[l];
    BlockLevel& B = Lv.blk[f];
    const int g = 1 - f;
    const int64_t off = f == 0 ? 0 : (int64_t)Lv.n * Lv.d[0];
    T* tbuf = vecs<T>(Lv).t.p + off;
    const bool has_cpl = xg != nullptr;
    const bool timed = h->time_launches();
    if (B.rows) {
        for (int k = 0; k < h->p.inner_sweeps; ++k)
            for (int c = 0; c < B.n_colours; ++c) {
                const bool skip = zero && k == 0 && c == 0;
                double bytes = timed ? gs_bytes(B, c, zero, skip, has_cpl, (int)sizeof(T), Lv.d[g]) : 0.0;
                TimerScope ts(h, s, timed, launch_kind(l, (!zero && has_cpl) ? 0 : 3), bytes);
                GsRowArgs<T> a{};
                a.r_begin = B.colour_row[c];
                a.r_count = B.colour_row[c + 1] - B.colour_row[c];
                a.aff = rview<T>(B.raff);
                a.afg = rview<T>(B.rafg);
                a.dinv = rdinv<T>(B);
                a.b = b;
                a.x = x;
                a.t = tbuf;
                a.xn = xn;
                a.xg = xg;
                a.cstart = k == 0 ? B.colour_row[c] : INT_MAX;
                a.omega = (T)h->p.omega;
                a.w_row = Lv.damped ? wrow<T>(B) : nullptr;
                a.skip_off = (zero && k == 0 && c == 0) ? 1 : 0;
                launch_gs_rows<T>(B.d, B.row_split, zero, has_cpl, a, s);
            }
        return;
    }
    for (int k = 0; k < h->p.inner_sweeps; ++k) {
        for (int c = 0; c < B.n_colours; ++c) {
            GsArgs<T> a{};
            a.s_begin = B.colour_slice[c];
            a.s_count = B.colour_slice[c + 1] - B.colour_slice[c];
            a.sl = B.slices();
            a.off = B.off.view<T>();
            a.cpl = B.cpl.view<T>();
            a.dinv = B.dinv.view<T>();
            a.b = b;
            a.x = x;
            a.t = tbuf;
            a.xn = xn;
            a.xg = xg;
            a.cstart = k == 0 ? B.colour_row[c] : INT_MAX;
            a.omega = (T)h->p.omega;
            a.w_row = Lv.damped ? wrow<T>(B) : nullptr;
            a.skip_off = (zero && k == 0 && c == 0) ? 1 : 0;
            double bytes = timed ? gs_bytes(B, c, zero, a.skip_off, has_cpl, (int)sizeof(T), Lv.d[g]) : 0.0;
            // kind 0: passes from a nonzero iterate with the coupling term; kind 3: the others
            TimerScope ts(h, s, timed, launch_kind(l, (!zero && has_cpl) ? 0 : 3), bytes);
            launch_gs<T>(B.d, B.split, zero, has_cpl, a, s);
        }
    }
}

template <class T>
static void resid(mbamg_hierarchy* h, int l, const T* b, const T* x, T* r, hipStream_t s, int kind) {
    Level& Lv = *h->L[l];
    const int64_t n0 = (int64_t)Lv.n * Lv.d[0];
    ResidArgs<T> a{};
    for (int f = 0; f < 2; ++f) {
        BlockLevel& B = Lv.blk[f];
        const int64_t off = f == 0 ? 0 : n0;
        a.s_count[f] = B.n_slices;
        a.sl[f] = B.slices();
        a.off[f] = B.off.view<T>();
        a.cpl[f] = B.cpl.view<T>();
        a.diag[f] = B.diag.view<T>();
        a.b[f] = b ? b + off : nullptr;
        a.x[f] = x + off;
        a.r[f] = r + off;
        a.order[f] = Lv.resid_order[f].p;
    }
    const bool timed = h->time_launches() && kind >= 0 && (l == 0 || kind == 1);
    double bytes = timed ? resid_bytes(Lv, (int)sizeof(T), b != nullptr) : 0.0;
    TimerScope ts(h, s, timed, launch_kind(l, kind), bytes);
    if (Lv.blk[0].rows && Lv.blk[1].rows) {
        ResidRowArgs<T> ra{};
        for (int f = 0; f < 2; ++f) {
            ra.n[f] = Lv.nodes(f);
            ra.aff[f] = rview<T>(Lv.blk[f].raff);
            ra.afg[f] = rview<T>(Lv.blk[f].rafg);
            ra.b[f] = a.b[f];
            ra.x[f] = a.x[f];
            ra.r[f] = a.r[f];
        }
        launch_resid_rows<T>(Lv.d[0], ra, s);
        return;
    }
    launch_resid<T>(Lv.d[0], Lv.resid_split, a, s);
}

// One V-cycle on level l from a zero guess: out = MGV(0, b).
template <class T>
static void vcycle_level(mbamg_hierarchy* h, int l, const T* b, T* out, hipStream_t s) {
    Level& Lv = *h->L[l];
    double seg_down = 0.0, seg_up = 0.0;
    const bool tl = h->time_levels();
    if (tl) level_vcycle_bytes(h, l, seg_down, seg_up);
    if (Lv.coarsest) {
        TimerScope ts(h, s, tl, TK_LEVEL + 2 * l, seg_down);
        launch_coarse<T>(h->coarse_n, h->coarse_inv.p, b, out, s);
        return;
    }
    std::optional<TimerScope> seg;
    seg.emplace(h, s, tl, TK_LEVEL + 2 * l, seg_down);
    Vecs<T>& V = vecs<T>(Lv);
    const int64_t n0 = (int64_t)Lv.n * Lv.d[0];
    const int writes = 2 * h->p.bgs_sweeps;
    // ping-pong so that the last write lands in out
    T* buf[2];
    buf[0] = (writes % 2 == 0) ? V.xs.p : out;
    buf[1] = (writes % 2 == 0) ? out : V.xs.p;
    int cur = -1;
    auto sweep = [&](bool zero) {
        int nx = cur < 0 ? 0 : 1 - cur;
        T* X = cur < 0 ? nullptr : buf[cur];
        if (Lv.fc) {
            smooth_fc<T>(h, l, zero, b, X, buf[nx], s);
            cur = nx;
            return;
        }
        // block 0 (uses the current x1 for the coupling term)
        smooth_block<T>(h, l, 0, zero, b, X, buf[nx], zero ? nullptr : X + n0, s);
        // block 1 (Algorithm 1 relaxes it with the already updated x0)
        smooth_block<T>(h, l, 1, zero, b + n0, X ? X + n0 : nullptr, buf[nx] + n0, buf[nx], s);
        cur = nx;
    };
    for (int k = 0; k < h->p.bgs_sweeps; ++k) sweep(k == 0);
    resid<T>(h, l, b, buf[cur], V.r.p, s, 1);
    Level& Nx = *h->L[l + 1];
    Vecs<T>& C = vecs<T>(Nx);
    const int64_t nc0 = (int64_t)Nx.n * Nx.d[0];
    if (Lv.smoothed && Lv.blk[0].res_rows) {
        XferRowArgs<T> a{};
        for (int f = 0; f < 2; ++f) {
            a.n[f] = Nx.nodes(f);
            a.A[f] = rview<T>(Lv.blk[f].rres);
            a.x[f] = V.r.p + (f ? n0 : 0);
            a.y[f] = C.b.p + (f ? nc0 : 0);
            a.out_row[f] = Nx.blk[f].d_iperm.p;
        }
        a.accumulate = 0;
        const bool tx = h->time_launches();
        double xb = 0.0;
        if (tx)
            for (int f = 0; f < 2; ++f) xb += xfer_bytes(Lv.blk[f].res, Nx.n, Lv.n, Lv.d[f], (int)sizeof(T), false);
        TimerScope ts(h, s, tx, launch_kind(l, 5), xb);
        launch_xfer_rows<T>(Lv.d[0], a, s);
    } else if (Lv.smoothed) {
        XferArgs<T> a{};
        for (int f = 0; f < 2; ++f) {
            a.s_count[f] = Lv.blk[f].res_slices;
            a.sl[f] = {Lv.blk[f].res_row0.p, Lv.blk[f].res_nrow.p};
            a.A[f] = Lv.blk[f].res.view<T>();
            a.x[f] = V.r.p + (f ? n0 : 0);
            a.y[f] = C.b.p + (f ? nc0 : 0);
            a.out_row[f] = Nx.blk[f].d_iperm.p;
        }
        a.accumulate = 0;
        const bool tx = h->time_launches();
        double xb = 0.0;
        if (tx)
            for (int f = 0; f < 2; ++f) xb += xfer_bytes(Lv.blk[f].res, Nx.n, Lv.n, Lv.d[f], (int)sizeof(T), false);
        TimerScope ts(h, s, tx, launch_kind(l, 5), xb);
        launch_xfer<T>(Lv.d[0], Lv.blk[0].res_split, a, s);
    } else {
        TransferArgs<T> a{};
        for (int f = 0; f < 2; ++f) {
            a.n_rows[f] = Nx.nodes(f);
            a.map[f] = Lv.blk[f].mem_ptr.p;
            a.idx[f] = Lv.blk[f].mem_idx.p;
            a.q[f] = qmptr<T>(Lv.blk[f]);
            a.in[f] = V.r.p + (f ? n0 : 0);
            a.out[f] = C.b.p + (f ? nc0 : 0);
            a.order[f] = Nx.blk[f].d_iperm.p;   // coarse rows in natural (aggregate) order
        }
        const bool tx = h->time_launches();
        TimerScope ts(h, s, tx, launch_kind(l, 5), tx ? tentative_restrict_bytes(Lv, Nx, (int)sizeof(T)) : 0.0);
        launch_restrict<T>(Lv.d[0], a, Lv.blk[0].res_group, s);
    }
    seg.reset();
    vcycle_level<T>(h, l + 1, C.b.p, C.x.p, s);
    seg.emplace(h, s, tl, TK_LEVEL + 2 * l + 1, seg_up);
    if (Lv.smoothed) {
        XferArgs<T> a{};
        for (int f = 0; f < 2; ++f) {
            a.s_count[f] = Lv.blk[f].n_slices;
            a.sl[f] = Lv.blk[f].slices();
            a.A[f] = Lv.blk[f].pro.view<T>();
            a.x[f] = C.x.p + (f ? nc0 : 0);
            a.y[f] = buf[cur] + (f ? n0 : 0);
        }
        a.accumulate = 1;
        const bool tx = h->time_launches();
        double xb = 0.0;
        if (tx)
            for (int f = 0; f < 2; ++f) xb += xfer_bytes(Lv.blk[f].pro, Lv.n, Nx.n, Lv.d[f], (int)sizeof(T), true);
        TimerScope ts(h, s, tx, launch_kind(l, 6), xb);
        launch_xfer<T>(Lv.d[0], Lv.blk[0].pro_split, a, s);
    } else {
        TransferArgs<T> a{};
        for (int f = 0; f < 2; ++f) {
            a.n_rows[f] = Lv.nodes(f);
            a.map[f] = Lv.blk[f].agg_p.p;
            a.idx[f] = nullptr;
            a.q[f] = qptr<T>(Lv.blk[f]);
            a.in[f] = C.x.p + (f ? nc0 : 0);
            a.out[f] = buf[cur] + (f ? n0 : 0);
        }
        const bool tx = h->time_launches();
        TimerScope ts(h, s, tx, launch_kind(l, 6), tx ? tentative_prolong_bytes(Lv, Nx, (int)sizeof(T)) : 0.0);
        launch_prolong<T>(Lv.d[0], a, s);
    }
    for (int k = 0; k < h->p.bgs_sweeps; ++k) sweep(false);
    MB_CHECK(buf[cur] == out, MBAMG_E_STATE, "internal: V-cycle result not in the output buffer");
}


// ----------------------------------------------------------------------------
// more than two blocks: setup and V-cycle
// ----------------------------------------------------------------------------
static void zero_block(SetupBsr& Z, int n_rows, int n_cols, int br, int bc, hipStream_t s) {
    Z = SetupBsr();
    Z.n_rows = n_rows;
    Z.n_cols = n_cols;
    Z.br = br;
    Z.bc = bc;
    Z.nnzb = 0;
    Z.rp.alloc(n_rows + 1);
    MB_HIP(hipMemsetAsync(Z.rp.p, 0, sizeof(int32_t) * (n_rows + 1), s));
    Z.ci.alloc(1);
    Z.val.alloc(1);
}

// Hierarchy of an nb-block system (nb = 3 or 4): strength graph and aggregates
// of A_00 cloned to every block (Sec. 4.3.1), a piecewise-constant P_f per
// block, Galerkin products P_f^T A_fg P_g of every stored block pair (a zero
// block stays zero), the coarsest inverse, and per level every block's colour
// order, smoother parts and row forms.  FP64, fixed weights.
static void gen_setup_impl(mbamg_hierarchy* h, const mbamg_bsr* Ab, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const mbamg_params& p = h->p;
    const int nb = h->nb;
    const int N = Ab[0].n_brows;
    MB_CHECK(N > 0, MBAMG_E_INVALID, "empty system");
    const int* dofs = h->fm.dofs;
    {
        auto first = std::make_unique<GLevel>();
        first->set_blocks(N, nb, dofs);
        for (int f = 0; f < nb; ++f)
            for (int g = 0; g < nb; ++g) copy_block(Ab[f * nb + g], first->A[f][g], N, N, dofs[f], dofs[g], s);
        for (int f = 0; f < nb; ++f)
            MB_CHECK(first->A[f][f].nnzb > 0, MBAMG_E_INVALID, "diagonal blocks must be nonzero");
        h->GL.push_back(std::move(first));
    }
    DevBuf<double> Bn[MAXB];
    for (int f = 0; f < nb; ++f) {
        Bn[f].alloc((size_t)N * dofs[f]);
        fill_ones(Bn[f].p, (int64_t)N * dofs[f], s);
    }
    int lvl = 0;
    while (true) {
        GLevel& cur = *h->GL.back();
        if (cur.ndof() <= p.max_coarse || (int)h->GL.size() >= p.max_levels) break;
        Strength S = build_strength(cur.A[0][0], p.theta, s);
        cur.G = build_aggregates(S, p.seed, lvl, s);
        if ((double)cur.G.n_agg > 0.9 * cur.n) {   // this level is the coarsest
            cur.G = Aggregates();
            break;
        }
        const int nc = cur.G.n_agg;
        auto nxt = std::make_unique<GLevel>();
        nxt->set_blocks(nc, nb, dofs);
        SetupBsr P[MAXB], PT[MAXB];
        DevBuf<double> q[MAXB], Bc[MAXB];
        for (int f = 0; f < nb; ++f) {
            q[f].alloc((size_t)cur.n * dofs[f]);
            Bc[f].alloc((size_t)std::max(nc, 1) * dofs[f]);
            build_tentative(cur.G, dofs[f], Bn[f].p, q[f].p, Bc[f].p, s);
            P[f] = tentative_bsr(cur.G, dofs[f], q[f].p, s);
            PT[f] = block_transpose(P[f], s);
        }
        for (int f = 0; f < nb; ++f)
            for (int g = 0; g < nb; ++g) {
                if (cur.A[f][g].nnzb == 0) {
                    zero_block(nxt->A[f][g], nc, nc, dofs[f], dofs[g], s);
                    continue;
                }
                SetupBsr T = spgemm(cur.A[f][g], P[g], s);
                nxt->A[f][g] = spgemm(PT[f], T, s);
            }
        for (int f = 0; f < nb; ++f) {
            cur.blk[f].q64 = std::move(q[f]);
            Bn[f] = std::move(Bc[f]);
        }
        h->GL.push_back(std::move(nxt));
        ++lvl;
    }
    h->GL.back()->coarsest = true;
    {   // coarsest: dense inverse
        GLevel& c = *h->GL.back();
        h->coarse_n = (int)c.ndof();
        const SetupBsr* ab[MAXB * MAXB];
        for (int f = 0; f < nb; ++f)
            for (int g = 0; g < nb; ++g) ab[f * nb + g] = &c.A[f][g];
        CoarseWork w;
        coarse_inverse_launch_blocks(ab, nb, c.d, h->coarse_inv, w, s);
        coarse_inverse_finish(w, s);
    }
    // colour orders (first fit over each diagonal block's symmetrised pattern), smoother
    // parts and row forms
    for (auto& lp : h->GL) {
        GLevel& Lv = *lp;
        for (int f = 0; f < nb; ++f) {
            BlockLevel& B = Lv.blk[f];
            B.d = Lv.d[f];
            if (Lv.coarsest) {
                B.colour.assign(Lv.n, 0);
                order_and_slice(B, Lv.n, 1);
            } else {
                const std::vector<int32_t> rp = Lv.A[f][f].rp.download(s, (size_t)Lv.n + 1);
                const std::vector<int32_t> ci = Lv.A[f][f].ci.download(s, (size_t)Lv.A[f][f].nnzb);
                std::vector<int32_t> trp, tci;
                const bool asym = transpose_pattern(Lv.n, rp.data(), ci.data(), trp, tci);
                const int ncol = asym ? greedy_colour(Lv.n, rp.data(), ci.data(), B.colour, trp.data(), tci.data())
                                      : greedy_colour(Lv.n, rp.data(), ci.data(), B.colour);
                order_and_slice(B, Lv.n, ncol, rp.data());
            }
            B.row0.upload(B.h_row0, s);
            B.nrow.upload(B.h_nrow, s);
            B.d_perm.upload(B.perm, s);
            B.d_iperm.upload(B.iperm, s);
        }
        for (int f = 0; f < nb; ++f)
            for (int g = 0; g < nb; ++g)
                build_rows(Lv.R[f][g], Lv.n, Lv.blk[f].d_perm.p, Lv.A[f][g], Lv.blk[g].d_iperm.p, false, s);
        if (!Lv.coarsest) {
            for (int f = 0; f < nb; ++f) {
                BlockLevel& B = Lv.blk[f];
                const int df = Lv.d[f];
                DevBuf<double> dinv((size_t)Lv.n * df * df);
                build_dinv(Lv.A[f][f], dinv.p, s);
                build_part(B.off, PartKind::Off, B, &Lv.A[f][f], B.d_iperm.p, Lv.A[f][f].val.p, df, df, false, s);
                build_part(B.dinv, PartKind::Dinv, B, nullptr, nullptr, dinv.p, df, df, false, s);
                int64_t slots = 0;
                for (int sl = 0; sl < B.n_slices; ++sl) slots += B.off.h_width[sl];
                const double avg_width = B.n_slices ? (double)slots / B.n_slices : 0.0;
                B.split = slot_split((double)B.n_slices / std::max(1, B.n_colours), avg_width);
            }
        }
        const int64_t nd = std::max<int64_t>(Lv.ndof(), 1);
        Lv.b.alloc(nd);
        Lv.x.alloc(nd);
        Lv.xs.alloc(nd);
        Lv.t.alloc(nd);
        Lv.r.alloc(nd);
        Lv.rhs.alloc(nd);
        MB_HIP(hipStreamSynchronize(s));
    }
    // transfers between each level's and the next level's colour orders
    for (size_t l = 0; l + 1 < h->GL.size(); ++l) {
        GLevel& Lv = *h->GL[l];
        GLevel& Nx = *h->GL[l + 1];
        for (int f = 0; f < nb; ++f) {
            BlockLevel& B = Lv.blk[f];
            const BlockLevel& C = Nx.blk[f];
            transfer_maps(Lv.n, Nx.n, B.d_perm.p, B.d_iperm.p, Lv.G.agg.p, C.d_perm.p, C.d_iperm.p, Lv.G.mptr.p,
                          Lv.G.midx.p, B.agg_p, B.mem_ptr, B.mem_idx, s);
            B.res_group = restrict_group(Lv.n, Nx.n);
            DevBuf<double> qp((size_t)Lv.n * B.d);
            launch_gather(Lv.n, B.d, B.d_perm.p, B.q64.p, qp.p, s);
            B.q64 = std::move(qp);
            B.qm64.alloc((size_t)Lv.n * B.d);
            launch_gather(Lv.n, B.d, B.mem_idx.p, B.q64.p, B.qm64.p, s);
        }
        MB_HIP(hipStreamSynchronize(s));
    }
    // Krylov workspace
    h->n_fine = h->GL[0]->ndof();
    const int m = p.restart;
    const int64_t n = h->n_fine;
    h->V.alloc((size_t)(m + 1) * n);
    h->Z64.alloc((size_t)m * n);
    h->w.alloc(n);
    h->xw.alloc(n);
    h->bw.alloc(n);
    h->vio.alloc(n);
    h->vio2.alloc(n);
    h->partial.alloc((size_t)KBLOCKS * KMAXQ);
    h->hbuf.alloc(KB_TOTAL);
    h->ybuf.alloc(KMAXQ);
    h->coef.alloc(KC_TOTAL);
    MB_HIP(hipHostMalloc((void**)&h->hbuf_host, sizeof(double) * KB_TOTAL, hipHostMallocDefault));
    MB_HIP(hipHostMalloc((void**)&h->coef_host, sizeof(double) * KC_TOTAL, hipHostMallocDefault));
    MB_HIP(hipHostMalloc((void**)&h->y_host, sizeof(double) * KMAXQ, hipHostMallocDefault));
    MB_HIP(hipStreamSynchronize(s));
    h->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int64_t nz0 = h->GL[0]->nnzb_total(), nzs = 0;
    for (auto& lv : h->GL) nzs += lv->nnzb_total();
    h->info.levels = (int)h->GL.size();
    h->info.op_complexity = nz0 ? (double)nzs / (double)nz0 : 1.0;
    h->info.t_setup_ms = h->t_setup_ms;
}

static RowView<double> grview(const RowPart& R) { return {R.rp.p, R.col.p, R.v64.p}; }

// y_f = b_f - sum over blocks g of A_fg x_g (b NULL: y = sum A_fg x_g); xs[g] NULL skips block g
static void gen_block_rows(const GLevel& Lv, int f, const double* b, const double* const* xs, double* y, bool skip_f,
                           hipStream_t s) {
    const int64_t len = (int64_t)Lv.n * Lv.d[f];
    if (b) MB_HIP(hipMemcpyAsync(y, b, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
    else fill_value(y, len, 0.0, s);
    for (int g = 0; g < Lv.nb; ++g) {
        if ((skip_f && g == f) || !xs[g] || Lv.R[f][g].nnzb == 0) continue;
        launch_rows_acc<double>(Lv.n, Lv.d[f], Lv.d[g], grview(Lv.R[f][g]), xs[g], y, b ? -1.0 : 1.0, s);
    }
}

// w = A x (b NULL) or r = b - A x on level l (colour order, all blocks)
static void gen_resid(mbamg_hierarchy* h, int l, const double* b, const double* x, double* r, hipStream_t s) {
    GLevel& Lv = *h->GL[l];
    const double* xs[MAXB];
    for (int g = 0; g < Lv.nb; ++g) xs[g] = x + Lv.off[g];
    for (int f = 0; f < Lv.nb; ++f) gen_block_rows(Lv, f, b ? b + Lv.off[f] : nullptr, xs, r + Lv.off[f], false, s);
}

// One V-cycle on level l from a zero guess (the MGV figure of Sec. 3) with
// Algorithm 1 over the level's blocks as pre- and post-smoother.
static void gen_vcycle_level(mbamg_hierarchy* h, int l, const double* b, double* out, hipStream_t s) {
    GLevel& Lv = *h->GL[l];
    if (Lv.coarsest) {
        launch_coarse<double>(h->coarse_n, h->coarse_inv.p, b, out, s);
        return;
    }
    const int nb = Lv.nb;
    const int writes = 2 * h->p.bgs_sweeps;
    double* buf[2];
    buf[0] = (writes % 2 == 0) ? Lv.xs.p : out;
    buf[1] = (writes % 2 == 0) ? out : Lv.xs.p;
    int cur = -1;
    auto sweep = [&](bool zero) {
        const int nx = cur < 0 ? 0 : 1 - cur;
        const double* X = cur < 0 ? nullptr : buf[cur];
        double* XN = buf[nx];
        for (int f = 0; f < nb; ++f) {
            // the couplings of block f with the blocks before it (already relaxed in this sweep)
            // and after it (the incoming iterate) go into its right-hand side
            const double* xs[MAXB];
            for (int g = 0; g < nb; ++g) xs[g] = g < f ? XN + Lv.off[g] : (X ? X + Lv.off[g] : nullptr);
            double* rhs = Lv.rhs.p + Lv.off[f];
            gen_block_rows(Lv, f, b + Lv.off[f], xs, rhs, true, s);
            BlockLevel& B = Lv.blk[f];
            for (int k = 0; k < h->p.inner_sweeps; ++k)
                for (int c = 0; c < B.n_colours; ++c) {
                    GsArgs<double> a{};
                    a.s_begin = B.colour_slice[c];
                    a.s_count = B.colour_slice[c + 1] - B.colour_slice[c];
                    a.sl = B.slices();
                    a.off = B.off.view<double>();
                    a.dinv = B.dinv.view<double>();
                    a.b = rhs;
                    a.x = X ? X + Lv.off[f] : nullptr;
                    a.t = Lv.t.p + Lv.off[f];
                    a.xn = XN + Lv.off[f];
                    a.xg = nullptr;
                    a.cstart = k == 0 ? B.colour_row[c] : INT_MAX;
                    a.omega = h->p.omega;
                    a.w_row = nullptr;
                    a.skip_off = (zero && k == 0 && c == 0) ? 1 : 0;
                    launch_gs<double>(B.d, B.split, zero, false, a, s);
                }
        }
        cur = nx;
    };
    for (int k = 0; k < h->p.bgs_sweeps; ++k) sweep(k == 0);
    gen_resid(h, l, b, buf[cur], Lv.r.p, s);
    GLevel& Nx = *h->GL[l + 1];
    for (int f = 0; f < nb; ++f) {   // restriction, one block at a time (its own block size)
        TransferArgs<double> a{};
        a.n_rows[0] = Nx.n;
        a.map[0] = Lv.blk[f].mem_ptr.p;
        a.idx[0] = Lv.blk[f].mem_idx.p;
        a.q[0] = Lv.blk[f].qm64.p;
        a.in[0] = Lv.r.p + Lv.off[f];
        a.out[0] = Nx.b.p + Nx.off[f];
        launch_restrict<double>(Lv.d[f], a, Lv.blk[f].res_group, s);
    }
    gen_vcycle_level(h, l + 1, Nx.b.p, Nx.x.p, s);
    for (int f = 0; f < nb; ++f) {   // prolongation
        TransferArgs<double> a{};
        a.n_rows[0] = Lv.n;
        a.map[0] = Lv.blk[f].agg_p.p;
        a.q[0] = Lv.blk[f].q64.p;
        a.in[0] = Nx.x.p + Nx.off[f];
        a.out[0] = buf[cur] + Lv.off[f];
        launch_prolong<double>(Lv.d[f], a, s);
    }
    for (int k = 0; k < h->p.bgs_sweeps; ++k) sweep(false);
    MB_CHECK(buf[cur] == out, MBAMG_E_STATE, "internal: V-cycle result not in the output buffer");
}

// z = M^-1 v for FP64 colour-order vectors of the finest level (either form).
static void apply_precond(mbamg_hierarchy* h, const double* v, double* z64, float* z32, hipStream_t s) {
    if (h->nb > 2) {
        TimerScope ts(h, s, h->time_vcycles(), TK_VCYCLE, 0.0);
        gen_vcycle_level(h, 0, v, z64, s);
        return;
    }
    if (h->p.precision == 1) {
        Level& L0 = *h->L[0];
        launch_cast64to32(h->n_fine, v, h->vin32.p, s);
        {
            TimerScope ts(h, s, h->time_vcycles(), TK_VCYCLE, 0.0);
            if (L0.coarsest) {
                launch_coarse<float>(h->coarse_n, h->coarse_inv.p, h->vin32.p, z32, s);
            } else {
                vcycle_level<float>(h, 0, h->vin32.p, z32, s);
            }
        }
        if (z64) launch_cast32to64(h->n_fine, z32, z64, s);
    } else {
        TimerScope ts(h, s, h->time_vcycles(), TK_VCYCLE, 0.0);
        vcycle_level<double>(h, 0, v, z64, s);
    }
}

static void to_colour(mbamg_hierarchy* h, const double* src, double* dst, hipStream_t s) {
    if (h->nb > 2) {
        const GLevel& L0 = *h->GL[0];
        for (int f = 0; f < L0.nb; ++f)
            launch_gather(L0.n, L0.d[f], L0.blk[f].d_perm.p, src + L0.off[f], dst + L0.off[f], s);
        return;
    }
    Level& L0 = *h->L[0];
    MB_CHECK(L0.blk[0].d_perm.p && L0.blk[1].d_perm.p, MBAMG_E_STATE, "internal: finest-level order missing");
    const int64_t n0 = (int64_t)L0.n * L0.d[0];
    for (int f = 0; f < 2; ++f)
        launch_gather(L0.nodes(f), L0.d[f], L0.blk[f].d_perm.p, src + (f ? n0 : 0), dst + (f ? n0 : 0), s);
}

static void from_colour(mbamg_hierarchy* h, const double* src, double* dst, hipStream_t s) {
    if (h->nb > 2) {
        const GLevel& L0 = *h->GL[0];
        for (int f = 0; f < L0.nb; ++f)
            launch_scatter(L0.n, L0.d[f], L0.blk[f].d_perm.p, src + L0.off[f], dst + L0.off[f], s);
        return;
    }
    Level& L0 = *h->L[0];
    MB_CHECK(L0.blk[0].d_perm.p && L0.blk[1].d_perm.p, MBAMG_E_STATE, "internal: finest-level order missing");
    const int64_t n0 = (int64_t)L0.n * L0.d[0];
    for (int f = 0; f < 2; ++f)
        launch_scatter(L0.nodes(f), L0.d[f], L0.blk[f].d_perm.p, src + (f ? n0 : 0), dst + (f ? n0 : 0), s);
}

// A x on the finest level (colour order), FP64
static void apply_A(mbamg_hierarchy* h, const double* x, double* w, hipStream_t s, int kind = 2) {
    if (h->nb > 2) {
        gen_resid(h, 0, nullptr, x, w, s);
        return;
    }
    Level& L0 = *h->L[0];
    if (L0.coarsest && !L0.apply_parts) throw Error(MBAMG_E_STATE, "internal: finest-level operator missing");
    resid<double>(h, 0, nullptr, x, w, s, kind);
}

// ----------------------------------------------------------------------------
// GMRES (right preconditioned) / FGMRES, restarted
// ----------------------------------------------------------------------------
// ||v||^2 through the deterministic two-pass reduction (synchronous)
static double norm2_dev(mbamg_hierarchy* h, const double* v, hipStream_t s) {
    const int nb = krylov_blocks(h->n_fine);
    double* kb = h->hbuf.p;
    launch_orth(h->n_fine, 0, nullptr, 0, v, h->partial.p, nb, s);
    launch_orth_reduce(h->partial.p, nb, 0, nullptr, kb + KB_NU0, nullptr, s);
    double r = 0.0;
    MB_HIP(hipMemcpyAsync(&r, kb + KB_NU0, sizeof(double), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    return r;
}

// Restarted GMRES (FGMRES when the cycle runs in FP32), right preconditioned.
// Orthogonalisation is classical Gram-Schmidt run twice ("twice is enough",
// Giraud, Langou & Rozloznik 2005) with the second pass delayed by one step
// (DCGS2, Swirydowicz et al. 2020; Bielich et al. 2022), so each step reads the
// basis twice (a dot pass, an update pass) rather than three times:
//   step j holds Q_0..Q_{j-1} (orthonormal) and the candidate u_j, projected
//   once, with a_j = Q^T u_j and |u_j|^2 from the previous update pass, so
//   nu_j = sqrt(|u_j|^2 - |a_j|^2) = |u_j - Q a_j|.  The preconditioner and the
//   operator are applied to u_j itself: zt_j = M u_j, w = A zt_j.  The direction
//   the Arnoldi process wants is z_j = (zt_j - sum_i a_{j,i} z_i) / nu_j, whose
//   image A z_j = (w - Q_{j+1} c) / nu_j with c = H_{0..j,0..j-1} a_j (the
//   Arnoldi relation of the earlier columns), so
//     H[l][j] = (b_l - c_l) / nu_j + a_{j+1,l}        (l < j, b = Q^T w)
//     H[j][j] = ((u_j.w - a_j.b) / nu_j - c_j) / nu_j + a_{j+1,j}
//     H[j+1][j] = nu_{j+1}
//   where the update pass writes Q_j = (u_j - Q a_j) / nu_j and the next
//   candidate u_{j+1} = (w - Q b - Q_j (u_j.w - a_j.b) / nu_j) / nu_j and sums
//   a_{j+1} and |u_{j+1}|^2.  The iterate gains Z y = Zt t with
//   zt_j = sum_i a_{j,i} z_i + nu_j z_j, i.e. U t = y for the upper-triangular U
//   of the a's and nu's.
// Solve-time fallback of a judged learned hierarchy (the setup's probe judge
// decides which preconditioner a solve starts with): when a complete restart
// cycle of the learned preconditioner reduces the residual by less than
// REVERT_STALL per iteration on average -- the solve stalls -- the solve goes
// on from the current iterate with the fixed-weight hierarchy.  The probe
// factors themselves are no threshold here: they measure the stationary
// iteration over 10 steps, which GMRES's reduction rate does not follow (a
// learned preconditioner can reduce more slowly than the fixed method's probe
// factor in its first iterations while the fixed method reduces more slowly
// still, and probe factors above 1 occur where GMRES converges).
// (MBAMG_REVERT_RHO overrides the threshold, for tests.)
constexpr double REVERT_STALL = 0.99;

static double revert_threshold() {
    if (const char* f = form_override("MBAMG_REVERT_RHO")) return std::atof(f);
    return REVERT_STALL;
}

static mbamg_status solve_impl(mbamg_hierarchy* h, const double* b, double* x, double rtol, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const bool can_revert = h->fallback != nullptr;
    const double revert_rho = can_revert ? revert_threshold() : 0.0;
    bool revert = false;
    h->info.reverted = 0;
    if (can_revert) h->info.used_learned = 1;
    const int64_t n = h->n_fine;
    const int m = h->p.restart;
    const bool fp32 = h->p.precision == 1;
    to_colour(h, b, h->bw.p, s);
    to_colour(h, x, h->xw.p, s);
    const double bnorm = std::sqrt(norm2_dev(h, h->bw.p, s));
    int its = 0;
    double rel = 0.0;
    mbamg_status st = MBAMG_OK;
    // H: the least-squares matrix (rotated as it grows), Hr: its unrotated columns
    // (the Arnoldi relation), Ac[j][i] = a_{j,i}, nuv[j] = nu_j
    const int ld = m + 1;
    std::vector<double> H((size_t)ld * m), Hr((size_t)ld * m), cs(m), sn(m), g(ld), y(m), t(m), nuv(ld),
        Ac((size_t)ld * ld);
    double* hb = h->hbuf_host;
    double* kb = h->hbuf.p;
    double* ch = h->coef_host;
    const int nb = krylov_blocks(n);
    if (bnorm == 0.0) {
        MB_HIP(hipMemsetAsync(h->xw.p, 0, sizeof(double) * n, s));
        rel = 0.0;
    } else {
        while (true) {
            // true residual into V_0: the first candidate, with a_0 = () and nu_0 = beta
            if (h->nb > 2) gen_resid(h, 0, h->bw.p, h->xw.p, h->V.p, s);
            else resid<double>(h, 0, h->bw.p, h->xw.p, h->V.p, s, 1);
            const double beta = std::sqrt(norm2_dev(h, h->V.p, s));
            rel = beta / bnorm;
            if (beta <= rtol * bnorm) break;
            if (its >= h->p.max_iters) { st = MBAMG_NOT_CONVERGED; break; }
            nuv[0] = beta;
            ch[KC_INV_NU] = 1.0 / beta;
            MB_HIP(hipMemcpyAsync(h->coef.p + KC_INV_NU, ch + KC_INV_NU, sizeof(double), hipMemcpyHostToDevice, s));
            std::fill(g.begin(), g.end(), 0.0);
            std::fill(Hr.begin(), Hr.end(), 0.0);
            g[0] = beta;
            int k = 0;
            for (int j = 0; j < m; ++j) {
                double* vj = h->V.p + (size_t)j * n;
                double* vn = h->V.p + (size_t)(j + 1) * n;
                double* zj64 = fp32 ? h->ztmp.p : h->Z64.p + (size_t)j * n;
                float* zj32 = fp32 ? h->Z32.p + (size_t)j * n : nullptr;
                apply_precond(h, vj, zj64, zj32, s);
                apply_A(h, zj64, h->w.p, s);
                // dot pass: b = Q^T w and u_j . w; c_j on the device
                launch_orth(n, j + 1, h->V.p, n, h->w.p, h->partial.p, nb, s);
                launch_orth_reduce(h->partial.p, nb, j + 1, kb + KB_D1, nullptr, h->coef.p, s);
                // update pass: Q_j over u_j, u_{j+1} into V_{j+1}, a_{j+1} and |u_{j+1}|^2
                launch_dcgs_update(n, j, h->V.p, n, h->coef.p, vj, h->w.p, vn, h->partial.p, nb, s);
                launch_orth_reduce(h->partial.p, nb, j + 1, kb + KB_D2, kb + KB_NU1, nullptr, s);
                MB_HIP(hipMemcpyAsync(hb, kb, sizeof(double) * KB_TOTAL, hipMemcpyDeviceToHost, s));
                MB_HIP(hipStreamSynchronize(s));
                const double* bq = hb + KB_D1;
                const double* an = hb + KB_D2;
                const double* aj = &Ac[(size_t)j * ld];
                const double nuj = nuv[j];
                double ab = 0.0;
                for (int i = 0; i < j; ++i) ab += aj[i] * bq[i];
                double* raw = &Hr[(size_t)j * ld];
                for (int l = 0; l <= j; ++l) {
                    double c = 0.0;
                    for (int i = std::max(0, l - 1); i < j; ++i) c += Hr[(size_t)i * ld + l] * aj[i];
                    const double proj = l < j ? bq[l] : (bq[j] - ab) / nuj;
                    raw[l] = (proj - c) / nuj + an[l];
                }
                double nu2 = hb[KB_NU1];
                for (int l = 0; l <= j; ++l) nu2 -= an[l] * an[l];
                // nu2 <= 0: the candidate lies in the basis (breakdown)
                const double nun = nu2 > 0.0 && std::isfinite(nu2) ? std::sqrt(nu2) : 0.0;
                raw[j + 1] = nun;
                nuv[j + 1] = nun;
                for (int l = 0; l <= j; ++l) Ac[(size_t)(j + 1) * ld + l] = an[l];
                if (nun > 0.0 && j + 1 < m) {
                    for (int l = 0; l <= j; ++l) ch[KC_A + l] = an[l];
                    ch[KC_INV_NU] = 1.0 / nun;
                    MB_HIP(hipMemcpyAsync(h->coef.p, ch, sizeof(double) * KC_TOTAL, hipMemcpyHostToDevice, s));
                }
                double* col = &H[(size_t)j * ld];
                for (int l = 0; l <= j + 1; ++l) col[l] = raw[l];
                for (int i = 0; i < j; ++i) {
                    double tq = cs[i] * col[i] + sn[i] * col[i + 1];
                    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                    col[i] = tq;
                }
                double den = std::hypot(col[j], col[j + 1]);
                cs[j] = den != 0.0 ? col[j] / den : 1.0;
                sn[j] = den != 0.0 ? col[j + 1] / den : 0.0;
                col[j] = den;
                col[j + 1] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++its;
                k = j + 1;
                if (std::fabs(g[j + 1]) <= rtol * bnorm || its >= h->p.max_iters || nun == 0.0) break;
                if (can_revert && k == m && !(std::pow(std::fabs(g[j + 1]) / beta, 1.0 / k) <= revert_rho)) {
                    revert = true;
                    break;
                }
            }
            // back substitution H[:k,:k] y = g[:k], then U t = y; x += sum_j t_j zt_j
            for (int i = k - 1; i >= 0; --i) {
                double sum = g[i];
                for (int c = i + 1; c < k; ++c) sum -= H[(size_t)c * ld + i] * y[c];
                y[i] = sum / H[(size_t)i * ld + i];
            }
            for (int i = k - 1; i >= 0; --i) {
                double sum = y[i];
                for (int l = i + 1; l < k; ++l) sum -= Ac[(size_t)l * ld + i] * t[l];
                t[i] = sum / nuv[i];
            }
            for (int i = 0; i < k; ++i) h->y_host[i] = t[i];
            MB_HIP(hipMemcpyAsync(h->ybuf.p, h->y_host, sizeof(double) * k, hipMemcpyHostToDevice, s));
            if (fp32) launch_combine32(n, k, h->Z32.p, n, h->ybuf.p, h->xw.p, s);
            else launch_combine(n, k, h->Z64.p, n, h->ybuf.p, h->xw.p, s);
            if (revert) break;
        }
    }
    from_colour(h, h->xw.p, x, s);
    MB_HIP(hipStreamSynchronize(s));
    if (revert) {
        // the rest of the solve with the fixed-weight hierarchy, from the current iterate
        mbamg_hierarchy* fb = h->fallback.get();
        const int keep_max = fb->p.max_iters;
        fb->p.max_iters = std::max(0, h->p.max_iters - its);
        try {
            st = solve_impl(fb, b, x, rtol, s);
        } catch (...) {
            fb->p.max_iters = keep_max;
            throw;
        }
        fb->p.max_iters = keep_max;
        h->info.iterations = its + fb->info.iterations;
        h->info.rel_residual = fb->info.rel_residual;
        h->info.conv_factor = h->info.iterations > 0 && fb->info.rel_residual > 0
                                  ? std::pow(fb->info.rel_residual, 1.0 / h->info.iterations) : 0.0;
        h->info.reverted = 1;
        h->info.used_learned = 0;
        h->info.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        h->info.t_setup_ms = h->t_setup_ms;
        return st;
    }
    auto t1 = std::chrono::steady_clock::now();
    h->info.iterations = its;
    h->info.rel_residual = rel;
    h->info.conv_factor = its > 0 && rel > 0 ? std::pow(rel, 1.0 / its) : 0.0;
    h->info.t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    h->info.t_setup_ms = h->t_setup_ms;
    return st;
}

// Asymptotic factor of e <- e - M A e from a seeded start (colour order).
static double probe_impl(mbamg_hierarchy* h, int iters, uint64_t seed, hipStream_t s) {
    MB_CHECK(iters >= 5, MBAMG_E_INVALID, "probe needs at least 5 iterations");
    const int64_t n = h->n_fine;
    double* e = h->vio.p;
    launch_seeded(n, seed, h->vio2.p, s);   // generated in the interface order, then reordered
    to_colour(h, h->vio2.p, e, s);
    double nk4 = 0.0, nk = 0.0;
    for (int k = 1; k <= iters; ++k) {
        apply_A(h, e, h->w.p, s, -1);
        apply_precond(h, h->w.p, h->vio2.p, h->p.precision == 1 ? h->Z32.p : nullptr, s);
        launch_axpby(n, -1.0, h->vio2.p, 1.0, e, s);
        if (k == iters - 4) nk4 = norm2_dev(h, e, s);
        if (k == iters) nk = norm2_dev(h, e, s);
    }
    if (nk4 <= 0.0) return 0.0;
    return std::pow(std::sqrt(nk / nk4), 0.25);
}

}  // namespace mbamg

// ----------------------------------------------------------------------------
// C-ABI
// ----------------------------------------------------------------------------
template <class F>
static mbamg_status guarded(F&& fn) {
    try {
        return fn();
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return MBAMG_E_NOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return MBAMG_E_INVALID;
    } catch (...) {
        g_last_error = "unknown error";
        return MBAMG_E_INVALID;
    }
}

extern "C" {

void mbamg_default_params(mbamg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->omega = 0.8;
    p->bgs_sweeps = 1;
    p->inner_sweeps = 1;
    p->theta = 0.0;
    p->max_levels = 10;
    p->max_coarse = 2500;
    p->clone_aggregates = 1;
    p->reuse_P = 1;
    p->precision = 0;
    p->restart = 30;
    p->max_iters = 1000;
    p->learned = 0;
    p->mlp = nullptr;
    p->seed = 0;
    p->omega_p = 0.0;
    p->judge = 1;
    p->weight_fn = nullptr;
    p->weight_ctx = nullptr;
}

const char* mbamg_last_error(void) { return g_last_error.c_str(); }

mbamg_status mbamg_setup(const mbamg_bsr* A_blocks, const mbamg_field_map* fm, const mbamg_params* p,
                         void* hip_stream, mbamg_hierarchy** out) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(A_blocks && fm && p && out, MBAMG_E_INVALID, "NULL argument");
        *out = nullptr;
        MB_CHECK(fm->n_blocks >= 2 && fm->n_blocks <= MAXB, MBAMG_E_INVALID, "2 to 4 blocks");
        if (fm->n_blocks > 2) {
            for (int f = 0; f < fm->n_blocks; ++f)
                MB_CHECK(fm->dofs[f] >= 1 && fm->dofs[f] <= 4, MBAMG_E_INVALID, "1..4 dofs per node and block");
            MB_CHECK(p->clone_aggregates != 0 && p->learned == 0 && p->omega_p == 0.0 && p->smoother == 0 &&
                         p->precision == 0,
                     MBAMG_E_INVALID,
                     "more than two blocks: co-located fields, FP64, fixed weights and the blocked smoother");
        } else {
            MB_CHECK(fm->dofs[0] >= 1 && fm->dofs[0] <= 4 && fm->dofs[1] == fm->dofs[0], MBAMG_E_INVALID,
                     "both blocks must have the same 1..4 dofs per node");
        }
        MB_CHECK(p->omega > 0.0 && std::isfinite(p->omega) && p->bgs_sweeps >= 1 && p->inner_sweeps >= 1 && p->max_levels >= 1 &&
                     p->restart >= 1 && p->restart <= KMAXQ - 2 && p->max_iters >= 0 && p->theta >= 0.0,
                 MBAMG_E_INVALID, "invalid parameters");
        MB_CHECK(p->clone_aggregates != 0 || (p->learned == 0 && p->omega_p == 0.0 && p->smoother == 0),
                 MBAMG_E_INVALID,
                 "separate block-1 aggregation is built for the fixed form with the blocked smoother");
        MB_CHECK(p->precision == 0 || p->precision == 1, MBAMG_E_INVALID, "precision must be 0 or 1");
        MB_CHECK(p->learned >= 0 && p->learned <= 2, MBAMG_E_INVALID, "learned must be 0, 1 or 2");
        MB_CHECK(p->learned != 1 || p->mlp != nullptr, MBAMG_E_INVALID, "learned == 1 needs the network parameters");
        MB_CHECK(p->learned != 2 || p->weight_fn != nullptr, MBAMG_E_INVALID, "learned == 2 needs a weight callback");
        MB_CHECK(p->omega_p >= 0.0 && std::isfinite(p->omega_p), MBAMG_E_INVALID, "omega_p must be >= 0");
        MB_CHECK(p->smoother == 0 || p->smoother == 1, MBAMG_E_INVALID, "smoother must be 0 or 1");
        for (int f = 0; f < 2; ++f)
            MB_CHECK(fm->n_vec[f] >= 0 && fm->n_vec[f] <= fm->dofs[f], MBAMG_E_INVALID, "n_vec out of range");
        hipStream_t s = (hipStream_t)hip_stream;
        auto t0 = std::chrono::steady_clock::now();
        auto make = [&](const mbamg_params& pp, hipStream_t st) {
            auto h = std::make_unique<mbamg_hierarchy>();
            h->p = pp;
            h->fm = *fm;
            h->d[0] = fm->dofs[0];
            h->d[1] = fm->dofs[1];
            if (pp.learned == 1) h->mlp.upload(pp.mlp, N_MLP_PARAMS + 2 * N_FEATURES, st);
            return h;
        };
        auto settle = [] {   // the build's temporaries are idle now and can serve the next allocations
            MB_HIP(hipDeviceSynchronize());
            pool_device_idle();
        };
        std::unique_ptr<mbamg_hierarchy> h;
        if (fm->n_blocks > 2) {
            h = make(*p, s);
            h->nb = fm->n_blocks;
            gen_setup_impl(h.get(), A_blocks, s);
            settle();
            h->info.used_learned = 0;
        } else if (p->learned != 0 && p->judge) {
            // the fixed-weight method is the fallback and the judge.  It is built, and then
            // probed, on a host thread and stream of its own while the learned hierarchy is
            // built here; the learned build copies the fixed build's level-0 aggregates and
            // smoother data as soon as they are published (the hierarchies share no buffers)
            mbamg_params pf = *p;
            pf.learned = 0;
            pf.omega_p = 0.0;
            PhaseClock jclk(s);
            int device = 0;
            MB_HIP(hipGetDevice(&device));
            SideStream sf;
            MB_HIP(hipEventRecord(sf.ready, s));   // the caller's inputs are ready on s
            MB_HIP(hipStreamWaitEvent(sf.stream, sf.ready, 0));
            auto hf = make(pf, sf.stream);
            DonorLink link;
            // declared after hf, sf and link: on an exception here the job is waited for first
            auto fixed_job = std::async(std::launch::async, [&hf, &link, &sf, A_blocks, device] {
                MB_HIP(hipSetDevice(device));
                try {
                    setup_impl(hf.get(), A_blocks, sf.stream, nullptr, &link, true);
                } catch (...) {
                    link.close();
                    throw;
                }
                finish_coarse(hf.get(), sf.stream);
                return probe_impl(hf.get(), 10, 12345, sf.stream);
            });
            h = make(*p, s);
            setup_impl(h.get(), A_blocks, s, &link, nullptr, false);
            settle();
            jclk.mark("learned hierarchy built", 0);
            const double rl = probe_impl(h.get(), 10, 12345, s);
            const double rf = fixed_job.get();
            jclk.mark("judge probes", 0);
            h->judge_rho[0] = hf->judge_rho[0] = rl;
            h->judge_rho[1] = hf->judge_rho[1] = rf;
            if (!(rl < rf)) {
                h = std::move(hf);
                h->info.used_learned = 0;
            } else {
                h->info.used_learned = 1;
                h->fallback = std::move(hf);
            }
        } else {
            h = make(*p, s);
            setup_impl(h.get(), A_blocks, s, nullptr, nullptr, false);
            settle();
            h->info.used_learned = p->learned != 0;
        }
        MB_HIP(hipDeviceSynchronize());
        pool_device_idle();
        auto t1 = std::chrono::steady_clock::now();
        h->t_setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        h->info.t_setup_ms = h->t_setup_ms;
        *out = h.release();
        return MBAMG_OK;
    });
}

mbamg_status mbamg_vcycle(mbamg_hierarchy* h, const double* r, double* z, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && r && z, MBAMG_E_INVALID, "NULL argument");
        MB_CHECK(r != z, MBAMG_E_INVALID, "r and z must not alias");
        hipStream_t s = (hipStream_t)hip_stream;
        to_colour(h, r, h->vio.p, s);
        if (h->nb > 2) {
            gen_vcycle_level(h, 0, h->vio.p, h->vio2.p, s);
        } else if (h->p.precision == 1) {
            apply_precond(h, h->vio.p, h->vio2.p, h->vin32.p == nullptr ? nullptr : h->Z32.p, s);
        } else {
            if (h->L[0]->coarsest) launch_coarse<double>(h->coarse_n, h->coarse_inv.p, h->vio.p, h->vio2.p, s);
            else vcycle_level<double>(h, 0, h->vio.p, h->vio2.p, s);
        }
        from_colour(h, h->vio2.p, z, s);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_apply(mbamg_hierarchy* h, const double* x, double* w, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && x && w, MBAMG_E_INVALID, "NULL argument");
        MB_CHECK(x != w, MBAMG_E_INVALID, "x and w must not alias");
        hipStream_t s = (hipStream_t)hip_stream;
        to_colour(h, x, h->vio.p, s);
        apply_A(h, h->vio.p, h->vio2.p, s);
        from_colour(h, h->vio2.p, w, s);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_solve(mbamg_hierarchy* h, const double* b, double* x, double rtol, mbamg_info* info,
                         void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && b && x, MBAMG_E_INVALID, "NULL argument");
        MB_CHECK(b != x, MBAMG_E_INVALID, "b and x must not alias");
        MB_CHECK(rtol > 0.0, MBAMG_E_INVALID, "rtol must be positive");
        mbamg_status st = solve_impl(h, b, x, rtol, (hipStream_t)hip_stream);
        if (info) *info = h->info;
        return st;
    });
}

mbamg_status mbamg_get_info(const mbamg_hierarchy* h, mbamg_info* info) {
    if (!h || !info) { g_last_error = "NULL argument"; return MBAMG_E_INVALID; }
    *info = h->info;
    return MBAMG_OK;
}

void mbamg_destroy(mbamg_hierarchy* h) {
    delete h;   // the destructor synchronises the device before its buffers are released
    pool_device_idle();
}

mbamg_status mbamg_num_levels(const mbamg_hierarchy* h, int32_t* n_levels) {
    if (h && n_levels && h->nb > 2) {
        *n_levels = (int32_t)h->GL.size();
        return MBAMG_OK;
    }
    if (!h || !n_levels) { g_last_error = "NULL argument"; return MBAMG_E_INVALID; }
    *n_levels = (int32_t)h->L.size();
    return MBAMG_OK;
}

mbamg_status mbamg_level_nodes(const mbamg_hierarchy* h, int32_t level, int32_t* n_nodes) {
    if (h && h->nb > 2) return mbamg_level_block_nodes(h, level, 0, n_nodes);
    if (!h || !n_nodes || level < 0 || level >= (int)h->L.size()) { g_last_error = "bad argument"; return MBAMG_E_INVALID; }
    *n_nodes = h->L[level]->n;
    return MBAMG_OK;
}

mbamg_status mbamg_copy_aggregates(const mbamg_hierarchy* h, int32_t level, int32_t* agg) {
    return mbamg_copy_block_aggregates(h, level, 0, agg);
}

mbamg_status mbamg_level_block_nodes(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t* n_nodes) {
    if (h && n_nodes && h->nb > 2) {
        if (level < 0 || level >= (int)h->GL.size() || f < 0 || f >= h->nb) {
            g_last_error = "bad argument";
            return MBAMG_E_INVALID;
        }
        *n_nodes = h->GL[level]->n;
        return MBAMG_OK;
    }
    if (!h || !n_nodes || level < 0 || level >= (int)h->L.size() || f < 0 || f > 1) {
        g_last_error = "bad argument";
        return MBAMG_E_INVALID;
    }
    *n_nodes = h->L[level]->nodes(f);
    return MBAMG_OK;
}

mbamg_status mbamg_copy_block_aggregates(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t* agg) {
    return guarded([&]() -> mbamg_status {
        if (h && h->nb > 2) {
            MB_CHECK(agg && level >= 0 && level + 1 < (int)h->GL.size() && f >= 0 && f < h->nb, MBAMG_E_INVALID,
                     "bad argument");
            const GLevel& L = *h->GL[level];
            MB_HIP(hipMemcpy(agg, L.G.agg.p, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
            return MBAMG_OK;
        }
        MB_CHECK(h && agg && level >= 0 && level + 1 < (int)h->L.size() && f >= 0 && f < 2, MBAMG_E_INVALID,
                 "bad argument");
        const Level& L = *h->L[level];
        MB_HIP(hipMemcpy(agg, L.agg_of(f).agg.p, sizeof(int32_t) * L.nodes(f), hipMemcpyDeviceToHost));
        return MBAMG_OK;
    });
}

mbamg_status mbamg_level_nnzb(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t g, int64_t* nnzb) {
    if (h && nnzb && h->nb > 2) {
        if (level < 0 || level >= (int)h->GL.size() || f < 0 || f >= h->nb || g < 0 || g >= h->nb) {
            g_last_error = "bad argument";
            return MBAMG_E_INVALID;
        }
        *nnzb = h->GL[level]->A[f][g].nnzb;
        return MBAMG_OK;
    }
    if (!h || !nnzb || level < 0 || level >= (int)h->L.size() || f < 0 || f > 1 || g < 0 || g > 1) {
        g_last_error = "bad argument";
        return MBAMG_E_INVALID;
    }
    *nnzb = h->L[level]->A[f][g].nnzb;
    return MBAMG_OK;
}

mbamg_status mbamg_copy_level_block(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t g, int32_t* row_ptr,
                                    int32_t* col_idx, double* vals) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && row_ptr && f >= 0 && f < h->nb && g >= 0 && g < h->nb, MBAMG_E_INVALID, "bad argument");
        MB_CHECK(level >= 0 && level < (int)(h->nb > 2 ? h->GL.size() : h->L.size()), MBAMG_E_INVALID, "bad argument");
        const SetupBsr& A = h->nb > 2 ? h->GL[level]->A[f][g] : h->L[level]->A[f][g];
        MB_HIP(hipMemcpy(row_ptr, A.rp.p, sizeof(int32_t) * (A.n_rows + 1), hipMemcpyDeviceToHost));
        if (A.nnzb) {
            MB_CHECK(col_idx && vals, MBAMG_E_INVALID, "NULL argument");
            MB_HIP(hipMemcpy(col_idx, A.ci.p, sizeof(int32_t) * A.nnzb, hipMemcpyDeviceToHost));
            MB_HIP(hipMemcpy(vals, A.val.p, sizeof(double) * A.nnzb * A.br * A.bc, hipMemcpyDeviceToHost));
        }
        return MBAMG_OK;
    });
}

mbamg_status mbamg_copy_colours(const mbamg_hierarchy* h, int32_t level, int32_t f, int32_t* colour) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && colour && f >= 0 && f < h->nb, MBAMG_E_INVALID, "bad argument");
        MB_CHECK(level >= 0 && level + 1 < (int)(h->nb > 2 ? h->GL.size() : h->L.size()), MBAMG_E_INVALID,
                 "bad argument");
        const BlockLevel& B = h->nb > 2 ? h->GL[level]->blk[f] : h->L[level]->blk[f];
        std::copy(B.colour.begin(), B.colour.end(), colour);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_timing_enable(mbamg_hierarchy* h, int32_t enable) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h, MBAMG_E_INVALID, "NULL argument");
        MB_HIP(hipDeviceSynchronize());
        for (auto& t : h->timed) {
            h->event_pool.push_back(t.a);
            h->event_pool.push_back(t.b);
        }
        h->timed.clear();
        MB_CHECK(enable >= 0 && enable <= 3, MBAMG_E_INVALID, "timing mode must be 0..3");
        h->timing = enable;
        return MBAMG_OK;
    });
}

mbamg_status mbamg_timing_get(mbamg_hierarchy* h, int32_t kind, int64_t* launches, double* total_ms, double* bytes) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && launches && total_ms && bytes, MBAMG_E_INVALID, "NULL argument");
        int64_t c = 0;
        double ms = 0.0, by = 0.0;
        for (auto& t : h->timed) {
            if (t.kind != kind) continue;
            MB_HIP(hipEventSynchronize(t.b));
            float e = 0.0f;
            MB_HIP(hipEventElapsedTime(&e, t.a, t.b));
            ++c;
            ms += e;
            by += t.bytes;
        }
        *launches = c;
        *total_ms = ms;
        *bytes = by;
        return MBAMG_OK;
    });
}

mbamg_status mbamg_vcycle_bytes(const mbamg_hierarchy* h, double* bytes) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && bytes, MBAMG_E_INVALID, "NULL argument");
        MB_CHECK(h->nb == 2, MBAMG_E_STATE, "the byte model covers two-block hierarchies");
        double tot = 0.0;
        for (int l = 0; l < (int)h->L.size(); ++l) {
            double down = 0.0, up = 0.0;
            level_vcycle_bytes(h, l, down, up);
            tot += down + up;
        }
        *bytes = tot;
        return MBAMG_OK;
    });
}

mbamg_status mbamg_level_vcycle_bytes(const mbamg_hierarchy* h, int32_t level, double* down, double* up) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && down && up, MBAMG_E_INVALID, "NULL argument");
        MB_CHECK(h->nb == 2, MBAMG_E_STATE, "the byte model covers two-block hierarchies");
        MB_CHECK(level >= 0 && level < (int)h->L.size(), MBAMG_E_INVALID, "bad argument");
        level_vcycle_bytes(h, level, *down, *up);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_features(const mbamg_hierarchy* h, int32_t level, float* features) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && features && level >= 0 && level + 1 < (int)h->L.size(), MBAMG_E_INVALID, "bad argument");
        const Level& L = *h->L[level];
        MB_CHECK(L.feat.p != nullptr, MBAMG_E_STATE, "features are computed only for the learned forms");
        MB_HIP(hipMemcpy(features, L.feat.p, sizeof(float) * L.G.n_agg * N_FEATURES, hipMemcpyDeviceToHost));
        return MBAMG_OK;
    });
}

mbamg_status mbamg_level_weights(const mbamg_hierarchy* h, int32_t level, double* omega_p, double* omega_s) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && omega_p && omega_s && level >= 0 && level + 1 < (int)h->L.size(), MBAMG_E_INVALID,
                 "bad argument");
        const Level& L = *h->L[level];
        const int nc = L.G.n_agg;
        if (L.smoothed) MB_HIP(hipMemcpy(omega_p, L.wp_agg.p, sizeof(double) * nc, hipMemcpyDeviceToHost));
        else std::fill(omega_p, omega_p + nc, 0.0);
        if (L.damped) {
            MB_HIP(hipMemcpy(omega_s, L.ws_agg.p, sizeof(double) * nc, hipMemcpyDeviceToHost));
        } else {
            std::fill(omega_s, omega_s + nc, h->p.omega);
        }
        return MBAMG_OK;
    });
}

mbamg_status mbamg_mlp_forward(const float* params, const float* x, int64_t n, float* out, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(params && x && out && n >= 0, MBAMG_E_INVALID, "bad argument");
        mlp_forward(params, x, n, out, (hipStream_t)hip_stream);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_mlp_loss_grad(const float* params, const float* x, const float* target, int64_t n, float* grad,
                                 float* loss, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(params && x && target && grad && n > 0, MBAMG_E_INVALID, "bad argument");
        static thread_local DevBuf<float> partial;
        hipStream_t s = (hipStream_t)hip_stream;
        mlp_loss_grad(params, x, target, n, grad, loss, partial, s);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_mlp_loss_grad_noalloc(const float* params, const float* x, const float* target, int64_t n,
                                         float* grad, float* loss, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(params && x && target && grad && n > 0, MBAMG_E_INVALID, "bad argument");
        mlp_loss_grad_noalloc(params, x, target, n, grad, loss, (hipStream_t)hip_stream);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                            float beta2, float eps, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(params && grad && m && v && step >= 1, MBAMG_E_INVALID, "bad argument");
        mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)hip_stream);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_probe(mbamg_hierarchy* h, int32_t iters, uint64_t seed, double* rho, void* hip_stream) {
    return guarded([&]() -> mbamg_status {
        MB_CHECK(h && rho, MBAMG_E_INVALID, "NULL argument");
        *rho = probe_impl(h, iters, seed, (hipStream_t)hip_stream);
        return MBAMG_OK;
    });
}

mbamg_status mbamg_set_omega(mbamg_hierarchy* h, double omega) {
    if (!h || !(omega > 0.0) || !std::isfinite(omega)) {
        g_last_error = "omega must be finite and > 0";
        return MBAMG_E_INVALID;
    }
    h->p.omega = omega;
    // a judged learned hierarchy's fixed-weight fallback smooths with the same damping
    if (h->fallback) h->fallback->p.omega = omega;
    return MBAMG_OK;
}

}  // extern "C"

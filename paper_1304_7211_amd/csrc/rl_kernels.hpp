// HIP kernels for CDNA4 (gfx950): the Richardson-Lucy hot path.
//
//   phase A   v = u^k * h  (forward convolution), r = f / v            (Section 2, eq. 3)
//   phase B   c = h^* * r  (adjoint correlation), u^{k+1} = u^k . c   (Section 2, eq. 3)
//   thinning  pixels with a converged counter are skipped; every R-th step is full,
//             and the active set is recompacted into a list           (Section 4, eq. 4-5)
//
// Operators are evaluated in "correlation form": out(a, b) = sum over spans of
// sum_t w[t] * src(a + lane_off, b + c0 + t).  Axis a is the lane axis (one wavefront lane
// per image line), axis b is the strip axis (each lane produces S consecutive outputs).
// ORIENT_ROWS: a = row, b = column.  ORIENT_COLS: a = column, b = row.
// The LDS tile is always stored row-major (image rows), with an odd pitch so that lanes
// reading different rows of the same column hit different banks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlk {

constexpr int ORIENT_ROWS = 0;
constexpr int ORIENT_COLS = 1;
constexpr int BC_REFLECT = 0;
constexpr int BC_REPLICATE = 1;
constexpr int THIN_OFF = 0;
constexpr int THIN_ABS = 1;
constexpr int THIN_REL = 2;
constexpr int SCHED_RING = 4096;  // per-iteration active-count ring
constexpr int ACT_SLOTS = 256;     // spread slots for the per-iteration active count

// device copy of rl::Span (same layout)
struct DevSpan {
    int32_t lane_off, c0, len, woff;
    float w0;
    int32_t uniform, row_end, pad;
};

// The PSF tables do not change while a kernel runs; reading them through the constant
// address space lets the compiler use scalar loads (one per wavefront, through the scalar
// cache) instead of per-lane vector loads with a full memory round trip per span.
typedef const __attribute__((address_space(4))) DevSpan* ConstSpanPtr;
typedef const __attribute__((address_space(4))) float* ConstFloatPtr;
__device__ __forceinline__ ConstSpanPtr as_const(const DevSpan* p) { return (ConstSpanPtr)p; }
__device__ __forceinline__ ConstFloatPtr as_const(const float* p) { return (ConstFloatPtr)p; }
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) i32x4* ConstI32x4Ptr;
// One span descriptor as two 16-byte scalar loads (the compiler merges them into one).
__device__ __forceinline__ DevSpan load_span(ConstSpanPtr t, int i) {
    const ConstI32x4Ptr q = (ConstI32x4Ptr)(t + i);
    const i32x4 a = q[0], b = q[1];
    DevSpan s;
    s.lane_off = a.x;
    s.c0 = a.y;
    s.len = a.z;
    s.woff = a.w;
    s.w0 = __int_as_float(b.x);
    s.uniform = b.y;
    s.row_end = b.z;
    s.pad = 0;
    return s;
}

// Index of this wavefront within its workgroup.  threadIdx.x >> 6 is the same for every
// lane of a wavefront, but the compiler cannot prove it; reading it through readfirstlane
// makes it a scalar, so loops and branches on it run on the scalar unit without exec-mask
// bookkeeping.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Boundary fold of index i into [0, n) (Section 2, "Boundary treatment").
__device__ __forceinline__ int fold_idx(int i, int n, int bc) {
    if ((unsigned)i < (unsigned)n) return i;
    if (bc == BC_REPLICATE) return i < 0 ? 0 : n - 1;
    int m = 2 * n;
    int p = i % m;
    if (p < 0) p += m;
    return p < n ? p : m - 1 - p;
}

// 1 for a non-zero value, 0 for +0 and -0 (inputs are >= 0 apart from the sign of zero,
// so min(bits << 1, 1) does it in integer ops).  Every input is >= 0, so a window sum is
// exactly 0 iff its count of non-zero inputs is 0, which a sliding float sum -- after
// subtracting the larger values that left the window -- does not reproduce exactly.  Exact
// zeros matter: v = 0 gives r = 0 where a near-zero v gives a huge ratio, and c = 0 gives
// u^{k+1} = 0 exactly.  The sliding kernels therefore count non-zero inputs where an
// all-zero window is possible (witness inputs or tile_zeros below decide where).
__device__ __forceinline__ int nz(float x) { return (int)min(__float_as_uint(x) << 1, 1u); }

// Kahan-compensated accumulation: s + x with running compensation c.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// The float32 convergence test of thinned RL (Section 4), one rounded op per step: false
// for tau <= 0; else true when a and b are both 0 or |a - b| < t (t = tau, or tau * b for
// the relative test).  Written without branches (bitwise and / or of the comparisons), so
// that a wavefront evaluates it without exec-mask bookkeeping.
__device__ __forceinline__ bool thin_below(float a, float b, int mode, float tau) {
    const float t = (mode == THIN_REL) ? __fmul_rn(tau, b) : tau;
    const bool zero = (a == 0.f) & (b == 0.f);
    return (tau > 0.f) & (zero | (fabsf(__fsub_rn(a, b)) < t));
}

// r = f / v for v > 0, else 0 (IEEE-rounded division).
__device__ __forceinline__ float rl_ratio(float f, float v) {
    return v > 0.f ? __fdiv_rn(f, v) : 0.f;
}

// Everything a phase kernel needs to know about one job.  Lives in device memory (the
// job's workspace, or a batch table) and is read with scalar loads.
struct PhaseArgs {
    int32_t H, W, bc, kahan;
    const float* src;     // u^k (phase A) or r (phase B)
    const float* f;       // phase A
    float* r;             // phase A output
    float* u;             // phase B in/out
    uint8_t* cnt;         // thinning counters (NULL when off): one per pixel, or one per
                          // block under the block rule (blk_lg > 0)
    const DevSpan* spans; // operator table
    const float* wts;     // operator weights (padded with zeros)
    int32_t n_spans;
    int32_t lane_min, lane_max, c_min, c_max;
    int32_t tiles_a, tiles_b;      // tile grid (lane axis, strip axis)
    const int32_t* tile_list;      // thinned: list of tile ids (used on non-full steps)
    const int64_t* tile_count;     // its length (device)
    int32_t thin_mode, hyst, reset_period, full;  // thinning (full is derived per launch)
    float tau;
    int32_t list_ok;               // thinned non-full steps: 1 = use the tile list, 0 = all
                                   // tiles (frozen pixels are still skipped per pixel)
    int64_t* sched;                // active-count ring (thinning)
    int64_t* active_total;         // running sum of |A_k|
    int32_t* act_part;             // 2 banks x ACT_SLOTS partial active counts
    int64_t k;                     // base iteration index (plus LaunchArgs::kb)
    const float* tvg;              // phase B: TV denominator 1 - lambda div(...) or NULL
    int32_t wit;                   // sliding kernel: a span at least one strip long, or -1
    float* store;                  // robust variant: store the window sum here and nothing else
    int32_t blk_lg;                // block rule: log2 of the block side (3..6), 0 = per pixel
    int32_t blk_w;                 // block rule: blocks per image row
    int32_t* tflag;                // block rule: per tile, 1 while it holds an active block
};

// One launch covers the tiles of n_jobs jobs: job j owns workgroups
// [prefix[j], prefix[j+1]).  kb is added to every job's base iteration index.
struct LaunchArgs {
    const PhaseArgs* table;
    const int32_t* prefix;
    int32_t n_jobs, n_tiles1;  // n_tiles1: tile count when n_jobs == 1
    int64_t kb;
    PhaseArgs one;             // the job itself when n_jobs == 1 (saves a dependent load)
};

typedef const __attribute__((address_space(4))) PhaseArgs* ConstArgsPtr;
typedef const __attribute__((address_space(4))) int32_t* ConstIntPtr;

__device__ __forceinline__ PhaseArgs load_args(ConstArgsPtr t) {
    PhaseArgs p;
    p.H = t->H; p.W = t->W; p.bc = t->bc; p.kahan = t->kahan;
    p.src = t->src; p.f = t->f; p.r = t->r; p.u = t->u; p.cnt = t->cnt;
    p.spans = t->spans; p.wts = t->wts; p.n_spans = t->n_spans;
    p.lane_min = t->lane_min; p.lane_max = t->lane_max; p.c_min = t->c_min; p.c_max = t->c_max;
    p.tiles_a = t->tiles_a; p.tiles_b = t->tiles_b;
    p.tile_list = t->tile_list; p.tile_count = t->tile_count;
    p.thin_mode = t->thin_mode; p.hyst = t->hyst; p.reset_period = t->reset_period;
    p.full = t->full; p.tau = t->tau; p.list_ok = t->list_ok;
    p.sched = t->sched; p.active_total = t->active_total; p.act_part = t->act_part; p.k = t->k;
    p.tvg = t->tvg;
    p.wit = t->wit;
    p.store = t->store;
    p.blk_lg = t->blk_lg;
    p.blk_w = t->blk_w;
    p.tflag = t->tflag;
    return p;
}

// Map a workgroup index to a tile so that each XCD (workgroups are dispatched to the 8
// XCDs round-robin) gets one contiguous range of tiles: neighbouring tiles share halo
// rows/columns, which then stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    int xcd = b & 7, idx = b >> 3;
    int base = n >> 3, rem = n & 7;
    int start = xcd * base + (xcd < rem ? xcd : rem);
    return start + idx;
}

// Add the spread partial active counts of iteration k (bank k & 1) to its schedule-ring
// slot and to the running total, and clear the bank (folding an already folded bank adds
// 0).  If k_next >= 0, also clear the ring slot of iteration k_next.  One wavefront.
__device__ __forceinline__ void thin_finalize_wave(int32_t* act_part, int64_t* sched,
                                                   int64_t* active_total, int64_t k,
                                                   int64_t k_next) {
    const int lane = threadIdx.x & 63;
    int64_t v = 0;
    if (k >= 0) {
        int32_t* bank = act_part + (k & 1) * ACT_SLOTS;
#pragma unroll
        for (int q = 0; q < ACT_SLOTS / 64; ++q) {
            v += bank[lane + 64 * q];
            bank[lane + 64 * q] = 0;
        }
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    }
    if (lane == 0) {
        if (k >= 0) {
            sched[k % SCHED_RING] += v;
            *active_total += v;
        }
        if (k_next >= 0) sched[k_next % SCHED_RING] = 0;
    }
}

// Find this workgroup's job and tile.  Returns false if the workgroup has no tile (thinned
// steps launch one workgroup per tile of the grid and use only as many as the list has).
// Thinned mode: iteration k is full when k == 0 or k % R == 0; on other steps the tiles
// come from the compacted list.  The first wavefront of a job's first workgroup in phase A
// folds the active count of iteration k - 1 into the schedule ring (phase B of iteration
// k - 1 spread it over ACT_SLOTS counters, one atomic add per tile in thin_finish: spread,
// so that thousands of tiles do not serialise on one address; integer adds, so the total
// does not depend on their order).
template <bool PHASE_B>
__device__ __forceinline__ bool resolve(const LaunchArgs& L, PhaseArgs& p, int TA, int TB,
                                        int& a0, int& b0) {
    const int b = blockIdx.x;
    int local;
    if (L.n_jobs == 1) {
        p = L.one;
        local = b;
    } else {
        const ConstIntPtr pre = (ConstIntPtr)L.prefix;
        int lo = 0, hi = L.n_jobs - 1;
        while (lo < hi) {  // last job with prefix <= b
            int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        p = load_args((ConstArgsPtr)L.table + lo);
        local = b - pre[lo];
    }
    p.k += L.kb;
    bool use_list = false;
    if (p.cnt) {
        // single-job launches carry the host's full-step flag; batch launches derive it
        if (L.n_jobs != 1)
            p.full = (p.k == 0 || (p.reset_period > 0 && p.k % p.reset_period == 0)) ? 1 : 0;
        use_list = !p.full && p.list_ok;
        if (!PHASE_B && local == 0 && threadIdx.x < 64)
            thin_finalize_wave(p.act_part, p.sched, p.active_total, p.k - 1, p.k);
    } else {
        p.full = 1;
    }
    // list length and entries through the constant address space: scalar loads, written
    // by the rebuild before this launch
    typedef const __attribute__((address_space(4))) int64_t* ConstI64Ptr;
    const int n = use_list ? (int)*(ConstI64Ptr)p.tile_count : p.tiles_a * p.tiles_b;
    // XCD-aware order (single-job launches): workgroups local < n form a permutation of the
    // n tiles (or list entries, which are ascending tile ids) with one contiguous range per
    // XCD; workgroups past n (thinned steps with a short list) have no tile
    if (local >= n) return false;
    const int slot = (L.n_jobs == 1) ? xcd_tile(local, n) : local;
    const int t = use_list ? ((ConstIntPtr)p.tile_list)[slot] : slot;
    // block rule, non-full step: a tile whose blocks have all frozen (since the list was
    // built, or since the last rebuild found nearly every tile active and dropped the list)
    // has nothing to do; its flag was written by the tile's own phase B of the previous
    // iteration
    if (p.cnt && p.blk_lg && !p.full && ((ConstIntPtr)p.tflag)[t] == 0) return false;
    a0 = (t % p.tiles_a) * TA;
    b0 = (t / p.tiles_a) * TB;
    return true;
}

// Cooperative load of the source tile (with halo and boundary fold) into LDS.
// LDS holds rows [ly0, ly0 + ny) x cols [lx0, lx0 + nx) of the folded image, row-major
// with the given pitch.  Each wavefront takes whole rows with its lanes along the columns
// (coalesced), and every (row, 64-column chunk) is one global-to-LDS DMA load
// (global_load_lds_dword: no VGPRs, no dependence on earlier loads), so the whole tile is
// in flight at once.  Lanes past the row end are masked off, so the DMA never writes
// outside the row.  Column folds and lane masks are computed once; the row loop runs on
// the scalar unit (row, its fold and the LDS row address are wavefront-uniform).  The
// caller waits (lds_dma_wait) and synchronises before reading.
constexpr int MAXC = 5;
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void load_tile(float* lds, const float* __restrict__ src, int H,
                                          int W, int bc, int ly0, int lx0, int ny, int nx,
                                          int pitch) {
    const int nwv = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, wv = wave_id();
    int gx[MAXC];
    bool on[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int col = lane + 64 * c;
        on[c] = col < nx;
        gx[c] = on[c] ? fold_idx(lx0 + col, W, bc) : 0;
    }
    const int nch = (nx + 63) >> 6;
    for (int row = wv; row < ny; row += nwv) {
        const float* srow = src + (size_t)fold_idx(ly0 + row, H, bc) * W;
        float* drow = lds + row * pitch;
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c < nch && on[c])
                __builtin_amdgcn_global_load_lds((const void*)(srow + gx[c]),
                                                 (lds_void*)(drow + 64 * c), 4, 0, 0);
        }
    }
}

// Wait for this wavefront's outstanding global loads, including LDS DMA.
__device__ __forceinline__ void lds_dma_wait() { __builtin_amdgcn_s_waitcnt(0); }

// Zero detection on a tile loaded by load_tile.  Called by every wavefront after its own
// lds_dma_wait(): it scans exactly the rows and columns its own loads wrote (rows wv,
// wv + nwv, ...; columns lane, lane + 64, ...) and publishes one flag word zf[wv] for the
// workgroup barrier that follows; tile_zeros() then reads the OR of the flags (uniform).
// The scan keeps the minimum of |value| with eight reads in flight per step, so it costs
// a few LDS round trips rather than one per row.
__device__ __forceinline__ void note_zeros(const float* lds, int ny, int nx, int pitch, int* zf) {
    const int nwv = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, wv = wave_id();
    float m = 1.f;
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        if (lane + 64 * c < nx) {
            const float* col = lds + lane + 64 * c;
            int row = wv;
            for (; row + 7 * nwv < ny; row += 8 * nwv) {
                float v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = fabsf(col[(row + i * nwv) * pitch]);
                m = fminf(m, fminf(fminf(fminf(v[0], v[1]), fminf(v[2], v[3])),
                                   fminf(fminf(v[4], v[5]), fminf(v[6], v[7]))));
            }
            for (; row < ny; row += nwv) m = fminf(m, fabsf(col[row * pitch]));
        }
    }
    const bool any = __ballot(m == 0.f) != 0ull;
    if (lane == 0) zf[wv] = any ? 1 : 0;
}

template <int NW>
__device__ __forceinline__ bool tile_zeros(const int* zf) {
    int o = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) o |= zf[w];
    return __builtin_amdgcn_readfirstlane(o) != 0;
}

// Epilogue inputs of one output at pixel (y, x), linear position q: f (phase A) or u^k
// (phase B), and the convergence counter in thinned mode (the pixel's own, or its block's
// under the block rule).  Gathered for all outputs of a lane before any is applied, so the
// global loads overlap.
struct EpiIn {
    float x;
    uint8_t c8;
};

// Index of the counter that decides pixel (y, x): q itself, or its block's under the block
// rule (blocks of 2^blk_lg pixels a side, aligned at (0, 0)).
__device__ __forceinline__ size_t cnt_idx(const PhaseArgs& p, int y, int x, size_t q) {
    return p.blk_lg ? (size_t)(y >> p.blk_lg) * p.blk_w + (x >> p.blk_lg) : q;
}

// Block rule: bit of pixel (y, x)'s block among the blocks of its 64 x 64 tile (tiles are
// 64-aligned, so the tile-relative position is the low six bits of y and x).
__device__ __forceinline__ int blk_bit(const PhaseArgs& p, int y, int x) {
    return (((y & 63) >> p.blk_lg) << (6 - p.blk_lg)) | ((x & 63) >> p.blk_lg);
}

template <bool PHASE_B>
__device__ __forceinline__ EpiIn epi_load(const PhaseArgs& p, int y, int x, size_t q) {
    EpiIn e;
    e.x = PHASE_B ? p.u[q] : p.f[q];
    e.c8 = p.cnt ? p.cnt[cnt_idx(p, y, x, q)] : (uint8_t)0;
    return e;
}

// Apply the epilogue: phase A writes r = f / v; phase B writes u^{k+1} = u^k . c and, in
// thinned mode, the counter (per-pixel rule) or, under the block rule, sets the pixel's
// block bit in fails when the pixel fails the convergence test (block_finish turns the bits
// into block counters).  Inactive pixels (thinned, non-full step) are left alone.  Returns
// 1 if the pixel was active.
template <bool PHASE_B>
__device__ __forceinline__ int epi_apply(const PhaseArgs& p, int y, int x, size_t q, EpiIn e,
                                         float val, uint64_t& fails) {
    if (p.cnt && !(p.full || (int)e.c8 < p.hyst)) return 0;
    if (p.store) {  // robust variant: the plain convolution or correlation
        p.store[q] = val;
        return 1;
    }
    if (!PHASE_B) {
        p.r[q] = rl_ratio(e.x, val);
    } else {
        float un = __fmul_rn(e.x, val);
        // TV-regularised jobs: the denominator is read here rather than prefetched, so
        // plain jobs carry no extra register per output
        if (p.tvg) un = __fdiv_rn(un, p.tvg[q]);
        p.u[q] = un;
        if (p.cnt && p.thin_mode != THIN_OFF) {
            bool below = thin_below(un, e.x, p.thin_mode, p.tau);
            if (p.blk_lg) {
                fails |= (uint64_t)(!below) << blk_bit(p, y, x);
            } else {
                p.cnt[q] = below ? (uint8_t)(e.c8 < 255 ? e.c8 + 1 : 255) : (uint8_t)0;
            }
        }
    }
    return 1;
}

// Block rule, phase B: the counter of block threadIdx.x of the 64 x 64 tile at (ty0, tx0)
// (row, column of its top-left pixel), loaded with the epilogue inputs so that block_finish
// needs no load of its own; 0 for threads without a block.
template <bool PHASE_B>
__device__ __forceinline__ uint8_t blk_own_load(const PhaseArgs& p, int ty0, int tx0) {
    if (!PHASE_B || !p.cnt || !p.blk_lg) return 0;
    const int per = 64 >> p.blk_lg, t = threadIdx.x;
    if (t >= per * per) return 0;
    const int by = (ty0 >> p.blk_lg) + t / per, bx = (tx0 >> p.blk_lg) + t % per;
    if ((by << p.blk_lg) >= p.H || (bx << p.blk_lg) >= p.W) return 0;
    return p.cnt[(size_t)by * p.blk_w + bx];
}

// OR and sum over the 64 lanes of a wavefront with DPP row shifts and row broadcasts
// (gfx9 lane movement, a few cycles per step): prefix within each row of 16 lanes, then
// across rows; lane 63 holds the result, which is returned to every lane.  Lanes whose
// source falls outside the row contribute 0, the identity of both operations.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return __builtin_amdgcn_readlane(v, 63);
}

// Block rule, end of phase B of one 64 x 64 tile (tile id `tile`, top-left pixel
// (ty0, tx0)): the failure bits of every lane are OR-ed over the workgroup, then each
// active block of the tile (one thread per block, own_c its counter) counts up if none of
// its pixels failed the test, else restarts at 0.  Blocks cut by the image edge hold only
// their pixels inside the image.  The tile's flag then records whether any of its blocks
// is active in the next iteration, and the pixels of the tile's active blocks go into the
// active count (one atomic add per tile).  Every thread of the workgroup must call it (it
// synchronises).
__device__ __forceinline__ void block_finish(const PhaseArgs& p, uint64_t fails, int ty0,
                                             int tx0, uint8_t own_c, int tile) {
    __shared__ uint64_t slot[16];
    const uint32_t lo = wave_or((uint32_t)fails), hi = wave_or((uint32_t)(fails >> 32));
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0) slot[wave_id()] = ((uint64_t)hi << 32) | lo;
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int lg = p.blk_lg, per = 64 >> lg;  // blocks per tile side
    const int t = threadIdx.x;
    bool next_active = false;
    int area = 0;
    if (t < per * per) {
        const int by = (ty0 >> lg) + t / per, bx = (tx0 >> lg) + t % per;
        const int y0 = by << lg, x0 = bx << lg;
        if (y0 < p.H && x0 < p.W) {
            uint64_t all = 0;
            for (int w = 0; w < nw; ++w) all |= slot[w];
            int c = own_c;
            if (p.full || c < p.hyst) {
                area = min(1 << lg, p.H - y0) * min(1 << lg, p.W - x0);
                c = ((all >> t) & 1ull) ? 0 : (c < 255 ? c + 1 : 255);
                p.cnt[(size_t)by * p.blk_w + bx] = (uint8_t)c;
            }
            next_active = c < p.hyst;
        }
    }
    const bool any = __ballot(next_active) != 0ull;
    const int n_active = wave_sum(area);
    if (t == 0) {
        p.tflag[tile] = any ? 1 : 0;
        if (n_active)
            atomicAdd(&p.act_part[(p.k & 1) * ACT_SLOTS + (int)(blockIdx.x % ACT_SLOTS)], n_active);
    }
}

// End of a phase launch's tile in thinned mode: the active count and, in phase B under the
// block rule, the block counters and the tile's flag.  a0, b0 are the tile origin along the
// lane and strip axes (64 x 64 tiles under the block rule).  Called by every thread of the
// workgroup.
template <bool PHASE_B>
__device__ __forceinline__ void thin_finish(const PhaseArgs& p, int n_active, uint64_t fails,
                                            int ty0, int tx0, uint8_t own_c, int a0, int b0) {
    if (!PHASE_B || !p.cnt) return;
    if (p.blk_lg) {  // the active count comes from the block areas
        block_finish(p, fails, ty0, tx0, own_c, (b0 >> 6) * p.tiles_a + (a0 >> 6));
    } else {
        // per-pixel rule: the wavefronts' counts summed in LDS, one atomic add per tile
        __shared__ int wsum[16];
        if ((threadIdx.x & 63) == 0) wsum[wave_id()] = n_active;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wsum[w];
            if (tot) atomicAdd(&p.act_part[(p.k & 1) * ACT_SLOTS + (int)(blockIdx.x % ACT_SLOTS)], tot);
        }
    }
}

// Common tile set-up.  TA = 64 lanes, TB = NW * S strip positions.
template <int ORIENT>
struct TileGeom {
    int a0, b0, ly0, lx0, ny, nx, pitch;
    // LDS index of the element at tile-relative (a, b) (a already includes -lane_min,
    // b already includes -c_min).
    __device__ __forceinline__ int idx(int a, int b) const {
        return ORIENT == ORIENT_ROWS ? a * pitch + b : b * pitch + a;
    }
    // idx(la + da, b) split into a per-lane part (computed once per kernel) and a
    // wavefront-uniform part (scalar arithmetic per span).
    __device__ __forceinline__ int lane_part(int la) const {
        return ORIENT == ORIENT_ROWS ? la * pitch : la;
    }
    __device__ __forceinline__ int uni_part(int da, int b) const {
        return ORIENT == ORIENT_ROWS ? da * pitch + b : b * pitch + da;
    }
    // distance between neighbouring strip positions
    __device__ __forceinline__ int bstep() const { return ORIENT == ORIENT_ROWS ? 1 : pitch; }
};

template <int ORIENT>
__device__ __forceinline__ TileGeom<ORIENT> make_geom(const PhaseArgs& p, int a0, int b0,
                                                       int TA, int TB, int extra) {
    TileGeom<ORIENT> g;
    g.a0 = a0;
    g.b0 = b0;
    int na = TA + p.lane_max - p.lane_min;
    int nb = TB + p.c_max - p.c_min + extra;
    if (ORIENT == ORIENT_ROWS) {
        g.ly0 = a0 + p.lane_min;
        g.lx0 = b0 + p.c_min;
        g.ny = na;
        g.nx = nb;
    } else {
        g.ly0 = b0 + p.c_min;
        g.lx0 = a0 + p.lane_min;
        g.ny = nb;
        g.nx = na;
    }
    g.pitch = g.nx | 1;
    return g;
}

// Epilogue inputs of the outputs a lane finishes: for ORIENT_COLS the lane's own strip
// (lanes are consecutive columns, so every access is coalesced), for ORIENT_ROWS the
// elements the lane handles after the LDS transpose.  Loaded at kernel entry so that they
// travel together with the tile.
// Plain jobs on images whose width is a multiple of 4, and thinned jobs under the block
// rule on such images: the ROWS epilogue moves four consecutive outputs per lane with
// 16-byte loads and stores (the four share one block, so one counter decides them).  (Jobs
// with per-pixel counters, TV and robust jobs keep the per-output epilogue: a general
// four-wide one measured slower for every job.)
__device__ __forceinline__ bool epi_vec(const PhaseArgs& p) {
    return (p.W & 3) == 0 && (!p.cnt || p.blk_lg) && !p.tvg && !p.store;
}

template <int ORIENT, int S, int NW>
struct EpiPlan {
    static constexpr int TB = NW * S;
    static constexpr int PER = ORIENT == ORIENT_COLS ? S : (64 * TB) / (NW * 64);
    EpiIn in[PER];
    uint8_t own_c;  // block rule, phase B: see blk_own_load
};

template <int ORIENT, int S, int NW>
__device__ __forceinline__ void epi_pos(int i, int a0, int b0, int& y, int& x) {
    constexpr int TB = NW * S;
    const int lane = threadIdx.x & 63, wv = wave_id();
    if (ORIENT == ORIENT_COLS) {
        x = a0 + lane;
        y = b0 + wv * S + i;
    } else {
        int e = threadIdx.x + i * NW * 64;
        int row = e / TB, col = e % TB;
        y = a0 + row;
        x = b0 + col;
    }
}

template <int ORIENT, int S, int NW, bool PHASE_B>
__device__ __forceinline__ void epi_prefetch(const PhaseArgs& p, int a0, int b0,
                                             EpiPlan<ORIENT, S, NW>& plan) {
    plan.own_c = blk_own_load<PHASE_B>(p, ORIENT == ORIENT_COLS ? b0 : a0,
                                       ORIENT == ORIENT_COLS ? a0 : b0);
    if (ORIENT == ORIENT_ROWS && S % 4 == 0 && epi_vec(p)) {
        constexpr int TB = NW * S;
#pragma unroll
        for (int j = 0; j < S / 4; ++j) {
            const int flat = 4 * ((int)threadIdx.x + j * NW * 64);
            const int y = a0 + flat / TB, x = b0 + flat % TB;
            if (y < p.H && x < p.W) {
                const size_t q = (size_t)y * p.W + x;
                const float4 v = *reinterpret_cast<const float4*>((PHASE_B ? p.u : p.f) + q);
                plan.in[4 * j].x = v.x;
                plan.in[4 * j + 1].x = v.y;
                plan.in[4 * j + 2].x = v.z;
                plan.in[4 * j + 3].x = v.w;
                plan.in[4 * j].c8 = p.cnt ? p.cnt[cnt_idx(p, y, x, q)] : (uint8_t)0;
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < EpiPlan<ORIENT, S, NW>::PER; ++i) {
        int y, x;
        epi_pos<ORIENT, S, NW>(i, a0, b0, y, x);
        if (x < p.W && y < p.H) plan.in[i] = epi_load<PHASE_B>(p, y, x, (size_t)y * p.W + x);
    }
}

template <int ORIENT, int S, int NW, bool PHASE_B>
__device__ __forceinline__ void write_outputs(const PhaseArgs& p, float* lds, int a0, int b0,
                                              const float (&out)[S],
                                              const EpiPlan<ORIENT, S, NW>& plan) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    int n_active = 0;    // wavefront total, summed from ballots (phase B, thinned)
    uint64_t fails = 0;  // block rule: blocks of this lane's pixels that failed the test
    const int ty0 = ORIENT == ORIENT_COLS ? b0 : a0, tx0 = ORIENT == ORIENT_COLS ? a0 : b0;
    if (ORIENT == ORIENT_COLS) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            int y, x;
            epi_pos<ORIENT, S, NW>(s, a0, b0, y, x);
            int act = 0;
            if (x < p.W && y < p.H)
                act = epi_apply<PHASE_B>(p, y, x, (size_t)y * p.W + x, plan.in[s], out[s], fails);
            if (PHASE_B && p.cnt && !p.blk_lg) n_active += __popcll(__ballot(act));
        }
    } else {
        constexpr int TB = NW * S;
        constexpr int SP = TB + 1;
        __syncthreads();  // everyone is done reading the source tile
#pragma unroll
        for (int s = 0; s < S; ++s) lds[lane * SP + wv * S + s] = out[s];
        __syncthreads();
        if (S % 4 == 0 && epi_vec(p)) {
#pragma unroll
            for (int j = 0; j < S / 4; ++j) {
                const int flat = 4 * ((int)threadIdx.x + j * NW * 64);
                const int row = flat / TB, col = flat % TB;
                const int y = a0 + row, x = b0 + col;
                bool act = false;
                if (y < p.H && x < p.W) {
                    const float* st = lds + row * SP + col;
                    const EpiIn* e = &plan.in[4 * j];
                    // block rule: the four outputs share one block and its counter
                    act = !p.cnt || p.full || (int)e[0].c8 < p.hyst;
                    float4 o;
                    if (act && !PHASE_B) {
                        o = make_float4(rl_ratio(e[0].x, st[0]), rl_ratio(e[1].x, st[1]),
                                        rl_ratio(e[2].x, st[2]), rl_ratio(e[3].x, st[3]));
                        *reinterpret_cast<float4*>(p.r + (size_t)y * p.W + x) = o;
                    } else if (act) {
                        o = make_float4(__fmul_rn(e[0].x, st[0]), __fmul_rn(e[1].x, st[1]),
                                        __fmul_rn(e[2].x, st[2]), __fmul_rn(e[3].x, st[3]));
                        *reinterpret_cast<float4*>(p.u + (size_t)y * p.W + x) = o;
                        if (p.cnt) {
                            const bool all = thin_below(o.x, e[0].x, p.thin_mode, p.tau) &
                                             thin_below(o.y, e[1].x, p.thin_mode, p.tau) &
                                             thin_below(o.z, e[2].x, p.thin_mode, p.tau) &
                                             thin_below(o.w, e[3].x, p.thin_mode, p.tau);
                            fails |= (uint64_t)(!all) << blk_bit(p, y, x);
                        }
                    }
                }
                if (PHASE_B && p.cnt && !p.blk_lg) n_active += 4 * __popcll(__ballot(act));
            }
            thin_finish<PHASE_B>(p, n_active, fails, ty0, tx0, plan.own_c, a0, b0);
            return;
        }
#pragma unroll
        for (int i = 0; i < EpiPlan<ORIENT, S, NW>::PER; ++i) {
            int e = threadIdx.x + i * NW * 64;
            int row = e / TB, col = e % TB;
            int y, x;
            epi_pos<ORIENT, S, NW>(i, a0, b0, y, x);
            int act = 0;
            if (y < p.H && x < p.W)
                act = epi_apply<PHASE_B>(p, y, x, (size_t)y * p.W + x, plan.in[i],
                                         lds[row * SP + col], fails);
            if (PHASE_B && p.cnt && !p.blk_lg) n_active += __popcll(__ballot(act));
        }
    }
    thin_finish<PHASE_B>(p, n_active, fails, ty0, tx0, plan.own_c, a0, b0);
}

// ---------------------------------------------------------------------------------------
// Span kernel: every PSF line is cut into pieces of at most LMAX taps (any weights).  Per
// piece a lane loads a register window of S + len - 1 source values and forms S outputs
// from it (register blocking: one LDS read per output per piece instead of one per tap).
// The piece length selects, by a wavefront-uniform switch, a body with exactly len FMAs
// per output, so short pieces cost no padding.  Partial sums are per PSF line in float32;
// with compensation on (kahan = 1) lines go alternately into two accumulators added at
// the end (cascade summation, one add per line), else into one.  LMAX = 1 with the per-tap
// table is the DIRECT path.
// ---------------------------------------------------------------------------------------
template <int ORIENT, int S, int L>
__device__ __forceinline__ void span_piece_w(const float* base, const TileGeom<ORIENT>& g,
                                             const float* w, float (&part)[S]) {
    float win[S + L - 1];
    const int st = g.bstep();
#pragma unroll
    for (int q = 0; q < S + L - 1; ++q) win[q] = base[q * st];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        float a = part[s];
#pragma unroll
        for (int t = 0; t < L; ++t) a = fmaf(w[t], win[s + t], a);
        part[s] = a;
    }
}

template <int ORIENT, int S, int L>
__device__ __forceinline__ void span_piece(const float* base, const TileGeom<ORIENT>& g,
                                           ConstFloatPtr wp, float (&part)[S]) {
    float w[L];
#pragma unroll
    for (int t = 0; t < L; ++t) w[t] = wp[t];
    span_piece_w<ORIENT, S, L>(base, g, w, part);
}

// One output tile of a phase (span kernel): tile origin (a0, b0) on the lane and strip
// axes; lds is the workgroup's dynamic LDS.  Shared by the per-phase kernel and the
// persistent schedule.
template <int ORIENT, int S, int LMAX, int NW, bool PHASE_B>
__device__ __forceinline__ void span_tile(const PhaseArgs& p, int a0, int b0, float* lds) {
    constexpr int TA = 64, TB = NW * S;
    TileGeom<ORIENT> g = make_geom<ORIENT>(p, a0, b0, TA, TB, 0);
    EpiPlan<ORIENT, S, NW> plan;
    epi_prefetch<ORIENT, S, NW, PHASE_B>(p, a0, b0, plan);
    load_tile(lds, p.src, p.H, p.W, p.bc, g.ly0, g.lx0, g.ny, g.nx, g.pitch);
    lds_dma_wait();
    __syncthreads();

    const int lane = threadIdx.x & 63, wv = wave_id();
    const float* lane_lds = lds + g.lane_part(lane - p.lane_min);
    const int lb = wv * S - p.c_min;
    float acc0[S], acc1[S], part[S];
#pragma unroll
    for (int s = 0; s < S; ++s) { acc0[s] = 0.f; acc1[s] = 0.f; part[s] = 0.f; }
    const bool cascade = p.kahan != 0;
    bool odd = false;

    const ConstSpanPtr spans = as_const(p.spans);
    const ConstFloatPtr wts = as_const(p.wts);
    // one span of lookahead: the current span's LMAX weights (the weight table carries 16
    // zeros past its end) and the next span's descriptor (the span table carries zero
    // descriptors past its end) are loaded together, so each span waits for one scalar
    // round trip instead of two in a row
    DevSpan nsp = load_span(spans, 0);
    for (int i = 0; i < p.n_spans; ++i) {
        const DevSpan sp = nsp;
        float wl[LMAX];
#pragma unroll
        for (int t = 0; t < LMAX; ++t) wl[t] = wts[sp.woff + t];
        nsp = load_span(spans, i + 1);
        const float* base = lane_lds + g.uni_part(sp.lane_off, lb + sp.c0);
        switch (sp.len) {
#define RL_PIECE(n) \
    case n:         \
        if (n <= LMAX) span_piece_w<ORIENT, S, (n <= LMAX ? n : 1)>(base, g, wl, part); \
        break;
            RL_PIECE(1) RL_PIECE(2) RL_PIECE(3) RL_PIECE(4) RL_PIECE(5) RL_PIECE(6)
            RL_PIECE(7) RL_PIECE(8) RL_PIECE(9) RL_PIECE(10) RL_PIECE(11) RL_PIECE(12)
            RL_PIECE(13) RL_PIECE(14) RL_PIECE(15) RL_PIECE(16)
#undef RL_PIECE
            default: break;
        }
        if (sp.row_end) {
            if (cascade && odd) {
#pragma unroll
                for (int s = 0; s < S; ++s) { acc1[s] += part[s]; part[s] = 0.f; }
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s) { acc0[s] += part[s]; part[s] = 0.f; }
            }
            odd = !odd;
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) acc0[s] += acc1[s];
    write_outputs<ORIENT, S, NW, PHASE_B>(p, lds, a0, b0, acc0, plan);
}

template <int ORIENT, int S, int LMAX, int NW, bool PHASE_B>
__global__ __launch_bounds__(NW * 64) void span_kernel(LaunchArgs L) {
    extern __shared__ float lds[];
    int a0, b0;
    PhaseArgs p;
    if (!resolve<PHASE_B>(L, p, 64, NW * S, a0, b0)) return;
    span_tile<ORIENT, S, LMAX, NW, PHASE_B>(p, a0, b0, lds);
}

// ---------------------------------------------------------------------------------------
// Matrix-core kernel for PSFs with dense lines (the list filter, Section 3, evaluated as
// matrix products).  For one PSF line di, the correlation over a 16 x 16 output block is a
// product with a banded matrix:
//     out[m][n] += sum_{c < 32} A[m][c] * B[c][n],
//     A[m][c] = src(y0 + m + di, x0 + c_min + c),   B[c][n] = w(di, c_min + c - n)
// (B is zero outside the line's taps; lines are at most MF_MAXW taps wide), one
// v_mfma_f32_16x16x32_bf16 per line and block.  Float32 accuracy is kept by splitting every
// source value and weight into three bfloat16 parts, x = x1 + x2 + x3 (each part the
// rounded remainder of the previous; exact for float32 inputs), and forming the six products
// x_i w_j with i + j <= 4: the three dropped ones are below 2^-24 of the full product, and a
// product of two bfloat16 values is exact in float32.  The leading products x1 w1 of even
// and odd lines go into two accumulators, the five smaller ones into a third; the output is
// (even + odd) + small.  A window whose inputs are all zero gives exactly zero.
//
// A workgroup of NW wavefronts owns a 64 x 64 output tile.  With NW = 4 wavefront w
// computes rows 16 w .. 16 w + 15 as four 16 x 16 blocks side by side, which share each
// line's weight operand; with NW = 8 wavefront w computes two such blocks, rows
// 16 (w % 4) .., columns 32 (w / 4) ...  Every block sees the same sequence of products
// either way, so both give identical results: eight wavefronts finish a tile sooner (a
// single job's launch at 1 Mpx: 10.6 against 12.7-13.2 us), four keep more tiles per CU
// (a batch of many jobs, whose launches overlap on several streams, 395-403 against
// 407-417 ms).  The source tile (PSF halo included, boundary fold applied) is converted once
// into three bfloat16 planes in LDS with a row pitch of MF_PITCH elements (10 x 16 bytes,
// the unpadded row: of the pitches 80 .. 136 measured, 80 gave the fewest LDS bank-conflict
// cycles on the operand loads, a ninth of those of 88).  Operand layout of v_mfma_f32_16x16x32_bf16 on a wavefront of 64: lane l
// holds A[l % 16][8 (l / 16) + t] and B[8 (l / 16) + t][l % 16] for t < 8 and receives
// D[4 (l / 16) + t][l % 16] for t < 4.  The weight operands (per line, per part, per lane:
// 8 bfloat16 values) are built on the host; p.wts points to them.  The epilogue is the
// one of the other phase kernels (ratio or update, thinning counters, TV, robust store).
// ---------------------------------------------------------------------------------------
constexpr int MF_T = 64;             // tile rows and columns
constexpr int MF_NX = MF_T + 16;     // LDS columns: the last block reads 16 * 3 + 32
constexpr int MF_PITCH = 80;         // LDS row pitch in bfloat16 elements
constexpr int MF_MAXW = 17;          // widest PSF line (16 + MF_MAXW - 1 <= 32)
constexpr int MF_MAXROWS = 64;       // most PSF lines
constexpr int MF_SPITCH = 84;        // row pitch (floats) of the float32 staging tile

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// LDS: the three bfloat16 planes; the float32 staging tile lies inside their last part
// (its rows are smaller than a row of the three planes) and is read into registers in full
// before the planes are written, so a workgroup needs only the planes' LDS.
__host__ __device__ constexpr size_t mfma_lds_bytes(int lines) {
    return (size_t)(MF_T + lines - 1) * (3 * MF_PITCH * 2);
}
constexpr int MF_Q = MF_NX / 4;  // four-column groups per staged row
// staged four-column groups per thread (at most), for a workgroup of NW wavefronts
__host__ __device__ constexpr int mf_maxq(int nw) {
    return ((MF_T + MF_MAXROWS - 1) * MF_Q + nw * 64 - 1) / (nw * 64);
}
static_assert(MF_SPITCH * 4 <= 3 * MF_PITCH * 2, "staging rows must fit in plane rows");

__device__ __forceinline__ void split3(float x, __bf16& p1, __bf16& p2, __bf16& p3) {
    p1 = (__bf16)x;
    const float r1 = x - (float)p1;
    p2 = (__bf16)r1;
    p3 = (__bf16)(r1 - (float)p2);
}

template <int NW, bool PHASE_B>
__global__ __launch_bounds__(NW * 64) void mfma_kernel(LaunchArgs L) {
    static_assert(NW == 4 || NW == 8, "four or eight wavefronts");
    constexpr int BPW = 16 / NW;  // 16 x 16 blocks per wavefront
    constexpr int MAXQ = mf_maxq(NW);
    extern __shared__ float lds_f[];
    __bf16* lds = reinterpret_cast<__bf16*>(lds_f);
    int a0, b0;
    PhaseArgs p;
    if (!resolve<PHASE_B>(L, p, MF_T, MF_T, a0, b0)) return;
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int m = lane & 15, q = lane >> 4;
    const int wr = wv & 3, wc = wv >> 2;  // row group and column group of this wavefront
    const int lines = p.lane_max - p.lane_min + 1;
    const int ny = MF_T + lines - 1;
    const int plane = ny * MF_PITCH;

    // epilogue inputs of this lane's 16 outputs, loaded before the tile so they overlap it
    EpiIn ein[BPW][4];
#pragma unroll
    for (int bx = 0; bx < BPW; ++bx)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int y = a0 + 16 * wr + 4 * q + t, x = b0 + 16 * (BPW * wc + bx) + m;
            if (y < p.H && x < p.W) ein[bx][t] = epi_load<PHASE_B>(p, y, x, (size_t)y * p.W + x);
        }

    const uint8_t own_c = blk_own_load<PHASE_B>(p, a0, b0);

    // source tile: float32 into LDS by DMA (load_tile: every row chunk in flight at once,
    // boundary fold applied to the addresses) at the end of the planes' area, read into
    // registers (four consecutive values per thread and step), then converted into the
    // three bfloat16 planes, which overwrite the staging area
    const int ly0 = a0 + p.lane_min, lx0 = b0 + p.c_min;
    float* stage = reinterpret_cast<float*>(lds + 3 * plane) - ny * MF_SPITCH;
    load_tile(stage, p.src, p.H, p.W, p.bc, ly0, lx0, ny, MF_NX, MF_SPITCH);
    lds_dma_wait();
    __syncthreads();
    float4 xs[MAXQ];
#pragma unroll
    for (int i = 0; i < MAXQ; ++i) {
        const int g = threadIdx.x + i * NW * 64;
        if (g < ny * MF_Q) {
            const int row = g / MF_Q, c4 = 4 * (g - row * MF_Q);
            xs[i] = *reinterpret_cast<const float4*>(stage + row * MF_SPITCH + c4);
        }
    }
    __syncthreads();  // the staging area is read in full before the planes overwrite it
#pragma unroll
    for (int i = 0; i < MAXQ; ++i) {
        const int g = threadIdx.x + i * NW * 64;
        if (g < ny * MF_Q) {
            const int row = g / MF_Q, c4 = 4 * (g - row * MF_Q);
            const float4 x = xs[i];
            __bf16 a[4], b[4], c[4];
            split3(x.x, a[0], b[0], c[0]);
            split3(x.y, a[1], b[1], c[1]);
            split3(x.z, a[2], b[2], c[2]);
            split3(x.w, a[3], b[3], c[3]);
            __bf16* d = lds + row * MF_PITCH + c4;
            __builtin_memcpy(d, a, 8);
            __builtin_memcpy(d + plane, b, 8);
            __builtin_memcpy(d + 2 * plane, c, 8);
        }
    }
    __syncthreads();

    f32x4 even[BPW], odd[BPW], small[BPW];
#pragma unroll
    for (int bx = 0; bx < BPW; ++bx)
        for (int t = 0; t < 4; ++t) even[bx][t] = odd[bx][t] = small[bx][t] = 0.f;
    // weight operands: each line's are loaded one line ahead (the table carries one zero
    // line past its end), so their round trip overlaps the previous line's products
    const bf16x8* tab = reinterpret_cast<const bf16x8*>(p.wts);
    bf16x8 nw1 = tab[lane], nw2 = tab[64 + lane], nw3 = tab[128 + lane];
    const __bf16* base = lds + (16 * wr + m) * MF_PITCH + 8 * q + 16 * BPW * wc;
    // one PSF line: its leading products into acc, the five smaller ones into small
    auto line = [&](int di, f32x4 (&acc)[BPW]) {
        const bf16x8 w1 = nw1, w2 = nw2, w3 = nw3;
        nw1 = tab[(3 * di + 3) * 64 + lane];
        nw2 = tab[(3 * di + 4) * 64 + lane];
        nw3 = tab[(3 * di + 5) * 64 + lane];
        const __bf16* rp = base + di * MF_PITCH;
#pragma unroll
        for (int bx = 0; bx < BPW; ++bx) {
            const bf16x8 x1 = *reinterpret_cast<const bf16x8*>(rp + 16 * bx);
            const bf16x8 x2 = *reinterpret_cast<const bf16x8*>(rp + plane + 16 * bx);
            const bf16x8 x3 = *reinterpret_cast<const bf16x8*>(rp + 2 * plane + 16 * bx);
            acc[bx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, w1, acc[bx], 0, 0, 0);
            f32x4 sm = small[bx];
            sm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, w2, sm, 0, 0, 0);
            sm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x2, w1, sm, 0, 0, 0);
            sm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, w3, sm, 0, 0, 0);
            sm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x2, w2, sm, 0, 0, 0);
            sm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x3, w1, sm, 0, 0, 0);
            small[bx] = sm;
        }
    };
    // even and odd lines in one loop trip, so that each accumulator set keeps its
    // registers (selecting the accumulator per line made the compiler copy all of them
    // between register files on every line)
    int di = 0;
    for (; di + 1 < lines; di += 2) {
        line(di, even);
        line(di + 1, odd);
    }
    if (di < lines) line(di, even);

    int n_active = 0;
    uint64_t fails = 0;
#pragma unroll
    for (int bx = 0; bx < BPW; ++bx)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int y = a0 + 16 * wr + 4 * q + t, x = b0 + 16 * (BPW * wc + bx) + m;
            const float v = (even[bx][t] + odd[bx][t]) + small[bx][t];
            int act = 0;
            if (y < p.H && x < p.W)
                act = epi_apply<PHASE_B>(p, y, x, (size_t)y * p.W + x, ein[bx][t], v, fails);
            if (PHASE_B && p.cnt && !p.blk_lg) n_active += __popcll(__ballot(act));
        }
    thin_finish<PHASE_B>(p, n_active, fails, a0, b0, own_c, a0, b0);
}

// ---------------------------------------------------------------------------------------
// Sliding kernel (generic box filter): every span is a run of equal weights.  Moving the
// output one step along the strip adds the entering tap and removes the leaving tap of each
// run, 2 operations per run per output.  The workgroup's NW wavefronts cover consecutive
// strips of one tile row; only the tile's first output needs the full sum (the seed), and
// its runs are split among the wavefronts.  Each wavefront forms the per-step changes of
// its whole strip (including the step into it), a Kahan-compensated prefix of them, and
// then its start value from the seed parts and the preceding wavefronts' totals, exchanged
// through LDS.  kahan = 0 uses plain float32 sums instead.
// ---------------------------------------------------------------------------------------
// exchange rows 0..3 (seed part, its compensation, strip total, its compensation), then
// the NW zero flags of note_zeros
template <int NW>
__host__ __device__ constexpr int slide_scratch_floats() { return 4 * NW * 64 + NW; }

// First half of a sliding tile: this wavefront's share of the seed (spans i with
// i % NW == wv, in increasing i), the per-step changes d[s] of its strip and their
// compensated prefix (value P, compensation C: true sum = P - C).  The seed share and the
// strip total go to the exchange rows.
template <int ORIENT, int S, int NW>
__device__ __forceinline__ void slide_steps(const PhaseArgs& p, const float* lds,
                                            const TileGeom<ORIENT>& g, float* xs,
                                            float (&P)[S], float (&C)[S]) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    const float* lane_lds = lds + g.lane_part(lane - p.lane_min);
    const int lb = wv * S - p.c_min;   // this wavefront's strip start
    const int lb0 = -p.c_min;          // the tile's first output
    const int st = g.bstep();
    const bool kahan = p.kahan != 0;
    const ConstSpanPtr spans = as_const(p.spans);
    float seed = 0.f, seed_c = 0.f;
    for (int i = wv; i < p.n_spans; i += NW) {
        const DevSpan sp = load_span(spans, i);
        const float* base = lane_lds + g.uni_part(sp.lane_off, lb0 + sp.c0);
        const int len = sp.len;
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
        int q = 0;
        for (; q + 4 <= len; q += 4) {
            p0 += base[q * st];
            p1 += base[(q + 1) * st];
            p2 += base[(q + 2) * st];
            p3 += base[(q + 3) * st];
        }
        for (; q < len; ++q) p0 += base[q * st];
        const float part = (p0 + p1) + (p2 + p3);
        if (kahan) kahan_add(seed, seed_c, sp.w0 * part);
        else seed = fmaf(sp.w0, part, seed);
    }
    // per-step changes d[s] (step into output s of the strip), accumulated over the spans
    // in increasing order; U spans per loop trip so that their LDS reads are in flight
    // together, and the next trip's descriptors are loaded one trip ahead (the span table
    // carries zero descriptors past its end).  The first wavefront's d[0] is not a step
    // (its first output is the seed): it reads an in-tile neighbour instead and is cleared
    // afterwards.
    constexpr int U = S <= 8 ? 2 : 1;
    float d[S];
#pragma unroll
    for (int s = 0; s < S; ++s) d[s] = 0.f;
    const int z0 = wv == 0 ? 1 : 0;
    int i = 0;
    DevSpan nsp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) nsp[u] = load_span(spans, u);
    for (; i + U <= p.n_spans; i += U) {
        DevSpan sp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sp[u] = nsp[u];
            nsp[u] = load_span(spans, i + U + u);
        }
        float din[U][S], dout[U][S];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float* base = lane_lds + g.uni_part(sp[u].lane_off, lb + sp[u].c0);
            const float* bin = base + (sp[u].len - 1) * st;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                din[u][s] = bin[s * st];
                dout[u][s] = base[(s == 0 ? z0 - 1 : s - 1) * st];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < S; ++s) d[s] = fmaf(sp[u].w0, din[u][s] - dout[u][s], d[s]);
    }
    for (; i < p.n_spans; ++i) {
        const DevSpan sp = load_span(spans, i);
        const float* base = lane_lds + g.uni_part(sp.lane_off, lb + sp.c0);
        const float* bin = base + (sp.len - 1) * st;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float vin = bin[s * st], vout = base[(s == 0 ? z0 - 1 : s - 1) * st];
            d[s] = fmaf(sp.w0, vin - vout, d[s]);
        }
    }
    if (z0) d[0] = 0.f;
    {
        float run = 0.f, c = 0.f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (kahan) kahan_add(run, c, d[s]);
            else run += d[s];
            P[s] = run;
            C[s] = c;
        }
    }
    xs[(0 * NW + wv) * 64 + lane] = seed;
    xs[(1 * NW + wv) * 64 + lane] = seed_c;
    xs[(2 * NW + wv) * 64 + lane] = P[S - 1];
    xs[(3 * NW + wv) * 64 + lane] = C[S - 1];
}

// Non-zero inputs in the windows of this wavefront's S outputs: the first window counted
// directly, then the changes of each step (entering minus leaving inputs of every span).
// Only wavefronts that may hold an all-zero window run it.
template <int ORIENT, int S>
__device__ __forceinline__ void slide_counts(const PhaseArgs& p, const float* lds,
                                             const TileGeom<ORIENT>& g, int (&n)[S]) {
    const int lane = threadIdx.x & 63, wv = wave_id();
    const float* lane_lds = lds + g.lane_part(lane - p.lane_min);
    const int lb = wv * S - p.c_min;
    const int st = g.bstep();
    const ConstSpanPtr spans = as_const(p.spans);
#pragma unroll
    for (int s = 0; s < S; ++s) n[s] = 0;
#pragma unroll 1
    for (int i = 0; i < p.n_spans; ++i) {
        const DevSpan sp = load_span(spans, i);
        const float* base = lane_lds + g.uni_part(sp.lane_off, lb + sp.c0);
#pragma unroll 1
        for (int q = 0; q < sp.len; ++q) n[0] += nz(base[q * st]);
        const float* bin = base + (sp.len - 1) * st;
#pragma unroll
        for (int s = 1; s < S; ++s) n[s] += nz(bin[s * st]) - nz(base[(s - 1) * st]);
    }
#pragma unroll
    for (int s = 1; s < S; ++s) n[s] += n[s - 1];
}

template <int ORIENT, int S, int NW, bool PHASE_B>
__device__ __forceinline__ void slide_tile(const PhaseArgs& p, int a0, int b0, float* lds) {
    constexpr int TA = 64, TB = NW * S;
    TileGeom<ORIENT> g = make_geom<ORIENT>(p, a0, b0, TA, TB, 0);
    EpiPlan<ORIENT, S, NW> plan;
    epi_prefetch<ORIENT, S, NW, PHASE_B>(p, a0, b0, plan);
    load_tile(lds, p.src, p.H, p.W, p.bc, g.ly0, g.lx0, g.ny, g.nx, g.pitch);
    lds_dma_wait();
    const int lane = threadIdx.x & 63, wv = wave_id();
    float* xs = lds + g.ny * g.pitch;
    int* zf = reinterpret_cast<int*>(xs + 4 * NW * 64);
    // Exact zeros: does this wavefront need the non-zero counts?  With a span at least S
    // long (p.wit), its columns S - 1 .. len - 1 lie in all S windows of a lane's strip: a
    // non-zero input among four of them proves that none of the lane's windows is
    // all-zero, so the counts are kept only if some lane of the wavefront finds none (an
    // all-zero region, or zeros at all four places).  Without such a span, they are kept
    // in tiles that hold a zero.  Counting wavefronts count their first window directly,
    // so the decision need not be the same for the whole workgroup.
    if (p.wit < 0) note_zeros(lds, g.ny, g.nx, g.pitch, zf);
    __syncthreads();
    bool cnt;
    if (p.wit >= 0) {
        const DevSpan sw = load_span(as_const(p.spans), p.wit);
        const float* wb = lds + g.lane_part(lane - p.lane_min) +
                          g.uni_part(sw.lane_off, wv * S - p.c_min + sw.c0);
        const int st = g.bstep(), spread = sw.len - S;
        float m = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) m = fmaxf(m, fabsf(wb[(S - 1 + (spread * t) / 3) * st]));
        cnt = __ballot(!(m > 0.f)) != 0ull;
    } else {
        cnt = tile_zeros<NW>(zf);
    }
    float P[S], C[S];
    slide_steps<ORIENT, S, NW>(p, lds, g, xs, P, C);
    __syncthreads();
    // start value: the seed parts, then the strip totals of the preceding wavefronts
    const bool kahan = p.kahan != 0;
    float base = 0.f, bc = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const float part = xs[(0 * NW + w) * 64 + lane] - xs[(1 * NW + w) * 64 + lane];
        if (kahan) kahan_add(base, bc, part);
        else base += part;
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wv) {
            const float part = xs[(2 * NW + w) * 64 + lane] - xs[(3 * NW + w) * 64 + lane];
            if (kahan) kahan_add(base, bc, part);
            else base += part;
        }
    }
    const float b_true = base - bc;
    float out[S];
#pragma unroll
    for (int s = 0; s < S; ++s) out[s] = b_true + (P[s] - C[s]);
    if (cnt) {  // the tile is intact until write_outputs' first barrier
        int n[S];
        slide_counts<ORIENT, S>(p, lds, g, n);
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (n[s] == 0) out[s] = 0.f;
    }
    write_outputs<ORIENT, S, NW, PHASE_B>(p, lds, a0, b0, out, plan);
}

template <int ORIENT, int S, int NW, bool PHASE_B>
__global__ __launch_bounds__(NW * 64) void slide_kernel(LaunchArgs L) {
    extern __shared__ float lds[];
    int a0, b0;
    PhaseArgs p;
    if (!resolve<PHASE_B>(L, p, 64, NW * S, a0, b0)) return;
    slide_tile<ORIENT, S, NW, PHASE_B>(p, a0, b0, lds);
}

// ---------------------------------------------------------------------------------------
// Rectangle kernel (2-D box filter, separable): the operator is w times the sum over a
// kh x kw window, rows lane_min..lane_max and columns c_min..c_max relative to the output
// (ORIENT_ROWS tables).  On the LDS tile (64 + kh - 1 rows by TB + kw - 1 columns) a
// horizontal pass forms the kw-wide window sums of every tile row for the TB output
// columns (segments of 8 by sliding: one add and one subtract per step), then a vertical
// pass slides kh-tall sums of those down segments of 8 output rows.  Seeds are direct sums
// over four partial accumulators; the slides are Kahan-compensated when kahan = 1.  Work
// per output is constant in kh and kw apart from the seeds.
// ---------------------------------------------------------------------------------------
constexpr int RECT_SEG = 8;

template <int NW>
__host__ __device__ constexpr int rect_hs_pitch(int TB) { return TB + 1; }

__device__ __forceinline__ void rl_add(float& s, float& c, float x, bool kahan) {
    if (kahan) kahan_add(s, c, x);
    else s += x;
}

// LDS after the tile: ny rows of TB horizontal window sums (pitch TB + 1), then the NW
// zero flags of note_zeros.
template <int NW>
__host__ __device__ constexpr size_t rect_lds_floats(int ny, int nx, int TB) {
    return (size_t)ny * (nx | 1) + (size_t)ny * rect_hs_pitch<NW>(TB) + NW;
}

// Whether a rectangle tile needs the exact non-zero counts (see rect_tile).  For kh < 8
// the flags were published by note_zeros before the first barrier; otherwise every
// vertical task checks its witness inputs here, with one more barrier.
template <int NW>
__device__ __forceinline__ bool rect_need_counts(const float* lds, int pitch, int kh, int kw,
                                                 int vr, int vb, bool has_v, int* zf) {
    if (kh >= RECT_SEG) {
        bool bad = false;
        if (has_v) {
            float m = 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = vr * RECT_SEG + RECT_SEG - 1 + ((kh - RECT_SEG) * t) / 3;
                const int c = vb + ((kw - 1) * t) / 3;
                m = fmaxf(m, fabsf(lds[r * pitch + c]));
            }
            bad = !(m > 0.f);
        }
        const bool any = __ballot(bad) != 0ull;
        if ((threadIdx.x & 63) == 0) zf[wave_id()] = any ? 1 : 0;
        __syncthreads();
    }
    return tile_zeros<NW>(zf);
}

template <int S, int NW, bool PHASE_B>
__device__ __forceinline__ void rect_tile(const PhaseArgs& p, int a0, int b0, float* lds) {
    constexpr int TB = NW * S;
    constexpr int NSEG_H = TB / RECT_SEG;       // horizontal segments per tile row
    constexpr int NV = TB * (64 / RECT_SEG);    // vertical tasks (column, row segment)
    static_assert(NV <= NW * 64, "one vertical task per thread");
    const int kh = p.lane_max - p.lane_min + 1, kw = p.c_max - p.c_min + 1;
    const int ny = 64 + kh - 1, nx = TB + kw - 1, pitch = nx | 1;
    const int hp = rect_hs_pitch<NW>(TB);
    float* hs = lds + ny * pitch;  // ny rows of TB horizontal sums
    const int tid = threadIdx.x;
    const bool kahan = p.kahan != 0;
    // vertical task of this thread and its outputs' epilogue inputs (loaded up front)
    const int vb = tid % TB, vr = tid / TB;
    const bool has_v = tid < NV;
    EpiIn in[RECT_SEG];
    const uint8_t own_c = blk_own_load<PHASE_B>(p, a0, b0);
    if (has_v) {
#pragma unroll
        for (int j = 0; j < RECT_SEG; ++j) {
            const int y = a0 + vr * RECT_SEG + j, x = b0 + vb;
            if (y < p.H && x < p.W) in[j] = epi_load<PHASE_B>(p, y, x, (size_t)y * p.W + x);
        }
    }
    load_tile(lds, p.src, p.H, p.W, p.bc, a0 + p.lane_min, b0 + p.c_min, ny, nx, pitch);
    lds_dma_wait();
    int* zf = reinterpret_cast<int*>(lds + rect_lds_floats<NW>(ny, nx, TB) - NW);
    if (kh < RECT_SEG) note_zeros(lds, ny, nx, pitch, zf);
    __syncthreads();
    // horizontal pass
    for (int task = tid; task < ny * NSEG_H; task += NW * 64) {
        const int r = task / NSEG_H, c0 = (task % NSEG_H) * RECT_SEG;
        const float* row = lds + r * pitch + c0;
        float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
        int t = 0;
        for (; t + 4 <= kw; t += 4) {
            q0 += row[t];
            q1 += row[t + 1];
            q2 += row[t + 2];
            q3 += row[t + 3];
        }
        for (; t < kw; ++t) q0 += row[t];
        float sum = (q0 + q1) + (q2 + q3), comp = 0.f;
        float* out = hs + r * hp + c0;
        out[0] = sum;
#pragma unroll
        for (int j = 1; j < RECT_SEG; ++j) {
            rl_add(sum, comp, row[j + kw - 1] - row[j - 1], kahan);
            out[j] = sum - comp;
        }
    }
    __syncthreads();
    // vertical pass
    float v[RECT_SEG];
    if (has_v) {
        const float* col = hs + (vr * RECT_SEG) * hp + vb;
        float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
        int i = 0;
        for (; i + 4 <= kh; i += 4) {
            q0 += col[i * hp];
            q1 += col[(i + 1) * hp];
            q2 += col[(i + 2) * hp];
            q3 += col[(i + 3) * hp];
        }
        for (; i < kh; ++i) q0 += col[i * hp];
        float sum = (q0 + q1) + (q2 + q3), comp = 0.f;
        v[0] = sum;
#pragma unroll
        for (int j = 1; j < RECT_SEG; ++j) {
            rl_add(sum, comp, col[(j + kh - 1) * hp] - col[(j - 1) * hp], kahan);
            v[j] = sum - comp;
        }
    }
    // Exact zeros: the same two passes over non-zero counts (the horizontal ones in place
    // of the sums), windows with none give exactly 0.  They run only where an all-zero
    // window is possible: with kh >= 8, tile rows 8 vr + 7 .. 8 vr + kh - 1 lie in all
    // 8 windows of a vertical task, and a non-zero input among four of them (on the
    // task's columns) proves that none of its windows is all-zero; with kh < 8, in tiles
    // that hold a zero.  The decision is the same for the whole workgroup.
    const bool cnt = rect_need_counts<NW>(lds, pitch, kh, kw, vr, vb, has_v, zf);
    if (cnt) {
        int* hn = reinterpret_cast<int*>(hs);
        __syncthreads();  // everyone is done reading the sums
        for (int task = tid; task < ny * NSEG_H; task += NW * 64) {
            const int r = task / NSEG_H, c0 = (task % NSEG_H) * RECT_SEG;
            const float* row = lds + r * pitch + c0;
            int n = 0;
#pragma unroll 1
            for (int t = 0; t < kw; ++t) n += nz(row[t]);
            int* outn = hn + r * hp + c0;
            outn[0] = n;
#pragma unroll
            for (int j = 1; j < RECT_SEG; ++j) {
                n += nz(row[j + kw - 1]) - nz(row[j - 1]);
                outn[j] = n;
            }
        }
        __syncthreads();
        if (has_v) {
            const int* coln = hn + (vr * RECT_SEG) * hp + vb;
            int n = 0;
#pragma unroll 1
            for (int i = 0; i < kh; ++i) n += coln[i * hp];
            if (n == 0) v[0] = 0.f;
#pragma unroll
            for (int j = 1; j < RECT_SEG; ++j) {
                n += coln[(j + kh - 1) * hp] - coln[(j - 1) * hp];
                if (n == 0) v[j] = 0.f;
            }
        }
    }
    // epilogue
    int n_active = 0;
    uint64_t fails = 0;
    const float w = as_const(p.spans)[0].w0;
#pragma unroll
    for (int j = 0; j < RECT_SEG; ++j) {
        int act = 0;
        const int y = a0 + vr * RECT_SEG + j, x = b0 + vb;
        if (has_v && y < p.H && x < p.W)
            act = epi_apply<PHASE_B>(p, y, x, (size_t)y * p.W + x, in[j], w * v[j], fails);
        if (PHASE_B && p.cnt && !p.blk_lg) n_active += __popcll(__ballot(act));
    }
    thin_finish<PHASE_B>(p, n_active, fails, a0, b0, own_c, a0, b0);
}

template <int S, int NW, bool PHASE_B>
__global__ __launch_bounds__(NW * 64) void rect_kernel(LaunchArgs L) {
    extern __shared__ float lds[];
    int a0, b0;
    PhaseArgs p;
    if (!resolve<PHASE_B>(L, p, 64, NW * S, a0, b0)) return;
    rect_tile<S, NW, PHASE_B>(p, a0, b0, lds);
}

// ---------------------------------------------------------------------------------------
// Summed-area-table kernel (2-D box filter from 2-D cumulated sums): the same operator as
// the rectangle kernel, evaluated as in the paper's cumulated-sum variant -- every window
// sum is T(a+kh, b+kw) - T(a, b+kw) - T(a+kh, b) + T(a, b) of the table T of cumulated sums
// -- but with T built per tile in LDS instead of over the whole image: the tile's rows are
// prefix-summed (one thread per row), then its columns (one thread per column).  T is held
// in FP64: its entries grow with the tile's total, and a float32 table would lose the small
// windows to cancellation.  Exact zeros (tiles holding a zero only): after the FP64 row
// pass, a count pass overwrites each tile value with the running count of non-zero values
// of its row (the values are not needed any more), a column pass turns those into 2-D
// counts, and windows with a zero count give exactly 0.  Work per output is constant in kh
// and kw: four corner reads and three FP64 adds.
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int sat_pitch(int nx) { return (nx + 1) | 1; }

// LDS layout in bytes: float tile (ny x pitch; count table in place), FP64 table
// ((ny + 1) x sat_pitch) at an 8-byte boundary, then the NW zero flags of note_zeros.
__host__ __device__ constexpr size_t sat_table_offset(int ny, int nx) {
    return (((size_t)ny * (nx | 1) * 4 + 7) / 8) * 8;
}
template <int NW>
__host__ __device__ constexpr size_t sat_lds_bytes(int ny, int nx) {
    return sat_table_offset(ny, nx) + (size_t)(ny + 1) * sat_pitch(nx) * 8 + NW * 4;
}

template <int S, int NW, bool PHASE_B>
__device__ __forceinline__ void sat_tile(const PhaseArgs& p, int a0, int b0, float* lds) {
    constexpr int TB = NW * S;
    constexpr int NV = TB * (64 / RECT_SEG);
    static_assert(NV <= NW * 64, "one output task per thread");
    const int kh = p.lane_max - p.lane_min + 1, kw = p.c_max - p.c_min + 1;
    const int ny = 64 + kh - 1, nx = TB + kw - 1, pitch = nx | 1, tp = sat_pitch(nx);
    double* T = reinterpret_cast<double*>(reinterpret_cast<char*>(lds) + sat_table_offset(ny, nx));
    int* N = reinterpret_cast<int*>(lds);  // inclusive counts, in place of the tile
    const int tid = threadIdx.x;
    const int vb = tid % TB, vr = tid / TB;
    const bool has_v = tid < NV;
    EpiIn in[RECT_SEG];
    const uint8_t own_c = blk_own_load<PHASE_B>(p, a0, b0);
    if (has_v) {
#pragma unroll
        for (int j = 0; j < RECT_SEG; ++j) {
            const int y = a0 + vr * RECT_SEG + j, x = b0 + vb;
            if (y < p.H && x < p.W) in[j] = epi_load<PHASE_B>(p, y, x, (size_t)y * p.W + x);
        }
    }
    load_tile(lds, p.src, p.H, p.W, p.bc, a0 + p.lane_min, b0 + p.c_min, ny, nx, pitch);
    lds_dma_wait();
    int* zf = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + sat_lds_bytes<NW>(ny, nx)) - NW;
    if (kh < RECT_SEG) note_zeros(lds, ny, nx, pitch, zf);
    __syncthreads();
    // row 0 of T is 0; each row's prefix starts at column 0 = 0
    for (int j = tid; j <= nx; j += NW * 64) T[j] = 0.0;
    // row prefix sums: T(i + 1, j + 1) = sum of tile row i, columns 0..j
    for (int i = tid; i < ny; i += NW * 64) {
        const float* row = lds + i * pitch;
        double* trow = T + (size_t)(i + 1) * tp;
        double s = 0.0;
        trow[0] = 0.0;
        int j = 0;
        for (; j + 4 <= nx; j += 4) {
            const float v0 = row[j], v1 = row[j + 1], v2 = row[j + 2], v3 = row[j + 3];
            s += (double)v0;
            trow[j + 1] = s;
            s += (double)v1;
            trow[j + 2] = s;
            s += (double)v2;
            trow[j + 3] = s;
            s += (double)v3;
            trow[j + 4] = s;
        }
        for (; j < nx; ++j) {
            s += (double)row[j];
            trow[j + 1] = s;
        }
    }
    __syncthreads();
    // column prefix sums: T(i, j) becomes the sum over tile rows < i and columns < j
    for (int j = 1 + tid; j <= nx; j += NW * 64) {
        double s = 0.0;
        int i = 1;
        for (; i + 4 <= ny + 1; i += 4) {
            const double t0 = T[(size_t)i * tp + j], t1 = T[(size_t)(i + 1) * tp + j];
            const double t2 = T[(size_t)(i + 2) * tp + j], t3 = T[(size_t)(i + 3) * tp + j];
            s += t0;
            T[(size_t)i * tp + j] = s;
            s += t1;
            T[(size_t)(i + 1) * tp + j] = s;
            s += t2;
            T[(size_t)(i + 2) * tp + j] = s;
            s += t3;
            T[(size_t)(i + 3) * tp + j] = s;
        }
        for (; i <= ny; ++i) {
            s += T[(size_t)i * tp + j];
            T[(size_t)i * tp + j] = s;
        }
    }
    // exact zeros: decided as in the rectangle kernel (witness inputs or the tile scan)
    const bool cnt = rect_need_counts<NW>(lds, pitch, kh, kw, vr, vb, has_v, zf);
    if (cnt) {
        // row prefixes of the non-zero counts, each overwriting its own tile row (the
        // values are not needed any more): N(i, j) counts row i, columns 0..j
        for (int i = tid; i < ny; i += NW * 64) {
            float* row = lds + i * pitch;
            int n = 0;
#pragma unroll 1
            for (int j = 0; j < nx; ++j) {
                n += nz(row[j]);
                reinterpret_cast<int*>(row)[j] = n;
            }
        }
        __syncthreads();
        // column prefixes: N(i, j) counts rows 0..i, columns 0..j
        for (int j = tid; j < nx; j += NW * 64) {
            int n = 0;
#pragma unroll 1
            for (int r = 0; r < ny; ++r) {
                n += N[r * pitch + j];
                N[r * pitch + j] = n;
            }
        }
    }
    __syncthreads();
    // outputs from four corners: thread task (column vb, rows vr*8 .. vr*8+7)
    const float w = as_const(p.spans)[0].w0;
    auto cnt_at = [&](int i, int j) { return (i < 0 || j < 0) ? 0 : N[i * pitch + j]; };
    int n_active = 0;
    uint64_t fails = 0;
#pragma unroll
    for (int j = 0; j < RECT_SEG; ++j) {
        int act = 0;
        const int a = vr * RECT_SEG + j;
        const int y = a0 + a, x = b0 + vb;
        if (has_v && y < p.H && x < p.W) {
            const size_t r0 = (size_t)a * tp, r1 = (size_t)(a + kh) * tp;
            const double sum = (T[r1 + vb + kw] - T[r0 + vb + kw]) - (T[r1 + vb] - T[r0 + vb]);
            float v = (float)sum;
            if (cnt) {
                const int n = (cnt_at(a + kh - 1, vb + kw - 1) - cnt_at(a - 1, vb + kw - 1)) -
                              (cnt_at(a + kh - 1, vb - 1) - cnt_at(a - 1, vb - 1));
                if (n == 0) v = 0.f;
            }
            act = epi_apply<PHASE_B>(p, y, x, (size_t)y * p.W + x, in[j], w * v, fails);
        }
        if (PHASE_B && p.cnt && !p.blk_lg) n_active += __popcll(__ballot(act));
    }
    thin_finish<PHASE_B>(p, n_active, fails, a0, b0, own_c, a0, b0);
}

template <int S, int NW, bool PHASE_B>
__global__ __launch_bounds__(NW * 64) void sat_kernel(LaunchArgs L) {
    extern __shared__ float lds[];
    int a0, b0;
    PhaseArgs p;
    if (!resolve<PHASE_B>(L, p, 64, NW * S, a0, b0)) return;
    sat_tile<S, NW, PHASE_B>(p, a0, b0, lds);
}

// ---------------------------------------------------------------------------------------
// Persistent schedule (plain RL): one launch runs every phase of every iteration of one or
// more jobs.  A task is (step s, tile t) with step s = 2 (k - k0) + phase; tasks are
// numbered step by step (q = s * total_tiles + tile index) and handed out in that order by
// an atomic ticket, so a workgroup only ever waits for tasks with smaller numbers, which
// running workgroups hold or have finished: the schedule cannot deadlock, whatever the
// number of resident workgroups.  Task (s, t) waits until every tile within the phase
// halo's reach has finished step s - 1 (done[t'] >= s): that covers the data it reads
// (u^k from phase B, or r from phase A) and the data it overwrites (which those tiles read
// in step s - 1).  Completion: every wavefront waits for its stores, the workgroup
// synchronises, and wavefront 0 publishes done[t] = s + 1 after an agent-scope release
// (the XCDs have separate L2 caches); the waiting side polls with relaxed agent-scope
// loads and then takes an agent-scope acquire before reading.
//
// Wavefront 0 as a whole takes the ticket, waits and publishes, under a condition that is
// uniform per wavefront (wave_id() goes through readfirstlane), and its lanes write
// identical values; only the ticket's atomic add runs on a single lane, inside a short
// branch that rejoins before anything else.  No lane-divergent region may span the loop's
// back edge: if lane 0 alone published and took the next ticket, the compiler may lay the
// loop out so that lanes 1..63 of wavefront 0 return to the barrier without lane 0, and
// the workgroup then re-reads the previous task from LDS and repeats that tile without
// end.  Waits are bounded: past spin_limit polls the launch raises *abort and every
// workgroup leaves; each pass of the loop takes a new ticket or leaves, so the loop runs
// at most total + 1 passes and the kernel always ends.
// ---------------------------------------------------------------------------------------
struct PersistJob {
    PhaseArgs a, b;        // phase A / phase B records (k = iteration index at launch)
    int32_t* done;         // per tile: steps finished in this launch (zero at launch)
    int32_t n_steps;       // 2 x iterations of this job in this launch
    int32_t reach_a, reach_b;  // tiles within the halo reach on each axis
    int32_t pad;
};

struct PersistArgs {
    const PersistJob* jobs;   // n_jobs entries (device); unused when n_jobs == 1
    const int32_t* prefix;    // tile prefix over jobs (n_jobs + 1)
    int32_t n_jobs, total_tiles, max_steps, spin_limit;
    int32_t* ticket;          // zero at launch
    int32_t* abort;           // zero at launch; set when a wait exceeded spin_limit
    PersistJob one;           // the job itself when n_jobs == 1
};

typedef const __attribute__((address_space(4))) PersistJob* ConstPersistPtr;

__device__ __forceinline__ PersistJob load_persist(ConstPersistPtr t) {
    PersistJob j;
    j.a = load_args((ConstArgsPtr)&t->a);
    j.b = load_args((ConstArgsPtr)&t->b);
    j.done = t->done;
    j.n_steps = t->n_steps;
    j.reach_a = t->reach_a;
    j.reach_b = t->reach_b;
    j.pad = 0;
    return j;
}

__device__ __forceinline__ int poll_done(int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront 0, all lanes: wait until every tile in the reach of tile t has finished step
// s - 1.  Lane l checks the tiles l, l + 64, ... of the reach rectangle; the wavefront
// decides together (ballot), so the result and the loop are wavefront-uniform.  Returns
// false if the launch is being aborted.
__device__ __forceinline__ bool wait_deps(const PersistJob& J, int t, int s, int spin_limit,
                                          int32_t* abort) {
    if (s == 0) return true;
    const int lane = threadIdx.x & 63;
    const int ta_n = J.a.tiles_a, tb_n = J.a.tiles_b;
    const int ta = t % ta_n, tb = t / ta_n;
    const int a_lo = max(0, ta - J.reach_a), a_hi = min(ta_n - 1, ta + J.reach_a);
    const int b_lo = max(0, tb - J.reach_b), b_hi = min(tb_n - 1, tb + J.reach_b);
    const int na = a_hi - a_lo + 1, nd = na * (b_hi - b_lo + 1);
    for (int spins = 0;; ++spins) {
        // spin_limit < 0 (a host-set test condition) gives up at the first poll
        bool ready = spin_limit >= 0;
        for (int d = lane; d < nd; d += 64) {
            const int y = b_lo + d / na, x = a_lo + d % na;
            if (poll_done(J.done + y * ta_n + x) < s) ready = false;
        }
        if (__ballot(!ready) == 0ull) return true;
        if (spins >= spin_limit) {
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((spins & 1023) == 1023 &&
            __builtin_amdgcn_readfirstlane(poll_done(abort)) != 0)
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

template <int KIND, int ORIENT, int S, int LMAX, int NW>
__global__ __launch_bounds__(NW * 64) void persist_kernel(PersistArgs P) {
    extern __shared__ float lds[];
    __shared__ int32_t task[3];  // job, tile, step (job -1: leave, -2: nothing to do)
    constexpr int TA = 64, TB = NW * S;
    const int64_t total = (int64_t)P.max_steps * P.total_tiles;
    const bool lead = wave_id() == 0;  // wavefront-uniform
    for (int64_t pass = 0; pass <= total; ++pass) {
        if (lead) {
            int q = 0;
            if ((threadIdx.x & 63) == 0) q = atomicAdd(P.ticket, 1);
            q = __builtin_amdgcn_readfirstlane(q);
            int jn = -1, t = 0, st = 0;
            if (q < total && __builtin_amdgcn_readfirstlane(poll_done(P.abort)) == 0) {
                st = q / P.total_tiles;
                const int idx = q - st * P.total_tiles;
                int lo = 0;
                if (P.n_jobs > 1) {
                    const ConstIntPtr pre = (ConstIntPtr)P.prefix;
                    int hi = P.n_jobs - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (pre[mid] <= idx) lo = mid;
                        else hi = mid - 1;
                    }
                    t = idx - pre[lo];
                } else {
                    t = idx;
                }
                jn = lo;
                const PersistJob J = P.n_jobs > 1 ? load_persist((ConstPersistPtr)P.jobs + lo) : P.one;
                if (st >= J.n_steps) {
                    jn = -2;  // this job has no step st: nothing to do
                } else if (!wait_deps(J, t, st, P.spin_limit, P.abort)) {
                    jn = -1;
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            task[0] = jn;  // every lane of wavefront 0 writes the same values
            task[1] = t;
            task[2] = st;
        }
        __syncthreads();
        const int jn = task[0], t = task[1], st = task[2];
        __syncthreads();  // task[] is rewritten at the next pass
        if (jn == -1) break;
        if (jn == -2) continue;
        const PersistJob J = P.n_jobs > 1 ? load_persist((ConstPersistPtr)P.jobs + jn) : P.one;
        const bool phase_b = (st & 1) != 0;
        PhaseArgs p = phase_b ? J.b : J.a;
        p.k += st >> 1;
        p.full = 1;
        const int a0 = (t % p.tiles_a) * TA, b0 = (t / p.tiles_a) * TB;
        if (KIND == 0) {
            if (phase_b) span_tile<ORIENT, S, LMAX, NW, true>(p, a0, b0, lds);
            else span_tile<ORIENT, S, LMAX, NW, false>(p, a0, b0, lds);
        } else {
            if (phase_b) slide_tile<ORIENT, S, NW, true>(p, a0, b0, lds);
            else slide_tile<ORIENT, S, NW, false>(p, a0, b0, lds);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wavefront's stores have reached L2
        __syncthreads();                // every wavefront's have; LDS is free again
        if (lead) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // visible to every XCD
            __hip_atomic_store(J.done + t, st + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Fused iteration kernel: conv -> ratio -> corr -> update in one launch (ORIENT_ROWS,
// lanes are image rows).  A workgroup owns a 64 x (NW*S) output tile.  It loads u^k for the
// tile plus both halos (conv halo around the corr halo) into LDS, forms r = f / (u^k * h)
// for the tile plus the corr halo into a second LDS tile, copies the boundary continuation
// into the out-of-image part of that r tile, then correlates and writes
// u^{k+1} = u^k . (h^* * r) into the other u plane (neighbouring workgroups still read
// u^k).  Tiles at the bottom/right edge are shifted inwards so that every tile lies inside
// the image; the folded positions its r halo needs are then inside its own r tile (needs
// H >= 64, W >= NW*S and halos <= 63).  Overlapping tiles compute identical values.
// ---------------------------------------------------------------------------------------
struct FusedArgs {
    int32_t H, W, bc, kahan;
    const float* f;
    float* u0;            // u^k for even k, u^{k+1} for odd k
    float* u1;            // the other plane
    const DevSpan* cspans;  // conv table (forward, mirrored taps)
    const float* cwts;
    const DevSpan* rspans;  // corr table (adjoint)
    const float* rwts;
    int32_t n_cspans, n_rspans;
    int32_t vl_min, vl_max, vc_min, vc_max;  // conv extents (lane, strip)
    int32_t cl_min, cl_max, cc_min, cc_max;  // corr extents
    int32_t tiles_a, tiles_b;
    int64_t k;
};

typedef const __attribute__((address_space(4))) FusedArgs* ConstFusedPtr;

__device__ __forceinline__ FusedArgs load_fused(ConstFusedPtr t) {
    FusedArgs a;
    a.H = t->H; a.W = t->W; a.bc = t->bc; a.kahan = t->kahan;
    a.f = t->f; a.u0 = t->u0; a.u1 = t->u1;
    a.cspans = t->cspans; a.cwts = t->cwts; a.rspans = t->rspans; a.rwts = t->rwts;
    a.n_cspans = t->n_cspans; a.n_rspans = t->n_rspans;
    a.vl_min = t->vl_min; a.vl_max = t->vl_max; a.vc_min = t->vc_min; a.vc_max = t->vc_max;
    a.cl_min = t->cl_min; a.cl_max = t->cl_max; a.cc_min = t->cc_min; a.cc_max = t->cc_max;
    a.tiles_a = t->tiles_a; a.tiles_b = t->tiles_b; a.k = t->k;
    return a;
}

// S outputs of one strip: out[s] = sum over the table of w * src(a + lane_off, b + s + c0),
// src an LDS tile of the given pitch, (a, b) already relative to the tile origin.
template <int S, int LMAX>
__device__ __forceinline__ void strip_sum(const float* src, int pitch, int a, int b,
                                          ConstSpanPtr spans, ConstFloatPtr wts, int n,
                                          bool cascade, float (&out)[S]) {
    TileGeom<ORIENT_ROWS> g;
    g.pitch = pitch;
    float acc1[S], part[S];
#pragma unroll
    for (int s = 0; s < S; ++s) { out[s] = 0.f; acc1[s] = 0.f; part[s] = 0.f; }
    bool odd = false;
    for (int i = 0; i < n; ++i) {
        const DevSpan sp = load_span(spans, i);
        const ConstFloatPtr wp = wts + sp.woff;
        const float* base = src + g.idx(a + sp.lane_off, b + sp.c0);
        switch (sp.len) {
#define RL_PIECE(m) \
    case m:         \
        if (m <= LMAX) span_piece<ORIENT_ROWS, S, (m <= LMAX ? m : 1)>(base, g, wp, part); \
        break;
            RL_PIECE(1) RL_PIECE(2) RL_PIECE(3) RL_PIECE(4) RL_PIECE(5) RL_PIECE(6)
            RL_PIECE(7) RL_PIECE(8) RL_PIECE(9) RL_PIECE(10) RL_PIECE(11) RL_PIECE(12)
            RL_PIECE(13) RL_PIECE(14) RL_PIECE(15) RL_PIECE(16)
#undef RL_PIECE
            default: break;
        }
        if (sp.row_end) {
            if (cascade && odd) {
#pragma unroll
                for (int s = 0; s < S; ++s) { acc1[s] += part[s]; part[s] = 0.f; }
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s) { out[s] += part[s]; part[s] = 0.f; }
            }
            odd = !odd;
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) out[s] += acc1[s];
}

template <int S, int LMAX, int NW>
__global__ __launch_bounds__(NW * 64) void fused_kernel(const FusedArgs* table, int64_t kb) {
    extern __shared__ float lds[];
    constexpr int TA = 64, TB = NW * S;
    const FusedArgs p = load_fused((ConstFusedPtr)table);
    const int64_t k = p.k + kb;
    const float* u_in = (k & 1) ? p.u1 : p.u0;
    float* u_out = (k & 1) ? p.u0 : p.u1;
    const int nt = p.tiles_a * p.tiles_b;
    if ((int)blockIdx.x >= nt) return;
    const int t = xcd_tile(blockIdx.x, nt);
    const int a0 = min((t % p.tiles_a) * TA, p.H - TA);
    const int b0 = min((t / p.tiles_a) * TB, p.W - TB);
    // r region (tile + corr halo), u region (r region + conv halo), relative origins
    const int RA = TA + p.cl_max - p.cl_min, RB = TB + p.cc_max - p.cc_min;
    const int ra0 = a0 + p.cl_min, rb0 = b0 + p.cc_min;
    const int UA = RA + p.vl_max - p.vl_min, UB = RB + p.vc_max - p.vc_min;
    const int ua0 = ra0 + p.vl_min, ub0 = rb0 + p.vc_min;
    const int upitch = UB | 1, rpitch = RB | 1;
    float* ut = lds;
    float* rt = lds + UA * upitch;
    load_tile(ut, u_in, p.H, p.W, p.bc, ua0, ub0, UA, UB, upitch);
    lds_dma_wait();
    __syncthreads();

    const int lane = threadIdx.x & 63, wv = wave_id();
    const bool cascade = p.kahan != 0;
    const ConstSpanPtr cs = as_const(p.cspans), rs = as_const(p.rspans);
    const ConstFloatPtr cw = as_const(p.cwts), rw = as_const(p.rwts);
    // 1. r = f / (u*h) on the in-image part of the r region
    const int blocks = (RA + 63) >> 6, strips = (RB + S - 1) / S;
    for (int it = wv; it < blocks * strips; it += NW) {
        const int blk = it / strips, st = it - blk * strips;
        const int ra = blk * 64 + lane, rb = st * S;  // r-tile coordinates
        const int y = ra0 + ra;
        float fv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int x = rb0 + rb + s;
            fv[s] = (ra < RA && rb + s < RB && y >= 0 && y < p.H && x >= 0 && x < p.W)
                        ? p.f[(size_t)y * p.W + x] : 0.f;
        }
        if (ra < RA) {
            float v[S];
            // u-tile coordinates of r position (ra, rb): (ra - vl_min, rb - vc_min)
            strip_sum<S, LMAX>(ut, upitch, ra - p.vl_min, rb - p.vc_min, cs, cw, p.n_cspans,
                               cascade, v);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int x = rb0 + rb + s;
                if (rb + s < RB && y >= 0 && y < p.H && x >= 0 && x < p.W)
                    rt[ra * rpitch + rb + s] = rl_ratio(fv[s], v[s]);
            }
        }
    }
    __syncthreads();
    // 2. out-of-image r positions take the value of their folded in-image position
    for (int e = threadIdx.x; e < RA * RB; e += NW * 64) {
        const int ra = e / RB, rb = e - ra * RB;
        const int y = ra0 + ra, x = rb0 + rb;
        if (y >= 0 && y < p.H && x >= 0 && x < p.W) continue;
        const int fy = fold_idx(y, p.H, p.bc) - ra0, fx = fold_idx(x, p.W, p.bc) - rb0;
        rt[ra * rpitch + rb] = rt[fy * rpitch + fx];
    }
    __syncthreads();
    // 3. c = h^* * r on the output tile; u^{k+1} = u^k . c
    float c[S];
    // r-tile coordinates of output (lane, wv*S): (lane - cl_min, wv*S - cc_min)
    strip_sum<S, LMAX>(rt, rpitch, lane - p.cl_min, wv * S - p.cc_min, rs, rw, p.n_rspans,
                       cascade, c);
    float un[S];
    const int uy = lane - p.cl_min - p.vl_min;            // u-tile row of this output row
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int ux = wv * S + s - p.cc_min - p.vc_min;  // u-tile column
        un[s] = __fmul_rn(ut[uy * upitch + ux], c[s]);
    }
    // coalesced store through LDS (the r tile is no longer needed)
    constexpr int SP = TB + 1;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) rt[lane * SP + wv * S + s] = un[s];
    __syncthreads();
    for (int e = threadIdx.x; e < TA * TB; e += NW * 64) {
        const int row = e / TB, col = e - row * TB;
        u_out[(size_t)(a0 + row) * p.W + b0 + col] = rt[row * SP + col];
    }
}

// ---------------------------------------------------------------------------------------
// Resident line solver for axis-aligned box PSFs (1 x L or L x 1).  Such a PSF couples
// pixels only along one image line, so every line is an independent 1-D RL problem.  A
// workgroup keeps LINES whole lines of u and r in LDS (f in registers) and runs all
// iterations of the call on chip; HBM is touched once at the start and once at the end.
// One or more wavefronts per line; each lane owns SEG consecutive pixels and evaluates
// the box by a sliding window (seeded per segment, Kahan-compensated when kahan = 1).
// Each LDS line carries a halo of HALO = L - 1 positions on both sides (plus SEG on the
// right for the last segment's unused tail) holding the boundary continuation: whoever
// writes a pixel also writes its mirror images, so no read needs a fold.  This needs
// HALO <= line length (a single reflection); deeper folds use the tiled kernels.
// LDS index of line position pos (pos >= -HALO): pos + HALO plus one pad word per SEG
// positions, which keeps the lanes of a wavefront on distinct banks.
// ---------------------------------------------------------------------------------------
struct ResidentArgs {
    int32_t H, W, bc, kahan;
    float* u;          // in/out (global)
    const float* f;
    int32_t n_iter;
    int32_t lines_per_wg, wpl;      // lines per workgroup, wavefronts per line
    int32_t conv_c0, corr_c0, len;  // window [c0, c0 + len) for conv and corr
    int32_t halo;                   // L - 1
    int32_t line_words;             // LDS words per line and plane
    float w;                        // box weight
};

template <int SEG>
__device__ __forceinline__ int line_idx(int pos, int halo) {
    const unsigned e = (unsigned)(pos + halo);
    return (int)(e + e / SEG);
}

// Write v at line position pos in [0, n) and at every halo position that continues it.
template <int SEG>
__device__ __forceinline__ void line_store(float* line, int pos, int n, int halo, int bc,
                                           float v) {
    line[line_idx<SEG>(pos, halo)] = v;
    if (bc == BC_REFLECT) {
        if (pos < halo) line[line_idx<SEG>(-1 - pos, halo)] = v;
        if (pos >= n - halo) line[line_idx<SEG>(2 * n - 1 - pos, halo)] = v;
    } else {
        if (pos == 0)
            for (int m = 1; m <= halo; ++m) line[line_idx<SEG>(-m, halo)] = v;
        if (pos == n - 1)
            for (int m = 0; m < halo; ++m) line[line_idx<SEG>(n + m, halo)] = v;
    }
}

// Window sums out[q] = sum_{t < len} line[p0 + q + c0 + t], q = 0..SEG-1 (halo-extended
// line, no folds), by a sliding window seeded at q = 0.  All LDS reads are issued before
// the dependent running sum.
// Sliding 1-D box sums of SEG consecutive outputs of one line (window [p0 + c0 + q,
// p0 + c0 + q + len) for output q), seed by a direct sum, slide Kahan-compensated.
// Exact zeros: every input is >= 0, so a direct float sum is 0 iff all of its terms are,
// but a slid sum is not.  The inputs at [lo + SEG - 1, lo + len) lie in all SEG windows,
// and a non-zero input among four of them proves that no window is all-zero, so the slide
// stands.  Otherwise (rare) the non-zero inputs are counted exactly along the slide and
// windows without any are set to 0.
template <int SEG>
__device__ __forceinline__ void box_segment(const float* line, int halo, int p0, int c0,
                                            int len, bool kahan, float (&out)[SEG]) {
    const int lo = p0 + c0;
    const int nh = min(SEG - 1, len);
    auto at = [&](int q) { return line[line_idx<SEG>(lo + q, halo)]; };
    // seed: four partial sums over [0, len)
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int q = 0;
#pragma unroll 1
    for (; q + 4 <= len; q += 4) {
        s0 += at(q);
        s1 += at(q + 1);
        s2 += at(q + 2);
        s3 += at(q + 3);
    }
    for (; q < len; ++q) s0 += at(q);
    // witness: four of the inputs at [nh, len), which every window of the segment holds
    float m = 0.f;
    if (len >= SEG) {
#pragma unroll
        for (int t = 0; t < 4; ++t) m = fmaxf(m, fabsf(at(nh + ((len - 1 - nh) * t) / 3)));
    }
    float din[SEG], dout[SEG];
#pragma unroll
    for (int q2 = 1; q2 < SEG; ++q2) {
        din[q2] = at(q2 + len - 1);
        dout[q2] = at(q2 - 1);
    }
    float run = (s0 + s1) + (s2 + s3), c = 0.f;
    out[0] = run;
#pragma unroll
    for (int q2 = 1; q2 < SEG; ++q2) {
        float d = din[q2] - dout[q2];
        if (kahan) kahan_add(run, c, d);
        else run += d;
        out[q2] = run;
    }
    if (!(m > 0.f)) {
        int n = 0;  // non-zero inputs in the window
#pragma unroll 1
        for (int t = 0; t < len; ++t) n += nz(at(t));
        if (n == 0) out[0] = 0.f;
#pragma unroll
        for (int q2 = 1; q2 < SEG; ++q2) {
            n += nz(at(q2 + len - 1)) - nz(at(q2 - 1));
            if (n == 0) out[q2] = 0.f;
        }
    }
}

// All iterations of one job's lines wg * lines_per_wg .. on chip (see resident_kernel).
// Threads past the job's lines_per_wg * 64 * wpl take part in the barriers only.
template <int ORIENT, int SEG>
__device__ __forceinline__ void resident_body(const ResidentArgs& a, int wg, float* lds) {
    const int n = (ORIENT == ORIENT_ROWS) ? a.W : a.H;       // line length
    const int m = (ORIENT == ORIENT_ROWS) ? a.H : a.W;       // number of lines
    const int tpl = 64 * a.wpl;                               // threads per line
    const int j = threadIdx.x / tpl;                          // line within the workgroup
    const int t = threadIdx.x % tpl;                          // segment within the line
    const int line = wg * a.lines_per_wg + j;
    const bool live = (j < a.lines_per_wg) && (line < m);
    const int halo = a.halo;
    float* ul = lds + (size_t)j * 2 * a.line_words;
    float* rl = ul + a.line_words;
    const int p0 = t * SEG;
    const bool work = live && p0 < n;

    auto gidx = [&](int pos) -> size_t {
        return ORIENT == ORIENT_ROWS ? (size_t)line * a.W + pos : (size_t)pos * a.W + line;
    };

    // zero both planes once (the last segment's tail reads past the right halo)
    for (int e = threadIdx.x; e < a.lines_per_wg * 2 * a.line_words; e += blockDim.x) lds[e] = 0.f;
    __syncthreads();
    float fr[SEG];
    if (live) {
        float uv[SEG];
#pragma unroll
        for (int q = 0; q < SEG; ++q) {
            int pos = p0 + q;
            fr[q] = pos < n ? a.f[gidx(pos)] : 0.f;
            uv[q] = pos < n ? a.u[gidx(pos)] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < SEG; ++q)
            if (p0 + q < n) line_store<SEG>(ul, p0 + q, n, halo, a.bc, uv[q]);
    }
    __syncthreads();
    const bool kahan = a.kahan != 0;

    for (int it = 0; it < a.n_iter; ++it) {
        if (work) {  // forward box + ratio
            float v[SEG];
            box_segment<SEG>(ul, halo, p0, a.conv_c0, a.len, kahan, v);
#pragma unroll
            for (int q = 0; q < SEG; ++q)
                if (p0 + q < n) line_store<SEG>(rl, p0 + q, n, halo, a.bc, rl_ratio(fr[q], a.w * v[q]));
        }
        __syncthreads();
        if (work) {  // adjoint box + multiplicative update
            float c[SEG];
            box_segment<SEG>(rl, halo, p0, a.corr_c0, a.len, kahan, c);
#pragma unroll
            for (int q = 0; q < SEG; ++q) {
                int pos = p0 + q;
                if (pos < n) {
                    float un = __fmul_rn(ul[line_idx<SEG>(pos, halo)], a.w * c[q]);
                    line_store<SEG>(ul, pos, n, halo, a.bc, un);
                }
            }
        }
        __syncthreads();
    }
    if (live) {
#pragma unroll
        for (int q = 0; q < SEG; ++q) {
            int pos = p0 + q;
            if (pos < n) a.u[gidx(pos)] = ul[line_idx<SEG>(pos, halo)];
        }
    }
}

// Neighbouring lines share cache lines (column lines especially): each XCD gets a
// contiguous range of workgroups, so that those lines are fetched once per XCD.
template <int ORIENT, int SEG>
__global__ __launch_bounds__(256) void resident_kernel(ResidentArgs a) {
    extern __shared__ float lds[];
    resident_body<ORIENT, SEG>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

// Several resident jobs of one line orientation and segment length in one launch (batches):
// job j owns workgroups [prefix[j], prefix[j + 1]) of the XCD-ordered index, and each
// workgroup runs its own job's iteration count.
typedef const __attribute__((address_space(4))) ResidentArgs* ConstResPtr;
template <int ORIENT, int SEG>
__global__ __launch_bounds__(256) void resident_multi_kernel(const ResidentArgs* table,
                                                             const int32_t* prefix, int n_jobs) {
    extern __shared__ float lds[];
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const ConstIntPtr pre = (ConstIntPtr)prefix;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {  // last job with prefix <= b
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const ConstResPtr t = (ConstResPtr)table + lo;
    ResidentArgs a;
    a.H = t->H; a.W = t->W; a.bc = t->bc; a.kahan = t->kahan;
    a.u = t->u; a.f = t->f; a.n_iter = t->n_iter;
    a.lines_per_wg = t->lines_per_wg; a.wpl = t->wpl;
    a.conv_c0 = t->conv_c0; a.corr_c0 = t->corr_c0; a.len = t->len;
    a.halo = t->halo; a.line_words = t->line_words; a.w = t->w;
    resident_body<ORIENT, SEG>(a, b - pre[lo], lds);
}

// ---------------------------------------------------------------------------------------
// Thinning bookkeeping.
// ---------------------------------------------------------------------------------------
// Per block of 256 pixels: number of active pixels (cnt < hyst), via wavefront ballots.
// Also flags the tile of every active pixel (all writers store 1).
struct ThinListArgs {
    const uint8_t* cnt;
    int64_t N;
    int32_t W, hyst, orient, tiles_a, TA, TB;
    int32_t* block_counts;
    int32_t* block_offsets;
    int32_t* tflag;
    int32_t* plist;
    int64_t* plist_len;
    int32_t n_blocks;
};

__device__ __forceinline__ int tile_of(const ThinListArgs& a, int64_t p) {
    int y = (int)(p / a.W), x = (int)(p - (int64_t)y * a.W);
    int ta, tb;
    if (a.orient == ORIENT_ROWS) { ta = y / a.TA; tb = x / a.TB; }
    else { ta = x / a.TA; tb = y / a.TB; }
    return tb * a.tiles_a + ta;
}

__global__ __launch_bounds__(256) void thin_count_kernel(ThinListArgs a) {
    __shared__ int wsum[4];
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool act = (p < a.N) && ((int)a.cnt[p] < a.hyst);
    if (act) a.tflag[tile_of(a, p)] = 1;
    unsigned long long m = __ballot(act);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) a.block_counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Exclusive scan of the block counts by one workgroup of 1024 threads (fixed order).
__global__ __launch_bounds__(1024) void scan_counts_kernel(const int32_t* counts,
                                                           int32_t* offsets, int n,
                                                           int64_t* total) {
    __shared__ int64_t part[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per;
    int64_t s = 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < n) s += counts[lo + i];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partials
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < n) {
            offsets[lo + i] = (int32_t)run;
            run += counts[lo + i];
        }
    if (threadIdx.x == 1023) *total = part[1023];
}

// Ascending compaction: block b writes its active indices at offsets[b] + rank, where the
// rank comes from the wavefront ballot (mbcnt) plus the preceding wavefronts' popcounts.
__global__ __launch_bounds__(256) void thin_scatter_kernel(ThinListArgs a) {
    __shared__ int wsum[4];
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool act = (p < a.N) && ((int)a.cnt[p] < a.hyst);
    unsigned long long m = __ballot(act);
    const int lane = threadIdx.x & 63, wv = wave_id();
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int base = a.block_offsets[blockIdx.x];
    for (int w = 0; w < wv; ++w) base += wsum[w];
    unsigned long long below = lane ? (m & ((~0ull) >> (64 - lane))) : 0ull;
    if (act) a.plist[base + __popcll(below)] = (int32_t)p;
}

// Tile list: ascending ids of flagged tiles (one workgroup); clear = 1 also clears the
// flags (per-pixel rule: thin_count sets them afresh), clear = 0 keeps them (block rule:
// they are the tiles' live activity flags).
__global__ __launch_bounds__(1024) void tile_compact_kernel(int32_t* tflag, int n,
                                                            int32_t* tlist, int64_t* count,
                                                            int clear) {
    __shared__ int wsum[16];
    __shared__ int base_s;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = wave_id();
    for (int t0 = 0; t0 < n; t0 += 1024) {
        int t = t0 + threadIdx.x;
        bool on = t < n && tflag[t] != 0;
        unsigned long long m = __ballot(on);
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int base = base_s;
        for (int w = 0; w < wv; ++w) base += wsum[w];
        unsigned long long below = lane ? (m & ((~0ull) >> (64 - lane))) : 0ull;
        if (on) {
            tlist[base + __popcll(below)] = t;
            if (clear) tflag[t] = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wsum[w];
            base_s += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base_s;
}

// Block rule (counters per block of 2^lg pixels a side): set the flag of each 64 x 64 tile
// to 1 if it holds an active block (counter < hyst), else 0, one thread per tile.  Tile t covers lane-axis tile
// t % tiles_a and strip-axis tile t / tiles_a, rows for ORIENT_ROWS, columns otherwise.
__global__ __launch_bounds__(256) void block_tiles_kernel(const uint8_t* cntb, int H, int W,
                                                          int lg, int bw, int hyst, int orient,
                                                          int tiles_a, int n_tiles,
                                                          int32_t* tflag) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tiles) return;
    const int ta = t % tiles_a, tb = t / tiles_a;
    const int y0 = (orient == ORIENT_ROWS ? ta : tb) * 64;
    const int x0 = (orient == ORIENT_ROWS ? tb : ta) * 64;
    const int by1 = min(y0 + 64, H), bx1 = min(x0 + 64, W);
    int on = 0;
    for (int y = y0; y < by1; y += 1 << lg)
        for (int x = x0; x < bx1; x += 1 << lg)
            on |= (int)cntb[(size_t)(y >> lg) * bw + (x >> lg)] < hyst;
    tflag[t] = on;
}

// Block rule: every pixel's counter from its block's (get_state, statistics and the
// per-pixel list), and back: each block's counter from its top-left pixel (set_state).
__global__ __launch_bounds__(256) void block_expand_kernel(const uint8_t* cntb, uint8_t* cnt,
                                                           int64_t N, int W, int lg, int bw) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * 256) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        cnt[p] = cntb[(size_t)(y >> lg) * bw + (x >> lg)];
    }
}

__global__ __launch_bounds__(256) void block_compress_kernel(const uint8_t* cnt, uint8_t* cntb,
                                                             int W, int lg, int bw,
                                                             int64_t n_blocks) {
    for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < n_blocks;
         b += (int64_t)gridDim.x * 256) {
        const int64_t by = b / bw, bx = b - by * bw;
        cntb[b] = cnt[(by << lg) * W + (bx << lg)];
    }
}

// ---------------------------------------------------------------------------------------
// Deterministic FP64 reductions (flux, active count) and small utilities.
// ---------------------------------------------------------------------------------------
constexpr int RED_BLOCKS = 512;

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// partial[b] = sum of u over the elements b*256 + t + j*RED_BLOCKS*256 (fixed order)
__global__ __launch_bounds__(256) void reduce_sum_kernel(const float* u, int64_t N,
                                                         double* partial) {
    __shared__ double ws[4];
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N;
         p += (int64_t)RED_BLOCKS * 256)
        s += (double)u[p];
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

__global__ __launch_bounds__(256) void count_active_kernel(const uint8_t* cnt, int64_t N,
                                                           int hyst, int64_t* partial_i) {
    __shared__ int64_t ws[4];
    int64_t s = 0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N;
         p += (int64_t)RED_BLOCKS * 256)
        s += ((int)cnt[p] < hyst) ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial_i[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void final_reduce_kernel(const double* partial,
                                                           const int64_t* partial_i,
                                                           double* out_d, int64_t* out_i) {
    __shared__ double ds[256];
    __shared__ int64_t is[256];
    double s = 0.0;
    int64_t c = 0;
    for (int b = threadIdx.x; b < RED_BLOCKS; b += 256) {
        s += partial[b];
        if (partial_i) c += partial_i[b];
    }
    ds[threadIdx.x] = s;
    is[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            ds[threadIdx.x] += ds[threadIdx.x + off];
            is[threadIdx.x] += is[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out_d = ds[0];
        if (out_i) *out_i = is[0];
    }
}

// f must be finite and >= 0; sets *flag = 1 otherwise.
// Denominator of the TV-regularised update, g = 1 - lambda * div(grad u / |grad u|_eps):
// forward-difference gradient (0 across the last column / row), backward-difference
// divergence (no flux before the first column / row).  One thread per pixel, reading the
// pixel, its right and lower neighbours and the two pixels that feed n at (y, x-1) and
// (y-1, x).
__device__ __forceinline__ void tv_n_at(const float* u, int H, int W, int y, int x, float eps2,
                                        float& nx, float& ny) {
    const float c = u[(size_t)y * W + x];
    const float gx = x + 1 < W ? u[(size_t)y * W + x + 1] - c : 0.f;
    const float gy = y + 1 < H ? u[(size_t)(y + 1) * W + x] - c : 0.f;
    const float m = __fsqrt_rn(gx * gx + gy * gy + eps2);
    nx = __fdiv_rn(gx, m);
    ny = __fdiv_rn(gy, m);
}

__global__ __launch_bounds__(256) void tv_factor_kernel(const float* u, float* g, int H, int W,
                                                        float lambda, float eps) {
    const int64_t N = (int64_t)H * W;
    const float eps2 = eps * eps;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < N;
         q += (int64_t)gridDim.x * 256) {
        const int y = (int)(q / W), x = (int)(q - (int64_t)y * W);
        float nx, ny, d;
        tv_n_at(u, H, W, y, x, eps2, nx, ny);
        d = nx + ny;
        if (x > 0) {
            float ax, ay;
            tv_n_at(u, H, W, y, x - 1, eps2, ax, ay);
            d -= ax;
        }
        if (y > 0) {
            float bx, by;
            tv_n_at(u, H, W, y - 1, x, eps2, bx, by);
            d -= by;
        }
        g[q] = 1.f - lambda * d;
    }
}

// Robust variant, between the forward convolution and the two correlations: from v (in
// the r plane) and f, the weight w = 1 / sqrt(d + eps^2) of the I-divergence
// d = v - f - f ln(v / f) (d = v where f = 0, d = 0 where v <= 0) and the weighted ratio
// w f / v (0 where v <= 0), written over v.  d = f (x - ln(1 + x)) with x = (v - f) / f:
// a short Taylor series below |x| = 0.1 (the direct difference cancels there), log1p
// above.  The divisions and the square root are correctly rounded.
__global__ __launch_bounds__(256) void robust_weights_kernel(float* r, const float* f, float* w,
                                                             int64_t N, float eps2) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < N;
         q += (int64_t)gridDim.x * 256) {
        const float v = r[q], fq = f[q];
        float d = 0.f, rq = 0.f;
        if (v > 0.f) {
            if (fq == 0.f) {
                d = v;
            } else {
                const float x = __fdiv_rn(v - fq, fq);
                float t;
                if (fabsf(x) < 0.1f) {
                    // x - ln(1 + x) = x^2 (1/2 - x/3 + x^2/4 - x^3/5 + x^4/6 - x^5/7 + x^6/8)
                    float s = 0.125f;
                    s = fmaf(s, x, -1.f / 7.f);
                    s = fmaf(s, x, 1.f / 6.f);
                    s = fmaf(s, x, -0.2f);
                    s = fmaf(s, x, 0.25f);
                    s = fmaf(s, x, -1.f / 3.f);
                    s = fmaf(s, x, 0.5f);
                    t = x * x * s;
                } else {
                    t = x - log1pf(x);
                }
                d = fq * t;
            }
            rq = __fdiv_rn(fq, v);
        }
        const float wq = __fdiv_rn(1.f, __fsqrt_rn(d + eps2));
        w[q] = wq;
        r[q] = wq * rq;
    }
}

// Job set-up in one pass: f and u^0 into the workspace, r = 0, and the check of f (the
// observed image must be non-negative and finite; a wavefront that meets a negative, NaN
// or infinite value sets *flag).  u0 may be f itself.
__global__ __launch_bounds__(256) void init_fields_kernel(float* wf, float* wu, float* wr,
                                                          const float* f, const float* u0,
                                                          int64_t N, int32_t* flag) {
    int bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * 256) {
        const float v = f[p];
        if (!(v >= 0.f) || isinf(v)) bad = 1;
        wf[p] = v;
        wu[p] = u0[p];
        wr[p] = 0.f;
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void copy_f32_kernel(float* dst, const float* src, int64_t n) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * 256)
        dst[p] = src[p];
}

__global__ __launch_bounds__(256) void copy_u8_kernel(uint8_t* dst, const uint8_t* src, int64_t n) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * 256)
        dst[p] = src[p];
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* dst, uint32_t v, int64_t n) {
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * 256)
        dst[p] = v;
}

__global__ void set_i64_kernel(int64_t* dst, int64_t v) { *dst = v; }

__global__ __launch_bounds__(64) void thin_finalize_kernel(int32_t* act_part, int64_t* sched,
                                                           int64_t* active_total, int64_t k) {
    thin_finalize_wave(act_part, sched, active_total, k, -1);
}

}  // namespace rlk

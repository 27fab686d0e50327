// C ABI of the Richardson-Lucy library: job set-up, kernel selection and launch sequencing.
// Every RL step runs in the kernels of rl_kernels.hpp; this file only decides which kernel,
// with which tables and tiles, and enqueues them on the job's stream.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <fstream>
#include <sstream>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "psf_compile.hpp"
#include "rl.h"
#include "rl_kernels.hpp"

using rlk::DevSpan;
using rlk::PhaseArgs;
using rlk::ResidentArgs;

static_assert(sizeof(DevSpan) == sizeof(rl::Span), "span layout");

namespace {

constexpr size_t kAlign = 256;
// dynamic LDS of one workgroup: 160 KB per CU less the phase kernels' static arrays (the
// block rule's per-wavefront failure words, the persistent schedule's task slot)
constexpr size_t kLdsLimit = 160 * 1024 - 256;
constexpr int kNW = 8;  // wavefronts per workgroup in the tiled kernels
// When the span and sliding kernels run four-wavefront workgroups (strips of 8): 0 never,
// 1 where eight wavefronts would run strips of 4 (images below 0.5 Mpx), 2 also in place of
// strips of 8 (64 x 32 tiles on every image)
constexpr int kFourWave = 1;
// wavefronts per workgroup of the matrix-core kernel: a job's own launches, batch launches
constexpr int kMfmaNW = 8;
constexpr int kMfmaBatchNW = 4;
constexpr size_t kSpanPad = 2;  // zero descriptors after each span table (read-ahead)

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

enum Kind { KIND_SPAN = 0, KIND_SLIDE = 1, KIND_RESIDENT = 2, KIND_FUSED = 3, KIND_RECT = 4, KIND_SAT = 5,
            KIND_MFMA = 6 };

// ---- kernel timing registry -----------------------------------------------------------
struct TimedLaunch {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_timed;

struct Config {
    int path = 0, sched = 0, kind = 0, orient = 0, S = 16, lmax = 1;
    int nw = kNW;            // wavefronts per workgroup of the span and sliding kernels
    int threads = kNW * 64;  // workgroup size of the phase kernels
    int TA = 64, TB = 64, tiles_a = 1, tiles_b = 1;
    int reach_a = 1, reach_b = 1;  // persistent schedule: tiles within the halo's reach
    // resident
    int line_n = 0, lines = 0, wpl = 1, seg = 2, lines_per_wg = 1, line_words = 0;
    size_t lds_a = 0, lds_b = 0;
    rl::OpTable conv, corr;
};

struct Layout {
    size_t f, u, r, conv_spans, conv_w, corr_spans, corr_w, mf_conv, mf_corr, cnt, plist, tflag, tlist,
        bcounts, boffs, ctr, sched, act, red, red_i, args, prefix, u2, fargs, done, pctl, tvg, wt,
        cntb, total;
    size_t blob_end;  // [conv_spans, blob_end): the regions rl_init uploads from the host
};

// counters block (int64 slots)
enum Ctr { C_PLIST_LEN = 0, C_TLIST_LEN, C_ACTIVE_TOTAL, C_F_INVALID, C_ACTIVE_NOW, C_FLUX,
           C_COUNT = 8 };

int64_t thin_blocks(int64_t N) { return (N + 255) / 256; }

// Block rule (thin.block >= 8): log2 of the block side, else 0 (per-pixel rule).
int block_lg(const rl_params* p) {
    if (p->thin.mode == RL_THIN_OFF || p->thin.block < 8) return 0;
    int lg = 0;
    while ((1 << lg) < p->thin.block) ++lg;
    return lg;
}
int64_t block_cols(const rl_params* p, int lg) { return (p->width + (1 << lg) - 1) >> lg; }
int64_t block_count(const rl_params* p, int lg) {
    return block_cols(p, lg) * ((p->height + (1 << lg) - 1) >> lg);
}

bool is_full(int64_t k, int R) { return k == 0 || (R > 0 && k % R == 0); }
bool is_rebuild(int64_t k, int R, int C) {
    if (is_full(k, R)) return false;
    return is_full(k - 1, R) || (C > 0 && (k - 1) % C == 0);
}

size_t tile_lds_bytes(const rl::OpTable& t, int orient, int TB, int extra) {
    (void)orient;
    size_t na = 64 + t.lane_max - t.lane_min;
    size_t nb = TB + t.c_max - t.c_min + extra;
    size_t ny = orient == rlk::ORIENT_ROWS ? na : nb;
    size_t nx = orient == rlk::ORIENT_ROWS ? nb : na;
    size_t pitch = nx | 1;
    size_t main = ny * pitch * sizeof(float);
    size_t stage = (size_t)64 * (TB + 1) * sizeof(float);
    return std::max(main, stage);
}

// Cost estimate per output (VALU-op equivalents), used to pick kernel and orientation.
double span_cost(const rl::OpTable& t, int S, int lmax, bool kahan) {
    (void)lmax;
    (void)kahan;
    double valu = 0, lds = 0;
    for (const rl::Span& s : t.spans) {
        valu += s.len + 3.0;  // FMAs + per-piece address and descriptor work
        lds += double(S + s.len - 1) / S;
        if (s.row_end) valu += 1.0;
    }
    return std::max(valu, 2.0 * lds) + 8.0;
}

double slide_cost(const rl::OpTable& t, int S, bool kahan) {
    double valu = 0, lds = 0;
    for (const rl::Span& s : t.spans) {
        valu += 2.0 + double(s.len) / S;
        lds += 2.0 + double(s.len) / S;
    }
    valu += kahan ? 4.0 : 1.0;
    return std::max(valu, 2.0 * lds) + 8.0;
}

bool all_uniform(const rl::OpTable& t) {
    for (const rl::Span& s : t.spans)
        if (!s.uniform) return false;
    return true;
}

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ---- weight operands of the matrix-core kernel ------------------------------------------
// bfloat16 of x rounded to nearest (ties to even); x is finite.
uint16_t bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

int mfma_lines(const rl::OpTable& t) { return t.lane_max - t.lane_min + 1; }
// one zero line past the end: the kernel loads each line's operands one line ahead
size_t mfma_table_bytes(const rl::OpTable& t) { return (size_t)(mfma_lines(t) + 1) * 3 * 64 * 16; }

// Per PSF line (lane_min .. lane_max of the ROWS table), per bfloat16 part (w = w1 + w2 + w3,
// each the rounded remainder of the previous), per lane l: the 8 entries
// B[8 (l / 16) + t][l % 16] = w(line, c_min + 8 (l / 16) + t - l % 16) of the banded weight
// operand (zero outside the line's taps).
std::vector<uint16_t> mfma_table(const rl::OpTable& t) {
    const int lines = mfma_lines(t), width = t.c_max - t.c_min + 1;
    std::vector<float> grid((size_t)lines * width, 0.f);
    for (const rl::Span& s : t.spans)
        for (int q = 0; q < s.len; ++q)
            grid[(size_t)(s.lane_off - t.lane_min) * width + (s.c0 + q - t.c_min)] = t.w[s.woff + q];
    std::vector<uint16_t> out((size_t)(lines + 1) * 3 * 64 * 8, 0);
    for (int li = 0; li < lines; ++li)
        for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
                const int dj = 8 * (l / 16) + e - l % 16;
                const float w = (dj >= 0 && dj < width) ? grid[(size_t)li * width + dj] : 0.f;
                const uint16_t p1 = bf16_rne(w);
                const float r1 = w - bf16_value(p1);
                const uint16_t p2 = bf16_rne(r1);
                const uint16_t p3 = bf16_rne(r1 - bf16_value(p2));
                const uint16_t parts[3] = {p1, p2, p3};
                for (int k = 0; k < 3; ++k) out[(((size_t)li * 3 + k) * 64 + l) * 8 + e] = parts[k];
            }
    return out;
}

// The matrix-core kernel applies to ROWS tables at most MF_MAXW taps wide with at most
// MF_MAXROWS lines.
bool mfma_fits(const rl::OpTable& t) {
    return t.c_max - t.c_min + 1 <= rlk::MF_MAXW && mfma_lines(t) <= rlk::MF_MAXROWS;
}

// Cost per output in the units of span_cost (VALU ops per output), fitted to measured
// launch times at 1024^2 and 2048^2 (dense 9 x 9 and 15 x 15, against the span kernel):
// about 10.5 per PSF line (six products per line, each taking as long per output as one
// VALU instruction, plus the LDS operand reads they wait on) and 52 for the tile's
// conversion and the epilogue.
double mfma_cost(const rl::OpTable& t) { return 10.5 * mfma_lines(t) + 52.0; }

// ---- tuning cache ----------------------------------------------------------------------
struct TuneKey {
    int path, kh, kw, taps, runs, bucket, thin, schedule;
    bool operator<(const TuneKey& o) const {
        return std::tie(path, kh, kw, taps, runs, bucket, thin, schedule) <
               std::tie(o.path, o.kh, o.kw, o.taps, o.runs, o.bucket, o.thin, o.schedule);
    }
};
struct TuneEntry {
    int schedule;  // schedule to use when the job asks for RL_SCHED_AUTO
    rl_tuning t;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

TuneKey tune_key(const rl_params* p, const rl::CompiledPsf& c) {
    TuneKey k{};
    k.path = p->path == RL_PATH_AUTO ? c.auto_path : p->path;
    k.kh = c.kh;
    k.kw = c.kw;
    k.taps = c.n_taps;
    k.runs = (int)c.runs.size();
    double px = (double)p->height * p->width;
    k.bucket = (int)std::lround(std::log2(std::max(1.0, px)));
    k.thin = p->thin.mode != RL_THIN_OFF;
    k.schedule = p->schedule;
    return k;
}

bool tuning_is_default(const rl_tuning& t) {
    return t.strip == 0 && t.seg == 0 && t.lines_per_wg == 0 && t.graph_iters == 0;
}

// Decide path, schedule and kernel for a job.  Deterministic in (params, PSF, cache).
rl_status choose_config_raw(const rl_params* p, const rl::CompiledPsf& c, Config* cfg,
                            std::string* why);

rl_status choose_config(const rl_params* p, const rl::CompiledPsf& c, Config* cfg,
                        std::string* why) {
    if (tuning_is_default(p->tuning)) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(p, c));
        if (it != g_tune.end()) {
            rl_params q = *p;
            q.tuning = it->second.t;
            if (q.schedule == RL_SCHED_AUTO) q.schedule = it->second.schedule;
            return choose_config_raw(&q, c, cfg, why);
        }
    }
    return choose_config_raw(p, c, cfg, why);
}

rl_status choose_config_raw(const rl_params* p, const rl::CompiledPsf& c, Config* cfg,
                            std::string* why) {
    const int H = p->height, W = p->width;
    const bool thin = p->thin.mode != RL_THIN_OFF;
    int path = p->path == RL_PATH_AUTO ? c.auto_path : p->path;
    if (path < RL_PATH_DIRECT || path > RL_PATH_MFMA) { *why = "unknown path"; return RL_E_INVAL; }
    if (path == RL_PATH_BOX_AXIS && !c.is_axis_box) {
        *why = "BOX_AXIS path needs a 1 x L or L x 1 uniform box PSF";
        return RL_E_INVAL;
    }
    if ((path == RL_PATH_BOX_RECT || path == RL_PATH_BOX_SAT) && !c.is_rect) {
        *why = "BOX_RECT and BOX_SAT paths need a uniform rectangle of at least 2 x 2 taps";
        return RL_E_INVAL;
    }
    cfg->path = path;
    int sched = p->schedule;
    if (sched < RL_SCHED_AUTO || sched > RL_SCHED_PERSISTENT) { *why = "unknown schedule"; return RL_E_INVAL; }
    const bool tv = p->tv_lambda > 0.f;
    if (tv && (thin || sched == RL_SCHED_FUSED || sched == RL_SCHED_RESIDENT)) {
        *why = "TV regularisation runs on the two-pass schedule without thinning";
        return RL_E_UNSUPPORTED;
    }
    const bool rob = p->rob_eps > 0.f;
    if (rob && (tv || thin || sched == RL_SCHED_FUSED || sched == RL_SCHED_RESIDENT)) {
        *why = "the robust data term runs on the two-pass schedule, without TV or thinning";
        return RL_E_UNSUPPORTED;
    }
    if (sched == RL_SCHED_PERSISTENT && (thin || tv || rob)) {
        *why = "the persistent schedule serves plain RL";
        return RL_E_UNSUPPORTED;
    }
    if (sched == RL_SCHED_FUSED) {
        if (thin) { *why = "the fused schedule serves plain RL"; return RL_E_UNSUPPORTED; }
        if (H < 64 || W < 64) { *why = "the fused schedule needs images of at least 64 x 64"; return RL_E_UNSUPPORTED; }
        cfg->sched = RL_SCHED_FUSED;
        cfg->kind = KIND_FUSED;
        cfg->orient = rlk::ORIENT_ROWS;
        cfg->S = 8;
        cfg->TA = 64;
        cfg->TB = kNW * cfg->S;
        cfg->lmax = 16;
        rl::Orient o = rl::Orient::Rows;
        cfg->conv = rl::build_op_table(p->psf, p->psf_h, p->psf_w, false, o, false, 16);
        cfg->corr = rl::build_op_table(p->psf, p->psf_h, p->psf_w, true, o, false, 16);
        const rl::OpTable &v = cfg->conv, &c2 = cfg->corr;
        const int ext[8] = {v.lane_min, v.lane_max, v.c_min, v.c_max, c2.lane_min, c2.lane_max, c2.c_min, c2.c_max};
        for (int e : ext)
            if (e < -63 || e > 63) { *why = "PSF extent too large for the fused schedule"; return RL_E_UNSUPPORTED; }
        if (std::abs(c2.lane_min + c2.lane_max) > cfg->TA || std::abs(c2.c_min + c2.c_max) > cfg->TB) {
            *why = "PSF too one-sided for the fused tile"; return RL_E_UNSUPPORTED;
        }
        const int RA = cfg->TA + c2.lane_max - c2.lane_min, RB = cfg->TB + c2.c_max - c2.c_min;
        const int UA = RA + v.lane_max - v.lane_min, UB = RB + v.c_max - v.c_min;
        cfg->lds_a = ((size_t)UA * (UB | 1) + (size_t)RA * (RB | 1) + cfg->S) * sizeof(float);
        if (cfg->lds_a > kLdsLimit) { *why = "PSF extent too large for the fused LDS tile"; return RL_E_UNSUPPORTED; }
        cfg->tiles_a = (H + cfg->TA - 1) / cfg->TA;
        cfg->tiles_b = (W + cfg->TB - 1) / cfg->TB;
        return RL_OK;
    }
    const int box_orient = c.box_orient == rl::Orient::Rows ? rlk::ORIENT_ROWS : rlk::ORIENT_COLS;
    if (path == RL_PATH_BOX_AXIS && !thin && !tv && !rob &&
        (sched == RL_SCHED_AUTO || sched == RL_SCHED_RESIDENT)) {
        int n = box_orient == rlk::ORIENT_ROWS ? W : H;
        int m = box_orient == rlk::ORIENT_ROWS ? H : W;
        // the on-chip halo holds a single reflection: needs L - 1 <= line length
        if (n <= 8192 && c.box_len - 1 <= n) {
            cfg->sched = RL_SCHED_RESIDENT;
            cfg->kind = KIND_RESIDENT;
            cfg->orient = box_orient;
            cfg->line_n = n;
            cfg->lines = m;
            int seg_t = p->tuning.seg;
            if (seg_t) {
                if (seg_t < 2 || seg_t > 32 || (seg_t & (seg_t - 1))) { *why = "tuning.seg"; return RL_E_INVAL; }
                cfg->seg = seg_t;
                cfg->wpl = std::max(1, (n + 64 * seg_t - 1) / (64 * seg_t));
                if (cfg->wpl > 4) { *why = "tuning.seg too small for this line"; return RL_E_INVAL; }
            } else {
                // default: 8 pixels per lane, at most 4 wavefronts per line
                cfg->seg = 8;
                cfg->wpl = (n + 64 * 8 - 1) / (64 * 8);
                while (cfg->wpl > 4) { cfg->seg *= 2; cfg->wpl = (n + 64 * cfg->seg - 1) / (64 * cfg->seg); }
                cfg->wpl = std::max(1, cfg->wpl);
            }
            const int tpl = 64 * cfg->wpl;
            const int halo = c.box_len - 1;
            const size_t span = (size_t)halo + n + halo + cfg->seg;
            cfg->line_words = (int)(span + span / cfg->seg + 1);
            const size_t per_line = 2 * (size_t)cfg->line_words * sizeof(float);
            int by_threads = 256 / tpl;
            int by_lds = (int)std::max<size_t>(1, (64 * 1024) / per_line);
            int want = std::max(1, (m + 511) / 512);  // aim for >= 512 workgroups
            if (p->tuning.lines_per_wg > 0) want = p->tuning.lines_per_wg;
            cfg->lines_per_wg = std::max(1, std::min(std::min(by_threads, by_lds), want));
            if (per_line > kLdsLimit) { *why = "line too long for LDS"; return RL_E_UNSUPPORTED; }
            cfg->lds_a = cfg->lines_per_wg * per_line;
            return RL_OK;
        }
        if (sched == RL_SCHED_RESIDENT) { *why = "line too long for the resident schedule"; return RL_E_UNSUPPORTED; }
    }
    if (sched == RL_SCHED_RESIDENT) {
        *why = "the resident schedule serves BOX_AXIS PSFs without thinning";
        return RL_E_UNSUPPORTED;
    }
    cfg->sched = sched == RL_SCHED_PERSISTENT ? RL_SCHED_PERSISTENT : RL_SCHED_TWO_PASS;
    const float* h = p->psf;
    const int kh = p->psf_h, kw = p->psf_w;
    const bool kahan = p->kahan != 0;
    const int64_t npx = (int64_t)H * W;
    // outputs per lane: long strips amortise seeds and windows, short strips give the
    // latency-bound kernels more wavefronts on small images
    // defaults from measurements with 8 wavefronts per workgroup on 64^2 .. 2048^2 images:
    // 4 outputs per lane below 0.5 Mpx, 8 from there on
    // the block rule takes its decisions per block inside 64 x 64 tiles: strips of 8
    const bool blk = block_lg(p) > 0;
    const int def_S = blk ? 8 : npx >= ((int64_t)1 << 19) ? 8 : 4;
    const int span_S = blk ? 8 : p->tuning.strip ? p->tuning.strip : def_S;
    const int slide_S = blk ? 8 : p->tuning.strip ? p->tuning.strip : def_S;
    if (span_S != 4 && span_S != 8 && span_S != 16 && span_S != 32) { *why = "tuning.strip"; return RL_E_INVAL; }
    const bool mfma_sched = sched == RL_SCHED_AUTO || sched == RL_SCHED_TWO_PASS;
    if (path == RL_PATH_MFMA) {
        rl::OpTable t = rl::build_op_table(h, kh, kw, false, rl::Orient::Rows, false, 0);
        if (!mfma_fits(t)) {
            *why = "the MFMA path needs PSF rows at most 17 taps wide and at most 64 rows";
            return RL_E_UNSUPPORTED;
        }
        if (!mfma_sched) { *why = "the MFMA path runs on the two-pass schedule"; return RL_E_UNSUPPORTED; }
    }
    if (path == RL_PATH_MFMA) {
        cfg->kind = KIND_MFMA;
        cfg->orient = rlk::ORIENT_ROWS;
        cfg->S = 16;
        cfg->lmax = 0;
        cfg->conv = rl::build_op_table(h, kh, kw, false, rl::Orient::Rows, false, 0);
        cfg->corr = rl::build_op_table(h, kh, kw, true, rl::Orient::Rows, false, 0);
    } else if (path == RL_PATH_DIRECT) {
        cfg->kind = KIND_SPAN;
        cfg->orient = rlk::ORIENT_ROWS;
        cfg->S = std::min(span_S, 16);
        cfg->lmax = 1;
        cfg->conv = rl::build_tap_table(h, kh, kw, false);
        cfg->corr = rl::build_tap_table(h, kh, kw, true);
    } else if (path == RL_PATH_BOX_RECT || path == RL_PATH_BOX_SAT) {
        if (slide_S != 4 && slide_S != 8) { *why = "BOX_RECT and BOX_SAT run strips of 4 or 8"; return RL_E_UNSUPPORTED; }
        cfg->kind = path == RL_PATH_BOX_SAT ? KIND_SAT : KIND_RECT;
        cfg->orient = rlk::ORIENT_ROWS;
        cfg->S = slide_S;
        cfg->lmax = 0;
        cfg->conv = rl::build_op_table(h, kh, kw, false, rl::Orient::Rows, true, 0);
        cfg->corr = rl::build_op_table(h, kh, kw, true, rl::Orient::Rows, true, 0);
    } else if (path == RL_PATH_BOX_AXIS) {
        cfg->kind = KIND_SLIDE;
        cfg->orient = box_orient;
        cfg->S = slide_S;
        rl::Orient o = c.box_orient;
        cfg->conv = rl::build_op_table(h, kh, kw, false, o, true, 0);
        cfg->corr = rl::build_op_table(h, kh, kw, true, o, true, 0);
    } else {
        // RUNS: cheapest of {sliding runs, register-blocked spans} x {rows, cols}
        double best = 1e30;
        for (int oi = 0; oi < 2; ++oi) {
            rl::Orient o = oi == 0 ? rl::Orient::Rows : rl::Orient::Cols;
            rl::OpTable u = rl::build_op_table(h, kh, kw, false, o, true, 0);
            if (all_uniform(u)) {
                double cost = slide_cost(u, slide_S, kahan);
                if (cost < best) {
                    best = cost;
                    cfg->kind = KIND_SLIDE;
                    cfg->orient = oi;
                    cfg->S = slide_S;
                    cfg->lmax = 0;
                }
            }
            for (int lm : {4, 8, 16}) {
                rl::OpTable t = rl::build_op_table(h, kh, kw, false, o, false, lm);
                double cost = span_cost(t, std::min(span_S, 16), lm, kahan);
                if (cost < best) {
                    best = cost;
                    cfg->kind = KIND_SPAN;
                    cfg->orient = oi;
                    cfg->S = std::min(span_S, 16);
                    cfg->lmax = lm;
                }
            }
        }
        // AUTO: dense lines go to the matrix cores where that is cheaper
        rl::OpTable mt = rl::build_op_table(h, kh, kw, false, rl::Orient::Rows, false, 0);
        if (p->path == RL_PATH_AUTO && mfma_sched && mfma_fits(mt) && mfma_cost(mt) < best) {
            cfg->path = RL_PATH_MFMA;
            cfg->kind = KIND_MFMA;
            cfg->orient = rlk::ORIENT_ROWS;
            cfg->S = 16;
            cfg->lmax = 0;
            cfg->conv = mt;
            cfg->corr = rl::build_op_table(h, kh, kw, true, rl::Orient::Rows, false, 0);
        } else {
            rl::Orient o = cfg->orient == 0 ? rl::Orient::Rows : rl::Orient::Cols;
            bool split = cfg->kind == KIND_SLIDE;
            int lm = cfg->kind == KIND_SLIDE ? 0 : cfg->lmax;
            cfg->conv = rl::build_op_table(h, kh, kw, false, o, split, lm);
            cfg->corr = rl::build_op_table(h, kh, kw, true, o, split, lm);
        }
    }
    // four-wavefront workgroups with strips of 8 in place of eight wavefronts with strips
    // of 4: the same 64 x 32 tile, half the seeds and windows per output (span and sliding
    // kernels with the default strip, two-pass and persistent alike, so that the schedules
    // keep giving the same results; the block rule needs 64 x 64 tiles)
    if (kFourWave && (cfg->kind == KIND_SPAN || cfg->kind == KIND_SLIDE) && !p->tuning.strip &&
        !blk && (cfg->S == 4 || (kFourWave == 2 && cfg->S == 8))) {
        cfg->S = 8;
        cfg->nw = 4;
        cfg->threads = 4 * 64;
    }
    cfg->TA = 64;
    cfg->TB = cfg->kind == KIND_MFMA ? rlk::MF_T : cfg->nw * cfg->S;
    if (cfg->kind == KIND_MFMA) {
        // a job's own launches: eight wavefronts per tile (rl_iterate_batch runs its matrix-core
        // groups with four, kMfmaBatchNW; the results are the same)
        cfg->nw = kMfmaNW;
        cfg->threads = kMfmaNW * 64;
    }
    const int extra = 0;  // windows never read past the last tap of a piece
    auto lds_for = [&](const rl::OpTable& t) {
        size_t b = tile_lds_bytes(t, cfg->orient, cfg->TB, extra);
        if (cfg->kind == KIND_SLIDE) {
            // tile plus the seed / strip-total exchange area (after the tile, not the stage)
            size_t na = 64 + t.lane_max - t.lane_min, nb = cfg->TB + t.c_max - t.c_min + extra;
            size_t ny = cfg->orient == rlk::ORIENT_ROWS ? na : nb;
            size_t nx = cfg->orient == rlk::ORIENT_ROWS ? nb : na;
            b = std::max(b, (ny * (nx | 1) + (size_t)(4 * cfg->nw * 64 + cfg->nw)) * sizeof(float));
        }
        if (cfg->kind == KIND_RECT) {
            // tile plus the horizontal window sums of every tile row
            size_t ny = 64 + t.lane_max - t.lane_min, nx = cfg->TB + t.c_max - t.c_min;
            b = rlk::rect_lds_floats<kNW>((int)ny, (int)nx, cfg->TB) * sizeof(float);
        }
        if (cfg->kind == KIND_SAT) {
            // tile plus the FP64 summed-area table and its non-zero counts
            int ny = 64 + t.lane_max - t.lane_min, nx = cfg->TB + t.c_max - t.c_min;
            b = rlk::sat_lds_bytes<kNW>(ny, nx);
        }
        if (cfg->kind == KIND_MFMA) b = rlk::mfma_lds_bytes(mfma_lines(t));  // three bf16 planes
        return b;
    };
    cfg->lds_a = lds_for(cfg->conv);
    cfg->lds_b = lds_for(cfg->corr);
    while (std::max(cfg->lds_a, cfg->lds_b) > kLdsLimit && cfg->kind == KIND_SLIDE && cfg->S > 8) {
        cfg->S /= 2;
        cfg->TB = cfg->nw * cfg->S;
        cfg->lds_a = lds_for(cfg->conv);
        cfg->lds_b = lds_for(cfg->corr);
    }
    if (std::max(cfg->lds_a, cfg->lds_b) > kLdsLimit) {
        *why = "PSF extent too large for the LDS tile";
        return RL_E_UNSUPPORTED;
    }
    {
        // the tile loader covers at most 64 * MAXC columns
        const rl::OpTable& t = cfg->conv;
        int nx = cfg->orient == rlk::ORIENT_ROWS
                     ? cfg->TB + t.c_max - t.c_min + extra
                     : 64 + t.lane_max - t.lane_min;
        if (nx > 64 * rlk::MAXC) { *why = "PSF extent too wide for the tile loader"; return RL_E_UNSUPPORTED; }
    }
    if (blk && (cfg->TA != 64 || cfg->TB != 64)) {
        *why = "the block rule needs 64 x 64 tiles";
        return RL_E_UNSUPPORTED;
    }
    const int la = cfg->orient == rlk::ORIENT_ROWS ? H : W;  // lane axis length
    const int lb = cfg->orient == rlk::ORIENT_ROWS ? W : H;
    cfg->tiles_a = (la + cfg->TA - 1) / cfg->TA;
    cfg->tiles_b = (lb + cfg->TB - 1) / cfg->TB;
    if (cfg->sched == RL_SCHED_PERSISTENT) {
        if (cfg->kind != KIND_SPAN && cfg->kind != KIND_SLIDE) {
            *why = "the persistent schedule runs the span and sliding kernels";
            return RL_E_UNSUPPORTED;
        }
        if (cfg->S != 4 && cfg->S != 8) { *why = "the persistent schedule runs strips of 4 or 8"; return RL_E_UNSUPPORTED; }
        // tiles whose data a tile's halo can reach, on each axis; a fold deeper than the
        // image can reach anywhere on that axis
        const rl::OpTable &v = cfg->conv, &c2 = cfg->corr;
        const int ha = std::max({-v.lane_min, v.lane_max, -c2.lane_min, c2.lane_max, 0});
        const int hb = std::max({-v.c_min, v.c_max, -c2.c_min, c2.c_max, 0});
        cfg->reach_a = ha >= la ? cfg->tiles_a : (ha + cfg->TA - 1) / cfg->TA;
        cfg->reach_b = hb >= lb ? cfg->tiles_b : (hb + cfg->TB - 1) / cfg->TB;
    }
    return RL_OK;
}

// The configuration chosen by the last rl_workspace_bytes call on this thread, reused by
// an rl_init with the same parameters and PSF: callers size the workspace first and then
// initialise, so each job runs the PSF compiler's search once.  The key is the parameter
// block with its pointers cleared, the PSF values and the tuning-cache generation (a
// change of the cache can change the choice).
std::atomic<uint64_t> g_tune_gen{0};
struct ConfigMemo {
    std::string key;
    Config cfg;
    bool valid = false;
};
thread_local ConfigMemo g_memo;

std::string config_key(const rl_params* p) {
    rl_params q = *p;
    q.f = nullptr;
    q.u0 = nullptr;
    q.psf = nullptr;
    q.stream = nullptr;
    const uint64_t gen = g_tune_gen.load();
    std::string k(reinterpret_cast<const char*>(&q), sizeof q);
    k.append(reinterpret_cast<const char*>(&gen), sizeof gen);
    k.append(reinterpret_cast<const char*>(p->psf), (size_t)p->psf_h * p->psf_w * sizeof(float));
    return k;
}

Layout make_layout(const rl_params* p, const Config& cfg) {
    Layout L{};
    const size_t N = (size_t)p->height * p->width;
    const bool thin = p->thin.mode != RL_THIN_OFF;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.f = take(N * 4);
    L.u = take(N * 4);
    L.r = take(N * 4);
    // the regions set from the host at rl_init (PSF tables, launch arguments, zeroed
    // counters) lie together, so that one copy uploads them all
    const size_t pad = 16;  // zero weights after the table (span kernel over-reads <= 15)
    // zero descriptors after each span table: the span and sliding kernels read up to
    // kSpanPad entries ahead
    L.conv_spans = take((cfg.conv.spans.size() + kSpanPad) * sizeof(DevSpan));
    L.conv_w = take((cfg.conv.w.size() + pad) * 4);
    L.corr_spans = take((cfg.corr.spans.size() + kSpanPad) * sizeof(DevSpan));
    L.corr_w = take((cfg.corr.w.size() + pad) * 4);
    if (cfg.kind == KIND_MFMA) {
        L.mf_conv = take(mfma_table_bytes(cfg.conv));
        L.mf_corr = take(mfma_table_bytes(cfg.corr));
    }
    L.ctr = take(C_COUNT * 8);
    L.args = take(2 * sizeof(PhaseArgs));
    L.fargs = take(sizeof(rlk::FusedArgs));
    L.prefix = take(2 * sizeof(int32_t));
    L.pctl = take(2 * sizeof(int32_t));  // persistent launches: ticket, abort flag
    L.blob_end = o;
    const size_t ntiles = (size_t)cfg.tiles_a * cfg.tiles_b;
    if (thin) {
        L.cnt = take(N);
        L.plist = take(N * 4);
        L.tflag = take(ntiles * 4);
        L.tlist = take(ntiles * 4);
        L.bcounts = take(thin_blocks(N) * 4);
        L.boffs = take(thin_blocks(N) * 4);
        L.sched = take(rlk::SCHED_RING * 8);
        L.act = take(2 * rlk::ACT_SLOTS * 4);
        const int lg = block_lg(p);
        L.cntb = lg ? take((size_t)block_count(p, lg)) : 0;  // block rule: one counter per block
    }
    L.u2 = cfg.kind == KIND_FUSED ? take(N * 4) : 0;
    L.red = take(rlk::RED_BLOCKS * 8);
    L.red_i = take(rlk::RED_BLOCKS * 8);
    L.done = cfg.sched == RL_SCHED_PERSISTENT ? take(ntiles * 4) : 0;
    const bool rob = p->rob_eps > 0.f;
    L.tvg = (p->tv_lambda > 0.f || rob) ? take(N * 4) : 0;  // TV factor or robust h^* * w
    L.wt = rob ? take(N * 4) : 0;                           // robust weights w
    L.total = o;
    return L;
}

rl_status validate_params(const rl_params* p, std::string* why) {
    if (!p) { *why = "NULL params"; return RL_E_INVAL; }
    if (p->height < 1 || p->width < 1) { *why = "image size must be >= 1"; return RL_E_INVAL; }
    if ((int64_t)p->height * p->width > (int64_t)1 << 30) { *why = "image too large"; return RL_E_INVAL; }
    if (p->boundary != RL_BC_REFLECT && p->boundary != RL_BC_REPLICATE) { *why = "boundary"; return RL_E_INVAL; }
    if (!(p->tv_lambda >= 0.f && p->tv_lambda < 0.25f)) { *why = "tv_lambda in [0, 0.25)"; return RL_E_INVAL; }
    if (p->tv_lambda > 0.f && !(p->tv_eps > 0.f && p->tv_eps < 1e30f)) { *why = "tv_eps > 0"; return RL_E_INVAL; }
    if (!(p->rob_eps >= 0.f && p->rob_eps < 1e18f)) { *why = "rob_eps >= 0 and finite"; return RL_E_INVAL; }
    if (p->thin.mode < RL_THIN_OFF || p->thin.mode > RL_THIN_REL) { *why = "thin mode"; return RL_E_INVAL; }
    if (p->thin.mode != RL_THIN_OFF) {
        if (!(p->thin.tau >= 0.f) || std::isinf(p->thin.tau)) { *why = "tau"; return RL_E_INVAL; }
        if (p->thin.hysteresis < 1 || p->thin.hysteresis > 255) { *why = "hysteresis in [1, 255]"; return RL_E_INVAL; }
        if (p->thin.reset_period < 0 || p->thin.compact_period < 0) { *why = "periods"; return RL_E_INVAL; }
        const int b = p->thin.block;
        if (!(b == 0 || b == 1 || b == 8 || b == 16 || b == 32 || b == 64)) {
            *why = "thin.block must be 0, 1, 8, 16, 32 or 64";
            return RL_E_INVAL;
        }
    }
    return RL_OK;
}

}  // namespace

struct rl_job {
    rl_params p;
    hipStream_t stream;
    int H, W;
    int64_t N;
    Config cfg;
    rl::CompiledPsf psf;
    Layout L;
    char* ws;
    int64_t k;
    bool list_valid;
    bool pending_finalize;  // thinned: the active count of iteration k - 1 is not folded yet
    bool live;
    std::vector<DevSpan> h_conv, h_corr;
    std::vector<float> h_conv_w, h_corr_w;
    std::vector<uint16_t> h_mf_conv, h_mf_corr;  // matrix-core weight operands (bf16 bits)
    PhaseArgs h_args[2];
    int32_t h_prefix[2];
    rlk::FusedArgs h_fargs;
    std::vector<char> h_blob;  // host image of [L.conv_spans, L.blob_end), uploaded by rl_init
    hipGraphExec_t graph = nullptr;  // captured chunk of graph_iters plain iterations
    int graph_n = 0;
    int graph_par = 0;  // parity of k the captured chunk starts at (fused schedule)
    bool persist_used = false;  // a persistent launch ran: check its abort flag
    // thinned jobs: asynchronous readback of the active-tile count after each rebuild
    int64_t* h_tcount = nullptr;  // pinned host word
    hipEvent_t tc_event = nullptr;
    bool tc_pending = false;
    int64_t tc_known = -1;        // last count that reached the host (-1: none yet)
    // the plane holding u^k: the fused schedule alternates between u and u2
    float* cur_u() const {
        return (cfg.kind == KIND_FUSED && (k & 1)) ? reinterpret_cast<float*>(ws + L.u2)
                                                   : reinterpret_cast<float*>(ws + L.u);
    }
    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

thread_local std::string g_last_error;

rl_status dev_err(hipError_t e, const char* what) {
    if (e == hipSuccess) return RL_OK;
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return RL_E_DEVICE;
}

// Raise a kernel's dynamic LDS limit once per device and size (the runtime call costs
// several microseconds, too much to repeat on every launch of a short kernel).
std::mutex g_lds_mu;
std::map<std::pair<int, const void*>, size_t> g_lds_set;

hipError_t allow_lds(const void* fn, size_t lds) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(g_lds_mu);
    size_t& have = g_lds_set[{dev, fn}];
    if (have >= lds) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) have = lds;
    return e;
}

template <typename... KArgs, typename... Args>
hipError_t launch(const char* name, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                  size_t lds, hipStream_t s, Args... args) {
    TimedLaunch tl;
    bool timed = false;
    {
        std::lock_guard<std::mutex> g(g_tmu);
        timed = g_timing;
    }
    if (lds > 64 * 1024) {
        hipError_t e = allow_lds(reinterpret_cast<const void*>(kernel), lds);
        if (e != hipSuccess) return e;
    }
    if (!timed) {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
        return hipGetLastError();
    }
    // Timed: the start and stop events travel with the dispatch packet itself
    // (hipExtLaunchKernel), so they bracket the kernel's execution and not the queueing of
    // separate event packets around it.
    (void)hipEventCreate(&tl.a);
    (void)hipEventCreate(&tl.b);
    std::tuple<KArgs...> targs(args...);
    void* argv[sizeof...(KArgs)];
    std::apply([&](auto&... a) {
        int i = 0;
        ((argv[i++] = static_cast<void*>(&a)), ...);
    }, targs);
    hipError_t e = hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv,
                                      lds, s, tl.a, tl.b, 0);
    tl.name = name;
    std::lock_guard<std::mutex> g(g_tmu);
    g_timed.push_back(tl);
    return e;
}

unsigned grid_for(int64_t n, int64_t per = 256, int64_t cap = 4096) {
    int64_t g = (n + per - 1) / per;
    return (unsigned)std::max<int64_t>(1, std::min(g, cap));
}

// ---- kernel instantiation tables --------------------------------------------------------
using PhaseFn = void (*)(rlk::LaunchArgs);

template <int O, int S, int NW, bool B>
PhaseFn span_fn(int lmax) {
    switch (lmax) {
        case 1: return rlk::span_kernel<O, S, 1, NW, B>;
        case 4: return rlk::span_kernel<O, S, 4, NW, B>;
        case 8: return rlk::span_kernel<O, S, 8, NW, B>;
        case 16: return rlk::span_kernel<O, S, 16, NW, B>;
    }
    return nullptr;
}

// nw = 4 (four-wavefront workgroups) exists for strips of 8 only
template <int O, bool B>
PhaseFn span_fn_s(int S, int lmax, int nw) {
    if (nw == 4) return S == 8 ? span_fn<O, 8, 4, B>(lmax) : nullptr;
    switch (S) {
        case 4: return span_fn<O, 4, kNW, B>(lmax);
        case 8: return span_fn<O, 8, kNW, B>(lmax);
        case 16: return span_fn<O, 16, kNW, B>(lmax);
    }
    return nullptr;
}

template <int O, bool B>
PhaseFn slide_fn(int S, int nw) {
    if (nw == 4) return S == 8 ? rlk::slide_kernel<O, 8, 4, B> : nullptr;
    switch (S) {
        case 4: return rlk::slide_kernel<O, 4, kNW, B>;
        case 8: return rlk::slide_kernel<O, 8, kNW, B>;
        case 16: return rlk::slide_kernel<O, 16, kNW, B>;
        case 32: return rlk::slide_kernel<O, 32, kNW, B>;
    }
    return nullptr;
}

using PersistFn = void (*)(rlk::PersistArgs);

template <int K, int O, int S, int NW>
PersistFn persist_fn_l(int lmax) {
    if (K == KIND_SLIDE) return rlk::persist_kernel<KIND_SLIDE, O, S, 1, NW>;
    switch (lmax) {
        case 1: return rlk::persist_kernel<KIND_SPAN, O, S, 1, NW>;
        case 4: return rlk::persist_kernel<KIND_SPAN, O, S, 4, NW>;
        case 8: return rlk::persist_kernel<KIND_SPAN, O, S, 8, NW>;
        case 16: return rlk::persist_kernel<KIND_SPAN, O, S, 16, NW>;
    }
    return nullptr;
}

template <int K, int O>
PersistFn persist_fn_s(int S, int lmax, int nw) {
    if (nw == 4) return S == 8 ? persist_fn_l<K, O, 8, 4>(lmax) : nullptr;
    switch (S) {
        case 4: return persist_fn_l<K, O, 4, kNW>(lmax);
        case 8: return persist_fn_l<K, O, 8, kNW>(lmax);
    }
    return nullptr;
}

PersistFn persist_fn(const Config& c) {
    if (c.kind == KIND_SPAN)
        return c.orient == rlk::ORIENT_ROWS ? persist_fn_s<KIND_SPAN, rlk::ORIENT_ROWS>(c.S, c.lmax, c.nw)
                                            : persist_fn_s<KIND_SPAN, rlk::ORIENT_COLS>(c.S, c.lmax, c.nw);
    return c.orient == rlk::ORIENT_ROWS ? persist_fn_s<KIND_SLIDE, rlk::ORIENT_ROWS>(c.S, 0, c.nw)
                                        : persist_fn_s<KIND_SLIDE, rlk::ORIENT_COLS>(c.S, 0, c.nw);
}

// Workgroups of a persistent kernel that the device holds at once.
int persist_capacity(PersistFn fn, size_t lds, int threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (lds > 64 * 1024) (void)allow_lds(reinterpret_cast<const void*>(fn), lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                     threads, lds) != hipSuccess)
        return 0;
    return std::max(1, per_cu) * std::max(1, cus);
}

constexpr int kSpinLimit = 1 << 20;  // polls (about a second) before a persistent launch gives up
std::atomic<int> g_spin_limit{kSpinLimit};  // rl_debug_spin_limit changes it for tests

// After a persistent launch: read its sticky abort flag (synchronises the job's stream).
rl_status check_persist_abort(rl_job* j, hipStream_t s);

PhaseFn phase_fn(const Config& c, bool phase_b) {
    if (c.kind == KIND_MFMA) {
        if (c.nw == 8) return phase_b ? rlk::mfma_kernel<8, true> : rlk::mfma_kernel<8, false>;
        return phase_b ? rlk::mfma_kernel<4, true> : rlk::mfma_kernel<4, false>;
    }
    if (c.kind == KIND_RECT) {
        if (c.S == 4) return phase_b ? rlk::rect_kernel<4, kNW, true> : rlk::rect_kernel<4, kNW, false>;
        if (c.S == 8) return phase_b ? rlk::rect_kernel<8, kNW, true> : rlk::rect_kernel<8, kNW, false>;
        return nullptr;
    }
    if (c.kind == KIND_SAT) {
        if (c.S == 4) return phase_b ? rlk::sat_kernel<4, kNW, true> : rlk::sat_kernel<4, kNW, false>;
        if (c.S == 8) return phase_b ? rlk::sat_kernel<8, kNW, true> : rlk::sat_kernel<8, kNW, false>;
        return nullptr;
    }
    if (c.kind == KIND_SPAN) {
        if (c.orient == rlk::ORIENT_ROWS)
            return phase_b ? span_fn_s<rlk::ORIENT_ROWS, true>(c.S, c.lmax, c.nw)
                           : span_fn_s<rlk::ORIENT_ROWS, false>(c.S, c.lmax, c.nw);
        return phase_b ? span_fn_s<rlk::ORIENT_COLS, true>(c.S, c.lmax, c.nw)
                       : span_fn_s<rlk::ORIENT_COLS, false>(c.S, c.lmax, c.nw);
    }
    if (c.orient == rlk::ORIENT_ROWS)
        return phase_b ? slide_fn<rlk::ORIENT_ROWS, true>(c.S, c.nw) : slide_fn<rlk::ORIENT_ROWS, false>(c.S, c.nw);
    return phase_b ? slide_fn<rlk::ORIENT_COLS, true>(c.S, c.nw) : slide_fn<rlk::ORIENT_COLS, false>(c.S, c.nw);
}

const char* phase_name(const Config& c, bool phase_b) {
    if (c.kind == KIND_MFMA) return phase_b ? "mfma_corr_update" : "mfma_conv_ratio";
    if (c.kind == KIND_RECT) return phase_b ? "rect_corr_update" : "rect_conv_ratio";
    if (c.kind == KIND_SAT) return phase_b ? "sat_corr_update" : "sat_conv_ratio";
    if (c.kind == KIND_SPAN)
        return phase_b ? (c.lmax == 1 ? "direct_corr_update" : "span_corr_update")
                       : (c.lmax == 1 ? "direct_conv_ratio" : "span_conv_ratio");
    return phase_b ? "slide_corr_update" : "slide_conv_ratio";
}

using ResFn = void (*)(ResidentArgs);
ResFn resident_fn(int orient, int seg) {
#define RL_RES(O)                                              \
    switch (seg) {                                             \
        case 2: return rlk::resident_kernel<O, 2>;             \
        case 4: return rlk::resident_kernel<O, 4>;             \
        case 8: return rlk::resident_kernel<O, 8>;             \
        case 16: return rlk::resident_kernel<O, 16>;           \
        case 32: return rlk::resident_kernel<O, 32>;           \
    }
    if (orient == rlk::ORIENT_ROWS) { RL_RES(rlk::ORIENT_ROWS) }
    else { RL_RES(rlk::ORIENT_COLS) }
#undef RL_RES
    return nullptr;
}

using ResMultiFn = void (*)(const ResidentArgs*, const int32_t*, int);
ResMultiFn resident_multi_fn(int orient, int seg) {
#define RL_RES(O)                                              \
    switch (seg) {                                             \
        case 2: return rlk::resident_multi_kernel<O, 2>;       \
        case 4: return rlk::resident_multi_kernel<O, 4>;       \
        case 8: return rlk::resident_multi_kernel<O, 8>;       \
        case 16: return rlk::resident_multi_kernel<O, 16>;     \
        case 32: return rlk::resident_multi_kernel<O, 32>;     \
    }
    if (orient == rlk::ORIENT_ROWS) { RL_RES(rlk::ORIENT_ROWS) }
    else { RL_RES(rlk::ORIENT_COLS) }
#undef RL_RES
    return nullptr;
}

// Device table entry of one phase of a job (base iteration index k0).
PhaseArgs phase_args(rl_job* j, bool phase_b, int64_t k0) {
    PhaseArgs a{};
    const Config& c = j->cfg;
    const rl::OpTable& t = phase_b ? c.corr : c.conv;
    a.H = j->H;
    a.W = j->W;
    a.bc = j->p.boundary;
    a.kahan = j->p.kahan;
    a.src = phase_b ? j->at<float>(j->L.r) : j->at<float>(j->L.u);
    a.f = j->at<float>(j->L.f);
    a.r = j->at<float>(j->L.r);
    a.u = j->at<float>(j->L.u);
    a.spans = phase_b ? j->at<DevSpan>(j->L.corr_spans) : j->at<DevSpan>(j->L.conv_spans);
    a.wts = phase_b ? j->at<float>(j->L.corr_w) : j->at<float>(j->L.conv_w);
    if (c.kind == KIND_MFMA)  // the banded bfloat16 weight operands
        a.wts = phase_b ? j->at<float>(j->L.mf_corr) : j->at<float>(j->L.mf_conv);
    a.n_spans = (int32_t)t.spans.size();
    a.lane_min = t.lane_min;
    a.lane_max = t.lane_max;
    a.c_min = t.c_min;
    a.c_max = t.c_max;
    a.tiles_a = c.tiles_a;
    a.tiles_b = c.tiles_b;
    a.k = k0;
    a.full = 1;
    a.list_ok = 1;
    // robust variant: phase A stores v (the r plane), phase B divides by h^* * w
    a.tvg = (phase_b && (j->p.tv_lambda > 0.f || j->p.rob_eps > 0.f)) ? j->at<float>(j->L.tvg)
                                                                      : nullptr;
    a.store = (!phase_b && j->p.rob_eps > 0.f) ? j->at<float>(j->L.r) : nullptr;
    // the sliding kernel's exact-zero witness: the longest run, if it covers a strip
    a.wit = -1;
    if (c.kind == KIND_SLIDE) {
        int best = 0;
        for (size_t i = 0; i < t.spans.size(); ++i)
            if (t.spans[i].len >= c.S && t.spans[i].len > best) {
                best = t.spans[i].len;
                a.wit = (int32_t)i;
            }
    }
    if (j->p.thin.mode != RL_THIN_OFF) {
        const int lg = block_lg(&j->p);
        a.cnt = lg ? j->at<uint8_t>(j->L.cntb) : j->at<uint8_t>(j->L.cnt);
        a.blk_lg = lg;
        a.blk_w = lg ? (int32_t)block_cols(&j->p, lg) : 0;
        a.tflag = lg ? j->at<int32_t>(j->L.tflag) : nullptr;
        a.thin_mode = j->p.thin.mode;
        a.hyst = j->p.thin.hysteresis;
        a.reset_period = j->p.thin.reset_period;
        a.tau = j->p.thin.tau;
        a.sched = j->at<int64_t>(j->L.sched);
        a.active_total = j->at<int64_t>(j->L.ctr) + C_ACTIVE_TOTAL;
        a.act_part = j->at<int32_t>(j->L.act);
        a.tile_list = j->at<int32_t>(j->L.tlist);
        a.tile_count = j->at<int64_t>(j->L.ctr) + C_TLIST_LEN;
    }
    return a;
}

// Block rule: write every pixel's counter (its block's) to dst (N bytes, device).
rl_status expand_blocks(rl_job* j, uint8_t* dst, hipStream_t s) {
    const int lg = block_lg(&j->p);
    return dev_err(launch("block_expand", rlk::block_expand_kernel, dim3(grid_for(j->N)), dim3(256), 0, s,
                          (const uint8_t*)j->at<uint8_t>(j->L.cntb), dst, j->N, j->W, lg,
                          (int)block_cols(&j->p, lg)), "block expand");
}

rl_status rebuild_lists(rl_job* j, hipStream_t s) {
    rlk::ThinListArgs a{};
    a.cnt = j->at<uint8_t>(j->L.cnt);
    a.N = j->N;
    a.W = j->W;
    a.hyst = j->p.thin.hysteresis;
    a.orient = j->cfg.orient;
    a.tiles_a = j->cfg.tiles_a;
    a.TA = j->cfg.TA;
    a.TB = j->cfg.TB;
    a.block_counts = j->at<int32_t>(j->L.bcounts);
    a.block_offsets = j->at<int32_t>(j->L.boffs);
    a.tflag = j->at<int32_t>(j->L.tflag);
    a.plist = j->at<int32_t>(j->L.plist);
    a.plist_len = j->at<int64_t>(j->L.ctr) + C_PLIST_LEN;
    const int nb = (int)thin_blocks(j->N);
    a.n_blocks = nb;
    rl_status st;
    int ntiles = j->cfg.tiles_a * j->cfg.tiles_b;
    const bool blk = block_lg(&j->p) > 0;
    if (blk) {
        // block rule: the phase-B kernels keep every tile's flag up to date, so the list is
        // compacted straight from the flags; the per-pixel list is built only when kept
        // (from the expanded counters; thin_count then sets flags that are already set)
        if (j->p.thin.keep_list) {
            if ((st = expand_blocks(j, j->at<uint8_t>(j->L.cnt), s))) return st;
            if ((st = dev_err(launch("thin_count", rlk::thin_count_kernel, dim3(nb), dim3(256), 0, s, a), "thin_count"))) return st;
        }
    } else if ((st = dev_err(launch("thin_count", rlk::thin_count_kernel, dim3(nb), dim3(256), 0, s, a), "thin_count"))) {
        return st;
    }
    if (j->p.thin.keep_list) {
        if ((st = dev_err(launch("thin_scan", rlk::scan_counts_kernel, dim3(1), dim3(1024), 0, s,
                                 (const int32_t*)a.block_counts, a.block_offsets, nb, a.plist_len), "thin_scan"))) return st;
        if ((st = dev_err(launch("thin_scatter", rlk::thin_scatter_kernel, dim3(nb), dim3(256), 0, s, a), "thin_scatter"))) return st;
    }
    int64_t* tcount = j->at<int64_t>(j->L.ctr) + C_TLIST_LEN;
    if ((st = dev_err(launch("tile_compact", rlk::tile_compact_kernel, dim3(1), dim3(1024), 0, s,
                             a.tflag, ntiles, j->at<int32_t>(j->L.tlist), tcount, blk ? 0 : 1), "tile_compact"))) return st;
    j->list_valid = true;
    // Read the active-tile count back without waiting: a later iteration uses it (once the
    // copy has landed) to skip the tile list when nearly every tile is active.
    if (j->h_tcount && j->tc_event) {
        hipError_t e = hipMemcpyAsync(j->h_tcount, tcount, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(j->tc_event, s);
        if ((st = dev_err(e, "tile count readback"))) return st;
        j->tc_pending = true;
    }
    return RL_OK;
}

// Whether non-full thinned steps should go through the tile list: yes unless the last
// active-tile count that has reached the host shows (almost) every tile active, in which
// case all tiles run and the per-pixel test in the epilogue alone skips frozen pixels
// (the same arithmetic either way).
bool use_tile_list(rl_job* j) {
    if (j->tc_pending && hipEventQuery(j->tc_event) == hipSuccess) {
        j->tc_known = *j->h_tcount;
        j->tc_pending = false;
    }
    const int64_t ntiles = (int64_t)j->cfg.tiles_a * j->cfg.tiles_b;
    return j->tc_known < 0 || j->tc_known * 10 < ntiles * 9;
}

// TV-regularised jobs: the update's denominator from u^k, before phase A of an iteration
// (phase B overwrites u^k).
rl_status enqueue_tv(rl_job* j, hipStream_t s) {
    if (!(j->p.tv_lambda > 0.f)) return RL_OK;
    return dev_err(launch("tv_factor", rlk::tv_factor_kernel, dim3(grid_for(j->N, 256, 4096)),
                          dim3(256), 0, s, (const float*)j->at<float>(j->L.u),
                          j->at<float>(j->L.tvg), j->H, j->W, j->p.tv_lambda, j->p.tv_eps),
                   "tv_factor");
}

rl_status enqueue_iterations(rl_job* j, int32_t n);
rl_status enqueue_direct(rl_job* j, int32_t n);

// Capture n plain iterations of a tiled job into an executable graph (kernel nodes only),
// on a private stream so the caller's stream is not put into capture mode.
rl_status capture_graph(rl_job* j, int n) {
    hipStream_t cs;
    rl_status st = dev_err(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
    if (st) return st;
    bool timing;
    {
        std::lock_guard<std::mutex> g(g_tmu);
        timing = g_timing;
        g_timing = false;  // no event records inside the graph
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipStream_t keep = j->stream;
        const int64_t k0 = j->k;
        j->stream = cs;
        st = enqueue_direct(j, n);
        j->stream = keep;
        j->k = k0;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (st == RL_OK) st = dev_err(e2, "end capture");
    } else {
        st = dev_err(e, "begin capture");
    }
    if (st == RL_OK) {
        st = dev_err(hipGraphInstantiate(&j->graph, graph, nullptr, nullptr, 0), "instantiate");
        if (st) j->graph = nullptr;
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    {
        std::lock_guard<std::mutex> g(g_tmu);
        g_timing = timing;
    }
    if (st == RL_OK) j->graph_n = n;
    return st;
}

// Arguments of n resident iterations of a job (KIND_RESIDENT).
ResidentArgs resident_args(const rl_job* j, int32_t n) {
    const Config& c = j->cfg;
    ResidentArgs a{};
    a.H = j->H;
    a.W = j->W;
    a.bc = j->p.boundary;
    a.kahan = j->p.kahan;
    a.u = j->at<float>(j->L.u);
    a.f = j->at<float>(j->L.f);
    a.n_iter = n;
    a.lines_per_wg = c.lines_per_wg;
    a.wpl = c.wpl;
    a.conv_c0 = j->psf.box_c0;
    a.len = j->psf.box_len;
    // adjoint window = mirror of the forward window
    a.corr_c0 = -(j->psf.box_c0 + j->psf.box_len - 1);
    a.w = j->psf.box_w;
    a.halo = j->psf.box_len - 1;
    a.line_words = c.line_words;
    return a;
}

int32_t resident_workgroups(const Config& c) {
    return (int32_t)((c.lines + c.lines_per_wg - 1) / c.lines_per_wg);
}

rl_status enqueue_iterations(rl_job* j, int32_t n) {
    const Config& c = j->cfg;
    hipStream_t s = j->stream;
    if (c.kind == KIND_RESIDENT) {
        if (n == 0) return RL_OK;
        const ResidentArgs a = resident_args(j, n);
        unsigned grid = (unsigned)resident_workgroups(c);
        unsigned block = (unsigned)(c.lines_per_wg * 64 * c.wpl);
        rl_status st = dev_err(launch("resident_box", resident_fn(c.orient, c.seg), dim3(grid),
                                      dim3(block), c.lds_a, s, a), "resident_box");
        if (st) return st;
        j->k += n;
        return RL_OK;
    }
    const bool thin = j->p.thin.mode != RL_THIN_OFF;
    const int gi = j->p.tuning.graph_iters;
    if (!thin && gi > 0 && n >= gi) {
        // Plain jobs: the launch sequence of the two-pass schedule does not depend on k,
        // and the fused kernel only uses the parity of k (which plane holds u^k), so one
        // captured chunk can be replayed at any k of the captured parity; fused chunks
        // have an even length, which keeps that parity.
        if (!j->graph) {
            const int gn = c.kind == KIND_FUSED ? (gi + 1) & ~1 : gi;
            rl_status st = capture_graph(j, gn);
            if (st) return st;
            j->graph_par = (int)(j->k & 1);
        }
        if (c.kind == KIND_FUSED && (int)(j->k & 1) != j->graph_par) {
            rl_status st = enqueue_direct(j, 1);
            if (st) return st;
            --n;
        }
        while (j->graph && j->graph_n > 0 && n >= j->graph_n) {
            rl_status st = dev_err(hipGraphLaunch(j->graph, s), "graph launch");
            if (st) return st;
            j->k += j->graph_n;
            n -= j->graph_n;
        }
    }
    return enqueue_direct(j, n);
}

// Launch n iterations of a tiled or fused job one kernel at a time.
rl_status enqueue_direct(rl_job* j, int32_t n) {
    const Config& c = j->cfg;
    hipStream_t s = j->stream;
    if (c.sched == RL_SCHED_PERSISTENT) {
        if (n == 0) return RL_OK;
        const int ntiles = c.tiles_a * c.tiles_b;
        int32_t* done = j->at<int32_t>(j->L.done);
        int32_t* pctl = j->at<int32_t>(j->L.pctl);
        rl_status st = dev_err(launch("fill", rlk::fill_u32_kernel, dim3(grid_for(ntiles)), dim3(256), 0,
                                      s, (uint32_t*)done, 0u, (int64_t)ntiles), "fill");
        if (st) return st;
        // the ticket starts at 0; the abort flag (pctl[1]) is sticky for the job's life
        st = dev_err(launch("fill", rlk::fill_u32_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)pctl,
                            0u, (int64_t)1), "fill");
        if (st) return st;
        rlk::PersistArgs P{};
        P.jobs = nullptr;
        P.prefix = nullptr;
        P.n_jobs = 1;
        P.total_tiles = ntiles;
        P.max_steps = 2 * n;
        P.spin_limit = g_spin_limit.load();
        P.ticket = pctl;
        P.abort = pctl + 1;
        P.one.a = phase_args(j, false, j->k);
        P.one.b = phase_args(j, true, j->k);
        P.one.done = done;
        P.one.n_steps = 2 * n;
        P.one.reach_a = c.reach_a;
        P.one.reach_b = c.reach_b;
        PersistFn fn = persist_fn(c);
        if (!fn) return RL_E_UNSUPPORTED;
        const size_t lds = std::max(c.lds_a, c.lds_b);
        const int64_t tasks = (int64_t)2 * n * ntiles;
        if (tasks > ((int64_t)1 << 30)) return RL_E_UNSUPPORTED;
        const int cap = persist_capacity(fn, lds, c.threads);
        if (cap <= 0) return RL_E_DEVICE;
        const unsigned grid = (unsigned)std::min<int64_t>(cap, tasks);
        st = dev_err(launch(c.kind == KIND_SLIDE ? "persist_slide" : "persist_span", fn, dim3(grid),
                            dim3(c.threads), lds, s, P), "persistent");
        if (st) return st;
        j->k += n;
        j->persist_used = true;
        return RL_OK;
    }
    if (c.kind == KIND_FUSED) {
        const rlk::FusedArgs* table = j->at<rlk::FusedArgs>(j->L.fargs);
        for (int i = 0; i < n; ++i) {
            rl_status st = dev_err(launch("fused_iteration", rlk::fused_kernel<8, 16, kNW>,
                                          dim3(c.tiles_a * c.tiles_b), dim3(kNW * 64), c.lds_a,
                                          s, table, (int64_t)j->k), "fused");
            if (st) return st;
            j->k += 1;
        }
        return RL_OK;
    }
    const bool thin = j->p.thin.mode != RL_THIN_OFF;
    const int ntiles = c.tiles_a * c.tiles_b;
    PhaseFn fa = phase_fn(c, false), fb = phase_fn(c, true);
    const char* na = phase_name(c, false);
    const char* nbn = phase_name(c, true);
    rlk::LaunchArgs la{}, lb{};
    la.table = j->at<PhaseArgs>(j->L.args);
    lb.table = la.table + 1;
    la.prefix = lb.prefix = j->at<int32_t>(j->L.prefix);
    la.n_jobs = lb.n_jobs = 1;
    la.one = j->h_args[0];
    lb.one = j->h_args[1];
    for (int i = 0; i < n; ++i) {
        if (thin && !is_full(j->k, j->p.thin.reset_period) &&
            (!j->list_valid ||
             is_rebuild(j->k, j->p.thin.reset_period, j->p.thin.compact_period))) {
            rl_status st = rebuild_lists(j, s);
            if (st) return st;
        }
        la.kb = lb.kb = j->k;
        if (thin) {
            la.one.list_ok = lb.one.list_ok = use_tile_list(j) ? 1 : 0;
            la.one.full = lb.one.full = is_full(j->k, j->p.thin.reset_period) ? 1 : 0;
        }
        if (rl_status tst = enqueue_tv(j, s)) return tst;
        rl_status st = dev_err(launch(na, fa, dim3(ntiles), dim3(c.threads), c.lds_a, s, la), na);
        if (st) return st;
        if (j->p.rob_eps > 0.f) {
            // robust variant: weights and weighted ratio from v, then h^* * w into the
            // denominator plane, then the update's correlation
            float* r = j->at<float>(j->L.r);
            float* wt = j->at<float>(j->L.wt);
            st = dev_err(launch("robust_weights", rlk::robust_weights_kernel,
                                dim3(grid_for(j->N, 256, 4096)), dim3(256), 0, s, r,
                                (const float*)j->at<float>(j->L.f), wt, (int64_t)j->N,
                                j->p.rob_eps * j->p.rob_eps), "robust_weights");
            if (st) return st;
            rlk::LaunchArgs lw = lb;
            lw.one.src = wt;
            lw.one.store = j->at<float>(j->L.tvg);
            lw.one.tvg = nullptr;
            st = dev_err(launch(nbn, fb, dim3(ntiles), dim3(c.threads), c.lds_b, s, lw), nbn);
            if (st) return st;
        }
        st = dev_err(launch(nbn, fb, dim3(ntiles), dim3(c.threads), c.lds_b, s, lb), nbn);
        if (st) return st;
        j->k += 1;
        if (thin) j->pending_finalize = true;
    }
    return RL_OK;
}

// Fold the active count of the last thinned iteration into the schedule (the next
// iteration's phase A would otherwise do it).
rl_status finalize_thin(rl_job* j, hipStream_t s) {
    if (!j->pending_finalize || j->p.thin.mode == RL_THIN_OFF || j->k == 0) return RL_OK;
    rl_status st = dev_err(launch("thin_finalize", rlk::thin_finalize_kernel, dim3(1), dim3(64), 0, s,
                                  j->at<int32_t>(j->L.act), j->at<int64_t>(j->L.sched),
                                  j->at<int64_t>(j->L.ctr) + C_ACTIVE_TOTAL, j->k - 1), "finalize");
    if (st) return st;
    j->pending_finalize = false;
    return RL_OK;
}

// Library-internal streams (non-blocking, default priority) on which independent groups
// of a batch run concurrently; forked from and joined back to the caller's stream with
// events.
constexpr int kSideStreams = 8;
std::mutex g_smu;
hipStream_t g_side[kSideStreams] = {};
hipEvent_t g_fork = nullptr;
hipEvent_t g_join[kSideStreams] = {};

// Side streams the batch spreads its kernel groups over.
constexpr int kBatchStreams = 8;
static_assert(kBatchStreams <= kSideStreams, "batch streams");

// Estimated microseconds per output of a two-pass phase launch per unit of this cost (the
// span_cost units), and per launch, from launch times measured at 1024^2 and 2048^2.
double unit_cost(const Config& c) {
    switch (c.kind) {
        case KIND_SPAN: return span_cost(c.conv, c.S, c.lmax, true);
        case KIND_SLIDE: return slide_cost(c.conv, c.S, true);
        case KIND_MFMA: return mfma_cost(c.conv);
        default: return 40.0;
    }
}

// Estimated microseconds of a job's launches outside the tiled groups: resident lines
// (about 4.2 ns per pixel-iteration at 1 Mpx), fused and robust jobs as two-pass ones.
double resident_work_us(const rl_job* j, int32_t n) {
    if (j->cfg.kind == KIND_RESIDENT) return 10.0 + 4.2e-6 * (double)j->N * n;
    return n * (20.0 + 5.8e-8 * 60.0 * (double)j->N);
}

rl_status side_streams(int n) {
    std::lock_guard<std::mutex> lk(g_smu);
    rl_status st;
    if (!g_fork && (st = dev_err(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming), "event"))) return st;
    for (int i = 0; i < n && i < kSideStreams; ++i) {
        if (!g_side[i] && (st = dev_err(hipStreamCreateWithFlags(&g_side[i], hipStreamNonBlocking), "stream"))) return st;
        if (!g_join[i] && (st = dev_err(hipEventCreateWithFlags(&g_join[i], hipEventDisableTiming), "event"))) return st;
    }
    return RL_OK;
}

// ---- pinned staging for host-to-device table uploads (rl_init, rl_iterate_batch) ------
// A copy from pageable host memory may make the host wait for the stream: with a batch in
// flight, creating the next batch's jobs would stall until the device drains, and the
// device would then idle while the host sets the rest up.  The upload therefore goes
// through pinned buffers, kept for reuse in upload order; a buffer is reused once the event
// recorded after its copy has completed.  Buffers live until the process ends (at most
// kPinCap bytes in all); beyond that, or if pinned memory is refused, the pageable copy
// is used.
struct PinBuf {
    char* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    int dev = -1;
};
std::mutex g_pin_mu;
std::deque<PinBuf> g_pin;  // oldest upload first
size_t g_pin_bytes = 0;
constexpr size_t kPinCap = size_t(256) << 20;
constexpr size_t kPinMin = size_t(64) << 10;

// Copy bytes from src to device address dst on stream s through a pinned buffer; false if
// no buffer could be had (nothing was enqueued then).
bool staged_upload(void* dst, const void* src, size_t bytes, hipStream_t s, hipError_t* err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    PinBuf b;
    bool found = false;
    // the oldest few buffers are the likeliest to be free
    for (size_t i = 0; i < g_pin.size() && i < 4; ++i) {
        PinBuf& c = g_pin[i];
        if (c.dev == dev && c.cap >= bytes && hipEventQuery(c.done) == hipSuccess) {
            b = c;
            g_pin.erase(g_pin.begin() + (std::ptrdiff_t)i);
            found = true;
            break;
        }
    }
    if (!found) {
        const size_t cap = std::max(kPinMin, (bytes + kPinMin - 1) / kPinMin * kPinMin);
        if (g_pin_bytes + cap > kPinCap) return false;
        if (hipHostMalloc((void**)&b.host, cap, hipHostMallocDefault) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(b.host);
            return false;
        }
        b.cap = cap;
        b.dev = dev;
        g_pin_bytes += cap;
    }
    std::memcpy(b.host, src, bytes);
    hipError_t e = hipMemcpyAsync(dst, b.host, bytes, hipMemcpyHostToDevice, s);
    *err = e;
    if (e != hipSuccess) {
        g_pin.push_back(b);  // nothing in flight: the event still reports its last state
        return true;
    }
    e = hipEventRecord(b.done, s);
    *err = e;
    // a copy in flight without its event could not be told apart from a finished one: such
    // a buffer is not reused
    if (e == hipSuccess) g_pin.push_back(b);
    return true;
}

struct BatchStage {
    std::vector<char> host;
    hipEvent_t done = nullptr;
    bool pending = false;
};
std::mutex g_bmu;
std::map<void*, BatchStage> g_stage;

// Upper bound of the batch tables: per group two PhaseArgs arrays and a prefix array,
// each 256-byte aligned; at most one group per job.
size_t batch_bytes(int32_t n_jobs) {
    return (size_t)n_jobs * (2 * sizeof(PhaseArgs) + 3 * kAlign + 2 * sizeof(int32_t)) + kAlign;
}

std::vector<DevSpan> to_dev(const rl::OpTable& t) {
    std::vector<DevSpan> v(t.spans.size());
    if (!t.spans.empty()) std::memcpy(v.data(), t.spans.data(), v.size() * sizeof(DevSpan));
    if (v.empty()) v.resize(1);
    return v;
}

rl_status check_persist_abort(rl_job* j, hipStream_t s) {
    int32_t flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, j->at<int32_t>(j->L.pctl) + 1, sizeof flag,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (rl_status st = dev_err(e, "read abort flag")) return st;
    if (flag) {
        g_last_error = "a persistent launch exceeded its wait limit; the result is incomplete";
        return RL_E_DEVICE;
    }
    return RL_OK;
}

}  // namespace

namespace {  // autotuner helpers

// Candidate (schedule, tuning) pairs for a job's kernel family.
std::vector<TuneEntry> tune_candidates(const rl_params* p, const Config& base) {
    std::vector<TuneEntry> v;
    auto add = [&](int sched, int strip, int seg, int lpw, int gi) {
        TuneEntry e{};
        e.schedule = p->schedule == RL_SCHED_AUTO ? sched : p->schedule;
        e.t.strip = strip;
        e.t.seg = seg;
        e.t.lines_per_wg = lpw;
        e.t.graph_iters = gi;
        v.push_back(e);
    };
    const bool thin = p->thin.mode != RL_THIN_OFF;
    if (base.kind == KIND_RESIDENT) {
        for (int seg : {4, 8, 16})
            for (int lpw : {1, 2, 4}) add(RL_SCHED_RESIDENT, 0, seg, lpw, 0);
        return v;
    }
    const int gi = thin ? 0 : 16;
    if (base.kind == KIND_MFMA) {  // no strip length to choose
        add(RL_SCHED_TWO_PASS, 0, 0, 0, 0);
        if (gi) add(RL_SCHED_TWO_PASS, 0, 0, 0, gi);
        return v;
    }
    for (int strip : {4, 8, 16}) {
        add(RL_SCHED_TWO_PASS, strip, 0, 0, 0);
        if (gi) add(RL_SCHED_TWO_PASS, strip, 0, 0, gi);
    }
    if (base.kind == KIND_SLIDE) add(RL_SCHED_TWO_PASS, 32, 0, 0, gi);
    if (!thin && p->schedule == RL_SCHED_AUTO) {
        add(RL_SCHED_FUSED, 0, 0, 0, 0);
        add(RL_SCHED_FUSED, 0, 0, 0, gi);
    }
    return v;
}

rl_params with_entry(const rl_params* p, const TuneEntry& e) {
    rl_params q = *p;
    q.tuning = e.t;
    q.schedule = e.schedule;
    return q;
}

}  // namespace

extern "C" {

const char* rl_status_str(rl_status s) {
    switch (s) {
        case RL_OK: return "RL_OK";
        case RL_E_INVAL: return "RL_E_INVAL";
        case RL_E_NOMEM: return "RL_E_NOMEM";
        case RL_E_DEVICE: return "RL_E_DEVICE";
        case RL_E_STATE: return "RL_E_STATE";
        case RL_E_UNSUPPORTED: return "RL_E_UNSUPPORTED";
    }
    return "RL_E_UNKNOWN";
}

const char* rl_last_error(void) { return g_last_error.c_str(); }

rl_status rl_workspace_bytes(const rl_params* p, size_t* bytes) {
    std::string why;
    if (!bytes) return RL_E_INVAL;
    rl_status st = validate_params(p, &why);
    if (st) return st;
    rl::CompiledPsf c;
    if (!rl::compile_psf(p->psf, p->psf_h, p->psf_w, &c, &why)) return RL_E_INVAL;
    Config cfg;
    st = choose_config(p, c, &cfg, &why);
    if (st) return st;
    *bytes = make_layout(p, cfg).total;
    g_memo.key = config_key(p);
    g_memo.cfg = std::move(cfg);
    g_memo.valid = true;
    return RL_OK;
}

}  // extern "C"

namespace {

// rl_init's body.  no_alloc: no pinned host word and no event for the asynchronous
// active-tile count (the tile list is then always used), so that set-up performs no
// allocation at all (rl_solve_static).
rl_status init_job(const rl_params* p, void* ws, size_t ws_bytes, rl_job** out, bool no_alloc) {
    std::string& why = g_last_error;  // reasons of rejections are kept for rl_last_error
    why.clear();
    if (!out || !ws) return RL_E_INVAL;
    *out = nullptr;
    rl_status st = validate_params(p, &why);
    if (st) return st;
    if (!p->f) return RL_E_INVAL;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return RL_E_INVAL;
    rl::CompiledPsf c;
    if (!rl::compile_psf(p->psf, p->psf_h, p->psf_w, &c, &why)) return RL_E_INVAL;
    rl_job* j = new (std::nothrow) rl_job();
    if (!j) return RL_E_NOMEM;
    j->p = *p;
    j->p.psf = nullptr;
    j->stream = reinterpret_cast<hipStream_t>(p->stream);
    j->H = p->height;
    j->W = p->width;
    j->N = (int64_t)p->height * p->width;
    j->psf = c;
    j->k = 0;
    j->list_valid = false;
    j->pending_finalize = false;
    j->live = true;
    if (g_memo.valid && g_memo.key == config_key(p)) {
        j->cfg = g_memo.cfg;
    } else {
        st = choose_config(p, c, &j->cfg, &why);
        if (st) { delete j; return st; }
    }
    j->L = make_layout(p, j->cfg);
    if (ws_bytes < j->L.total) { delete j; return RL_E_NOMEM; }
    j->ws = static_cast<char*>(ws);
    hipStream_t s = j->stream;
    // compiled PSF tables -> workspace (host copies stay alive in the job)
    j->h_conv = to_dev(j->cfg.conv);
    j->h_corr = to_dev(j->cfg.corr);
    j->h_conv.resize(j->h_conv.size() + kSpanPad, DevSpan{});
    j->h_corr.resize(j->h_corr.size() + kSpanPad, DevSpan{});
    j->h_conv_w = j->cfg.conv.w;
    j->h_conv_w.resize(j->h_conv_w.size() + 16, 0.f);
    j->h_corr_w = j->cfg.corr.w;
    j->h_corr_w.resize(j->h_corr_w.size() + 16, 0.f);
    if (j->cfg.kind == KIND_MFMA) {
        j->h_mf_conv = mfma_table(j->cfg.conv);
        j->h_mf_corr = mfma_table(j->cfg.corr);
    }
    if (j->cfg.kind == KIND_FUSED) {
        rlk::FusedArgs& a = j->h_fargs;
        a = rlk::FusedArgs{};
        a.H = j->H;
        a.W = j->W;
        a.bc = p->boundary;
        a.kahan = p->kahan;
        a.f = j->at<float>(j->L.f);
        a.u0 = j->at<float>(j->L.u);
        a.u1 = j->at<float>(j->L.u2);
        a.cspans = j->at<DevSpan>(j->L.conv_spans);
        a.cwts = j->at<float>(j->L.conv_w);
        a.rspans = j->at<DevSpan>(j->L.corr_spans);
        a.rwts = j->at<float>(j->L.corr_w);
        a.n_cspans = (int32_t)j->cfg.conv.spans.size();
        a.n_rspans = (int32_t)j->cfg.corr.spans.size();
        a.vl_min = j->cfg.conv.lane_min; a.vl_max = j->cfg.conv.lane_max;
        a.vc_min = j->cfg.conv.c_min; a.vc_max = j->cfg.conv.c_max;
        a.cl_min = j->cfg.corr.lane_min; a.cl_max = j->cfg.corr.lane_max;
        a.cc_min = j->cfg.corr.c_min; a.cc_max = j->cfg.corr.c_max;
        a.tiles_a = j->cfg.tiles_a;
        a.tiles_b = j->cfg.tiles_b;
        a.k = 0;
    } else if (j->cfg.kind != KIND_RESIDENT) {
        j->h_args[0] = phase_args(j, false, 0);
        j->h_args[1] = phase_args(j, true, 0);
        j->h_prefix[0] = 0;
        j->h_prefix[1] = j->cfg.tiles_a * j->cfg.tiles_b;
    }
    // one host image of every region set at init (tables, arguments, and the counters and
    // persistent-launch words, which start at zero), one copy: each copy is a dependent
    // operation on the stream, and a batch of many small jobs pays for every one of them
    {
        const size_t base = j->L.conv_spans;
        std::vector<char>& b = j->h_blob;
        b.assign(j->L.blob_end - base, 0);
        auto put = [&](size_t at, const void* src, size_t bytes) {
            if (bytes) std::memcpy(b.data() + (at - base), src, bytes);
        };
        put(j->L.conv_spans, j->h_conv.data(), j->h_conv.size() * sizeof(DevSpan));
        put(j->L.corr_spans, j->h_corr.data(), j->h_corr.size() * sizeof(DevSpan));
        put(j->L.conv_w, j->h_conv_w.data(), j->h_conv_w.size() * 4);
        put(j->L.corr_w, j->h_corr_w.data(), j->h_corr_w.size() * 4);
        if (j->cfg.kind == KIND_MFMA) {
            put(j->L.mf_conv, j->h_mf_conv.data(), j->h_mf_conv.size() * 2);
            put(j->L.mf_corr, j->h_mf_corr.data(), j->h_mf_corr.size() * 2);
        }
        if (j->cfg.kind == KIND_FUSED) {
            put(j->L.fargs, &j->h_fargs, sizeof j->h_fargs);
        } else if (j->cfg.kind != KIND_RESIDENT) {
            put(j->L.args, j->h_args, sizeof j->h_args);
            put(j->L.prefix, j->h_prefix, sizeof j->h_prefix);
        }
        hipError_t e = hipSuccess;
        if (no_alloc || !staged_upload(j->at<void>(base), b.data(), b.size(), s, &e))
            e = hipMemcpyAsync(j->at<void>(base), b.data(), b.size(), hipMemcpyHostToDevice, s);
        if ((st = dev_err(e, "upload tables"))) { delete j; return st; }
    }
    const int64_t N = j->N;
    // f and u^0 into the workspace, r = 0, and the check of f (negative, NaN or infinite
    // values set the invalid flag), in one pass
    if ((st = dev_err(launch("init_fields", rlk::init_fields_kernel, dim3(grid_for(N)), dim3(256), 0, s,
                             j->at<float>(j->L.f), j->at<float>(j->L.u), j->at<float>(j->L.r), p->f,
                             p->u0 ? p->u0 : p->f, N,
                             reinterpret_cast<int32_t*>(j->at<int64_t>(j->L.ctr) + C_F_INVALID)),
                      "init fields"))) { delete j; return st; }
    if (p->thin.mode != RL_THIN_OFF) {
        int64_t nt = (int64_t)j->cfg.tiles_a * j->cfg.tiles_b;
        if ((st = dev_err(launch("fill_u32", rlk::fill_u32_kernel, dim3(grid_for(N / 4 + 1)), dim3(256), 0, s, j->at<uint32_t>(j->L.cnt), 0u, (N + 3) / 4), "zero cnt"))) { delete j; return st; }
        const int lg = block_lg(p);
        if (lg) {
            const int64_t nbk = block_count(p, lg);
            if ((st = dev_err(launch("fill_u32", rlk::fill_u32_kernel, dim3(grid_for(nbk / 4 + 1)), dim3(256), 0, s, j->at<uint32_t>(j->L.cntb), 0u, (nbk + 3) / 4), "zero block cnt"))) { delete j; return st; }
        }
        // tile flags: scratch of the list rebuild (0), or under the block rule every tile
        // active (1, all counters start at 0)
        if ((st = dev_err(launch("fill_u32", rlk::fill_u32_kernel, dim3(grid_for(nt)), dim3(256), 0, s, j->at<uint32_t>(j->L.tflag), lg ? 1u : 0u, nt), "init tflag"))) { delete j; return st; }
        if ((st = dev_err(launch("fill_u32", rlk::fill_u32_kernel, dim3(grid_for(rlk::SCHED_RING * 2)), dim3(256), 0, s, j->at<uint32_t>(j->L.sched), 0u, (int64_t)rlk::SCHED_RING * 2), "zero ring"))) { delete j; return st; }
        if ((st = dev_err(launch("fill_u32", rlk::fill_u32_kernel, dim3(2), dim3(256), 0, s, j->at<uint32_t>(j->L.act), 0u, (int64_t)2 * rlk::ACT_SLOTS), "zero act"))) { delete j; return st; }
    }
    if (p->thin.mode != RL_THIN_OFF && !no_alloc) {
        // pinned word and event for the asynchronous active-tile count (optional: without
        // them the tile list is always used)
        if (hipHostMalloc((void**)&j->h_tcount, sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
            j->h_tcount = nullptr;
        if (j->h_tcount && hipEventCreateWithFlags(&j->tc_event, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(j->h_tcount);
            j->h_tcount = nullptr;
            j->tc_event = nullptr;
        }
    }
    *out = j;
    return RL_OK;
}

}  // namespace

extern "C" {

rl_status rl_init(const rl_params* p, void* ws, size_t ws_bytes, rl_job** out) {
    return init_job(p, ws, ws_bytes, out, false);
}

rl_status rl_iterate(rl_job* j, int32_t n_iter) {
    if (!j) return RL_E_INVAL;
    if (!j->live) return RL_E_STATE;
    if (n_iter < 0) return RL_E_INVAL;
    return enqueue_iterations(j, n_iter);
}

rl_status rl_result(rl_job* j, float* u_out, rl_stats* st) {
    if (!j) return RL_E_INVAL;
    if (!j->live) return RL_E_STATE;
    hipStream_t s = j->stream;
    rl_status rs;
    if (u_out) {
        if ((rs = dev_err(launch("copy_f32", rlk::copy_f32_kernel, dim3(grid_for(j->N)), dim3(256), 0, s, u_out, (const float*)j->cur_u(), j->N), "copy u"))) return rs;
    }
    if (!st) return j->persist_used ? check_persist_abort(j, s) : RL_OK;
    int64_t* ctr = j->at<int64_t>(j->L.ctr);
    const bool thin = j->p.thin.mode != RL_THIN_OFF;
    if (thin && (rs = finalize_thin(j, s))) return rs;
    if ((rs = dev_err(launch("reduce_sum", rlk::reduce_sum_kernel, dim3(rlk::RED_BLOCKS), dim3(256), 0, s,
                             (const float*)j->cur_u(), j->N, j->at<double>(j->L.red)), "reduce"))) return rs;
    if (thin && block_lg(&j->p) && (rs = expand_blocks(j, j->at<uint8_t>(j->L.cnt), s))) return rs;
    if (thin) {
        if ((rs = dev_err(launch("count_active", rlk::count_active_kernel, dim3(rlk::RED_BLOCKS), dim3(256), 0, s,
                                 (const uint8_t*)j->at<uint8_t>(j->L.cnt), j->N, (int)j->p.thin.hysteresis, j->at<int64_t>(j->L.red_i)), "count"))) return rs;
    }
    if ((rs = dev_err(launch("final_reduce", rlk::final_reduce_kernel, dim3(1), dim3(256), 0, s,
                             (const double*)j->at<double>(j->L.red), thin ? (const int64_t*)j->at<int64_t>(j->L.red_i) : (const int64_t*)nullptr,
                             reinterpret_cast<double*>(ctr + C_FLUX), thin ? ctr + C_ACTIVE_NOW : (int64_t*)nullptr), "final"))) return rs;
    int64_t h[C_COUNT];
    int32_t pc[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(h, ctr, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && j->persist_used)
        e = hipMemcpyAsync(pc, j->at<int32_t>(j->L.pctl), sizeof pc, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((rs = dev_err(e, "read stats"))) return rs;
    if (pc[1]) {
        g_last_error = "a persistent launch exceeded its wait limit; the result is incomplete";
        return RL_E_DEVICE;
    }
    std::memset(st, 0, sizeof *st);
    st->iters_done = j->k;
    double flux;
    std::memcpy(&flux, &h[C_FLUX], sizeof flux);
    st->flux = flux;
    if (thin) {
        st->active_now = is_full(j->k, j->p.thin.reset_period) ? j->N : h[C_ACTIVE_NOW];
        st->skipped_px_iters = j->k * j->N - h[C_ACTIVE_TOTAL];
    } else {
        st->active_now = j->N;
        st->skipped_px_iters = 0;
    }
    st->path = j->cfg.path;
    st->schedule = j->cfg.sched;
    int32_t finv;
    std::memcpy(&finv, &h[C_F_INVALID], sizeof finv);
    st->f_invalid = finv ? 1 : 0;
    return finv ? RL_E_INVAL : RL_OK;
}

rl_status rl_destroy(rl_job* j) {
    if (!j) return RL_E_INVAL;
    if (!j->live) return RL_E_STATE;
    j->live = false;
    if (j->graph) (void)hipGraphExecDestroy(j->graph);
    if (j->tc_event) {
        if (j->tc_pending) (void)hipEventSynchronize(j->tc_event);  // copy into h_tcount
        (void)hipEventDestroy(j->tc_event);
    }
    if (j->h_tcount) (void)hipHostFree(j->h_tcount);
    delete j;
    return RL_OK;
}

}  // extern "C"

// ---- allocation-free solve: the job workspace in a static device array ------------------
// One array per device (each device's code object holds its own copy for the life of the
// process).  Host code never passes the array's name to a kernel: `scratch` is a host-side
// stand-in there; the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[RL_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];  // held by rl_solve_static for its whole call
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

extern "C" {

rl_status rl_solve_static(const rl_params* p, int32_t n_iter, float* u_out, rl_stats* st) {
    if (!p || n_iter < 0) return RL_E_INVAL;
    if (p->tuning.graph_iters != 0) {
        g_last_error = "rl_solve_static launches kernels directly (tuning.graph_iters must be 0)";
        return RL_E_UNSUPPORTED;
    }
    size_t need = 0;
    rl_status s = rl_workspace_bytes(p, &need);
    if (s) return s;
    if (need > (size_t)RL_STATIC_SCRATCH_BYTES) {
        g_last_error = "rl_solve_static: the job needs " + std::to_string(need) +
                       " workspace bytes, more than the static array's " +
                       std::to_string((size_t)RL_STATIC_SCRATCH_BYTES);
        return RL_E_NOMEM;
    }
    int dev = 0;
    if ((s = dev_err(hipGetDevice(&dev), "hipGetDevice"))) return s;
    if (dev < 0 || dev >= kMaxDevices) {
        g_last_error = "rl_solve_static: device index out of range";
        return RL_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if ((s = dev_err(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                         "hipGetSymbolAddress(scratch)")))
            return s;
        g_scratch_ptr[dev] = ptr;
    }
    rl_job* j = nullptr;
    if ((s = init_job(p, g_scratch_ptr[dev], (size_t)RL_STATIC_SCRATCH_BYTES, &j, true))) return s;
    s = rl_iterate(j, n_iter);
    rl_stats local;
    if (!s) s = rl_result(j, u_out, st ? st : &local);  // synchronises the stream
    // every enqueued copy and kernel must have finished before the host handle (the
    // source of the table uploads) goes and before the next call reuses the array
    const rl_status se = dev_err(hipStreamSynchronize(j->stream), "synchronise");
    rl_destroy(j);
    return s ? s : se;
}

rl_status rl_batch_workspace_bytes(int32_t n_jobs, size_t* bytes) {
    if (!bytes || n_jobs < 1) return RL_E_INVAL;
    *bytes = batch_bytes(n_jobs);
    return RL_OK;
}

rl_status rl_iterate_batch(rl_job* const* jobs, const int32_t* n_iter, int32_t n_jobs, void* bws,
                           size_t bws_bytes, void* stream) {
    if (!jobs || !n_iter || n_jobs < 1 || !bws) return RL_E_INVAL;
    if (reinterpret_cast<uintptr_t>(bws) % kAlign) return RL_E_INVAL;
    if (bws_bytes < batch_bytes(n_jobs)) return RL_E_NOMEM;
    {
        std::vector<rl_job*> seen(jobs, jobs + n_jobs);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return RL_E_INVAL;
    }
    for (int32_t i = 0; i < n_jobs; ++i) {
        if (!jobs[i] || !jobs[i]->live) return RL_E_STATE;
        if (n_iter[i] < 0) return RL_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rl_status st;
    // tiled two-pass jobs (shared launches per kernel variant), resident line solvers
    // (shared launches per line orientation and segment length), and fused or robust jobs
    // (their own launches)
    std::vector<int> tiled, resident, other;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const rl_job* j = jobs[i];
        if (j->cfg.kind == KIND_RESIDENT) {
            if (n_iter[i] > 0) resident.push_back(i);
        } else if (j->cfg.kind == KIND_FUSED || j->p.rob_eps > 0.f) {
            other.push_back(i);
        } else {
            tiled.push_back(i);
        }
    }
    if (tiled.empty() && resident.empty() && other.empty()) return RL_OK;
    // group by kernel variant; inside a group, jobs with more iterations left come first,
    // so the jobs still running at batch iteration kb are always a prefix of the group
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> groups;
    for (int i : tiled) {
        const Config& c = jobs[i]->cfg;
        groups[std::make_tuple(c.kind, c.orient, c.S, c.lmax, c.nw)].push_back(i);
    }
    struct G {
        std::vector<int> idx;
        std::vector<int32_t> prefix;
        size_t off_a, off_b, off_p;
        size_t lds_a = 0, lds_b = 0;
        int threads = kNW * 64;
        PhaseFn fa, fb;
        const char *na, *nb;
    };
    // estimated work (us) of each job; a variant group whose work exceeds a share of the
    // whole batch is cut into several groups (consecutive in iteration order, so each stays
    // ordered by remaining iterations), so that no single chain of dependent launches
    // outlasts the others by much
    std::vector<double> work(n_jobs, 0.0);
    double total_work = 0.0;
    for (int i : tiled) {
        work[i] = 5.8e-8 * unit_cost(jobs[i]->cfg) * (double)jobs[i]->N * n_iter[i] + 20.0 * n_iter[i] / 8.0;
        total_work += work[i];
    }
    for (int i : resident) total_work += resident_work_us(jobs[i], n_iter[i]);
    for (int i : other) total_work += resident_work_us(jobs[i], n_iter[i]);
    const double share = total_work / (2.0 * kBatchStreams);
    std::vector<std::vector<int>> chunks;
    for (auto& kv : groups) {
        std::vector<int> v = kv.second;
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return n_iter[a] > n_iter[b]; });
        std::vector<int> cur;
        double acc = 0.0;
        for (int i : v) {
            cur.push_back(i);
            acc += work[i];
            if (acc >= share) {
                chunks.push_back(cur);
                cur.clear();
                acc = 0.0;
            }
        }
        if (!cur.empty()) chunks.push_back(cur);
    }
    std::vector<G> gs;
    size_t off = 0;
    for (auto& chunk : chunks) {
        G g;
        g.idx = chunk;
        g.prefix.push_back(0);
        for (int i : g.idx) {
            const Config& c = jobs[i]->cfg;
            g.prefix.push_back(g.prefix.back() + c.tiles_a * c.tiles_b);
            g.lds_a = std::max(g.lds_a, c.lds_a);
            g.lds_b = std::max(g.lds_b, c.lds_b);
        }
        Config c0 = jobs[g.idx[0]]->cfg;
        if (c0.kind == KIND_MFMA) {
            // batch launches of the matrix-core kernel: four wavefronts per tile, so that more
            // tiles share a CU while the other groups' launches overlap
            c0.nw = kMfmaBatchNW;
            c0.threads = kMfmaBatchNW * 64;
        }
        g.threads = c0.threads;
        g.fa = phase_fn(c0, false);
        g.fb = phase_fn(c0, true);
        g.na = phase_name(c0, false);
        g.nb = phase_name(c0, true);
        g.off_a = off;
        off = align_up(off + g.idx.size() * sizeof(PhaseArgs));
        g.off_b = off;
        off = align_up(off + g.idx.size() * sizeof(PhaseArgs));
        g.off_p = off;
        off = align_up(off + g.prefix.size() * sizeof(int32_t));
        gs.push_back(std::move(g));
    }
    // resident groups: one launch per (orientation, segment length) runs every iteration
    // of all its jobs, each workgroup its own job's count
    struct RG {
        std::vector<int> idx;
        std::vector<int32_t> prefix;
        size_t off_t = 0, off_p = 0, lds = 0;
        int orient = 0, seg = 0;
        double w = 0.0;
    };
    std::map<std::pair<int, int>, std::vector<int>> rmap;
    for (int i : resident) rmap[std::make_pair(jobs[i]->cfg.orient, jobs[i]->cfg.seg)].push_back(i);
    std::vector<RG> rgs;
    for (auto& kv : rmap) {
        RG g;
        g.idx = kv.second;
        g.orient = kv.first.first;
        g.seg = kv.first.second;
        g.prefix.push_back(0);
        for (int i : g.idx) {
            g.prefix.push_back(g.prefix.back() + resident_workgroups(jobs[i]->cfg));
            g.lds = std::max(g.lds, jobs[i]->cfg.lds_a);
            g.w += resident_work_us(jobs[i], n_iter[i]);
        }
        g.off_t = off;
        off = align_up(off + g.idx.size() * sizeof(ResidentArgs));
        g.off_p = off;
        off = align_up(off + g.prefix.size() * sizeof(int32_t));
        rgs.push_back(std::move(g));
    }
    // stage the tables on the host and copy them in; the staging buffer of this batch
    // workspace is reused only after its previous copy has completed
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        BatchStage& bs = g_stage[bws];
        if (bs.pending) {
            if ((st = dev_err(hipEventSynchronize(bs.done), "batch staging"))) return st;
            bs.pending = false;
        }
        if (!bs.done && (st = dev_err(hipEventCreateWithFlags(&bs.done, hipEventDisableTiming), "event"))) return st;
        bs.host.assign(off, 0);
        for (const G& g : gs) {
            PhaseArgs* ta = reinterpret_cast<PhaseArgs*>(bs.host.data() + g.off_a);
            PhaseArgs* tb = reinterpret_cast<PhaseArgs*>(bs.host.data() + g.off_b);
            for (size_t q = 0; q < g.idx.size(); ++q) {
                rl_job* j = jobs[g.idx[q]];
                ta[q] = phase_args(j, false, j->k);
                tb[q] = phase_args(j, true, j->k);
                if (j->p.thin.mode != RL_THIN_OFF)
                    ta[q].list_ok = tb[q].list_ok = use_tile_list(j) ? 1 : 0;
            }
            std::memcpy(bs.host.data() + g.off_p, g.prefix.data(), g.prefix.size() * sizeof(int32_t));
        }
        for (const RG& g : rgs) {
            ResidentArgs* t = reinterpret_cast<ResidentArgs*>(bs.host.data() + g.off_t);
            for (size_t q = 0; q < g.idx.size(); ++q) t[q] = resident_args(jobs[g.idx[q]], n_iter[g.idx[q]]);
            std::memcpy(bs.host.data() + g.off_p, g.prefix.data(), g.prefix.size() * sizeof(int32_t));
        }
        hipError_t e = hipSuccess;
        if (off && !staged_upload(bws, bs.host.data(), off, s, &e))
            e = hipMemcpyAsync(bws, bs.host.data(), off, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(bs.done, s);
        if ((st = dev_err(e, "batch tables"))) return st;
        bs.pending = true;
    }
    // fork: the kernel groups and the resident jobs are spread over kBatchStreams side
    // streams (8: of 2 to 24 streams, 8 gave the shortest batch, with HIP's default of four
    // hardware queues per process two streams to a queue), longest estimated work first,
    // each to the stream with the least work so far
    struct Item {
        double w;    // estimated us
        int kind;    // 0: tiled group, 1: resident group, 2: job on its own launches
        int index;
    };
    std::vector<Item> items;
    for (size_t gi = 0; gi < gs.size(); ++gi) {
        double w = 20.0 * n_iter[gs[gi].idx[0]];
        for (int i : gs[gi].idx) w += 5.8e-8 * unit_cost(jobs[i]->cfg) * (double)jobs[i]->N * n_iter[i];
        items.push_back(Item{w, 0, (int)gi});
    }
    for (size_t ri = 0; ri < rgs.size(); ++ri) items.push_back(Item{rgs[ri].w, 1, (int)ri});
    for (int i : other) items.push_back(Item{resident_work_us(jobs[i], n_iter[i]), 2, i});
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.w > b.w; });
    // with kernel timing on, everything runs on one side stream: each launch's events then
    // bracket that launch alone, rather than the time it shares the GPU with the others
    bool timing;
    {
        std::lock_guard<std::mutex> g(g_tmu);
        timing = g_timing;
    }
    const int n_streams = timing ? 1 : std::min<int>(kBatchStreams, (int)items.size());
    std::vector<double> load(n_streams, 0.0);
    std::vector<int> group_stream(gs.size(), 0), rgroup_stream(rgs.size(), 0);
    std::vector<std::pair<int, int>> other_stream;  // (job, stream)
    for (const Item& it : items) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[q] += it.w;
        if (it.kind == 0) group_stream[it.index] = q;
        else if (it.kind == 1) rgroup_stream[it.index] = q;
        else other_stream.emplace_back(it.index, q);
    }
    if ((st = side_streams(n_streams))) return st;
    std::lock_guard<std::mutex> lk(g_smu);
    if ((st = dev_err(hipEventRecord(g_fork, s), "fork"))) return st;
    for (int q = 0; q < n_streams; ++q)
        if ((st = dev_err(hipStreamWaitEvent(g_side[q], g_fork, 0), "fork wait"))) return st;
    auto stream_of_group = [&](size_t gi) { return g_side[group_stream[gi]]; };
    char* base = static_cast<char*>(bws);
    // resident groups: all iterations of all their jobs in one launch each
    for (size_t ri = 0; ri < rgs.size(); ++ri) {
        const RG& g = rgs[ri];
        st = dev_err(launch("resident_box", resident_multi_fn(g.orient, g.seg), dim3(g.prefix.back()),
                            dim3(256), g.lds, g_side[rgroup_stream[ri]],
                            reinterpret_cast<const ResidentArgs*>(base + g.off_t),
                            reinterpret_cast<const int32_t*>(base + g.off_p), (int)g.idx.size()),
                     "resident_box");
        if (st) return st;
        for (int i : g.idx) jobs[i]->k += n_iter[i];
    }
    // fused jobs one launch per iteration, robust ones four, on their side stream
    for (const auto& rq : other_stream) {
        rl_job* j = jobs[rq.first];
        hipStream_t keep = j->stream;
        j->stream = g_side[rq.second];
        st = enqueue_iterations(j, n_iter[rq.first]);
        j->stream = keep;
        if (st) return st;
    }
    for (size_t gi = 0; gi < gs.size(); ++gi) {
        const G& g = gs[gi];
        hipStream_t gsm = stream_of_group(gi);
        const int32_t kmax = n_iter[g.idx[0]];
        for (int32_t kb = 0; kb < kmax; ++kb) {
            for (int i : g.idx) {
                rl_job* j = jobs[i];
                if (n_iter[i] <= kb || j->p.thin.mode == RL_THIN_OFF) continue;
                const int64_t k = j->k + kb;
                if (!is_full(k, j->p.thin.reset_period) &&
                    (!j->list_valid || is_rebuild(k, j->p.thin.reset_period, j->p.thin.compact_period)))
                    if ((st = rebuild_lists(j, gsm))) return st;
            }
            int m = 0;
            while (m < (int)g.idx.size() && n_iter[g.idx[m]] > kb) ++m;
            for (int q = 0; q < m; ++q)
                if ((st = enqueue_tv(jobs[g.idx[q]], gsm))) return st;
            for (int phase = 0; phase < 2; ++phase) {
                rlk::LaunchArgs la{};
                la.table = reinterpret_cast<const PhaseArgs*>(base + (phase ? g.off_b : g.off_a));
                la.prefix = reinterpret_cast<const int32_t*>(base + g.off_p);
                la.n_jobs = m;
                la.kb = kb;
                if (m == 1) {
                    rl_job* j1 = jobs[g.idx[0]];
                    la.one = phase_args(j1, phase == 1, j1->k);
                    if (j1->p.thin.mode != RL_THIN_OFF) {
                        la.one.list_ok = use_tile_list(j1) ? 1 : 0;
                        la.one.full = is_full(j1->k + kb, j1->p.thin.reset_period) ? 1 : 0;
                    }
                }
                st = dev_err(launch(phase ? g.nb : g.na, phase ? g.fb : g.fa, dim3(g.prefix[m]),
                                    dim3(g.threads), phase ? g.lds_b : g.lds_a, gsm, la),
                             phase ? g.nb : g.na);
                if (st) return st;
            }
        }
    }
    // join
    for (int q = 0; q < n_streams; ++q) {
        if ((st = dev_err(hipEventRecord(g_join[q], g_side[q]), "join"))) return st;
        if ((st = dev_err(hipStreamWaitEvent(s, g_join[q], 0), "join wait"))) return st;
    }
    for (int i : tiled) {
        jobs[i]->k += n_iter[i];
        if (n_iter[i] > 0 && jobs[i]->p.thin.mode != RL_THIN_OFF) jobs[i]->pending_finalize = true;
    }
    return RL_OK;
}

rl_status rl_get_state(rl_job* j, float* u, float* r, uint8_t* cnt, int64_t* k_out) {
    if (!j) return RL_E_INVAL;
    if (!j->live) return RL_E_STATE;
    hipStream_t s = j->stream;
    unsigned g = grid_for(j->N);
    rl_status st;
    if (u && (st = dev_err(launch("copy_f32", rlk::copy_f32_kernel, dim3(g), dim3(256), 0, s, u, (const float*)j->cur_u(), j->N), "get u"))) return st;
    if (r && (st = dev_err(launch("copy_f32", rlk::copy_f32_kernel, dim3(g), dim3(256), 0, s, r, (const float*)j->at<float>(j->L.r), j->N), "get r"))) return st;
    if (cnt) {
        if (j->p.thin.mode == RL_THIN_OFF) return RL_E_STATE;
        if (block_lg(&j->p)) {
            if ((st = expand_blocks(j, cnt, s))) return st;
        } else if ((st = dev_err(launch("copy_u8", rlk::copy_u8_kernel, dim3(g), dim3(256), 0, s, cnt, (const uint8_t*)j->at<uint8_t>(j->L.cnt), j->N), "get cnt"))) {
            return st;
        }
    }
    if (k_out) *k_out = j->k;
    return j->persist_used ? check_persist_abort(j, s) : RL_OK;
}

rl_status rl_set_state(rl_job* j, const float* u, const float* r, const uint8_t* cnt, int64_t k) {
    if (!j) return RL_E_INVAL;
    if (!j->live) return RL_E_STATE;
    if (k < 0) return RL_E_INVAL;
    if (cnt && j->p.thin.mode == RL_THIN_OFF) return RL_E_STATE;
    hipStream_t s = j->stream;
    unsigned g = grid_for(j->N);
    rl_status st;
    j->k = k;  // selects the plane that holds u^k (fused schedule)
    if (u && (st = dev_err(launch("copy_f32", rlk::copy_f32_kernel, dim3(g), dim3(256), 0, s, j->cur_u(), u, j->N), "set u"))) return st;
    if (r && (st = dev_err(launch("copy_f32", rlk::copy_f32_kernel, dim3(g), dim3(256), 0, s, j->at<float>(j->L.r), r, j->N), "set r"))) return st;
    if (cnt && (st = dev_err(launch("copy_u8", rlk::copy_u8_kernel, dim3(g), dim3(256), 0, s, j->at<uint8_t>(j->L.cnt), cnt, j->N), "set cnt"))) return st;
    if (cnt) {
        if (const int lg = block_lg(&j->p)) {
            // block rule: each block takes the counter of its top-left pixel
            const int64_t nbk = block_count(&j->p, lg);
            if ((st = dev_err(launch("block_compress", rlk::block_compress_kernel, dim3(grid_for(nbk)), dim3(256), 0, s,
                                     (const uint8_t*)j->at<uint8_t>(j->L.cnt), j->at<uint8_t>(j->L.cntb), j->W, lg,
                                     (int)block_cols(&j->p, lg), nbk), "set block cnt"))) return st;
            const int ntiles = j->cfg.tiles_a * j->cfg.tiles_b;
            if ((st = dev_err(launch("block_tiles", rlk::block_tiles_kernel, dim3((ntiles + 255) / 256), dim3(256), 0, s,
                                     (const uint8_t*)j->at<uint8_t>(j->L.cntb), j->H, j->W, lg,
                                     (int)block_cols(&j->p, lg), (int)j->p.thin.hysteresis, j->cfg.orient,
                                     j->cfg.tiles_a, ntiles, j->at<int32_t>(j->L.tflag)), "set tile flags"))) return st;
        }
    }
    j->k = k;
    j->list_valid = false;
    if (j->p.thin.mode != RL_THIN_OFF) {
        if ((st = dev_err(launch("fill_u32", rlk::fill_u32_kernel, dim3(2), dim3(256), 0, s, j->at<uint32_t>(j->L.act), 0u, (int64_t)2 * rlk::ACT_SLOTS), "zero act"))) return st;
        j->pending_finalize = false;
    }
    return RL_OK;
}

rl_status rl_active_list(rl_job* j, int32_t* list_dev, int64_t cap, int64_t* n) {
    if (!j || !n) return RL_E_INVAL;
    if (!j->live || j->p.thin.mode == RL_THIN_OFF) return RL_E_STATE;
    hipStream_t s = j->stream;
    int64_t len = 0;
    hipError_t e = hipMemcpyAsync(&len, j->at<int64_t>(j->L.ctr) + C_PLIST_LEN, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    rl_status st = dev_err(e, "list len");
    if (st) return st;
    const bool have = j->list_valid && j->p.thin.keep_list;
    *n = have ? len : -1;
    if (list_dev && len > 0 && have) {
        if (cap < len) return RL_E_NOMEM;
        e = hipMemcpyAsync(list_dev, j->at<int32_t>(j->L.plist), (size_t)len * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if ((st = dev_err(e, "list copy"))) return st;
    }
    return RL_OK;
}

rl_status rl_thin_schedule(rl_job* j, int64_t* out, int32_t cap, int32_t* n) {
    if (!j || !n) return RL_E_INVAL;
    if (!j->live || j->p.thin.mode == RL_THIN_OFF) return RL_E_STATE;
    std::vector<int64_t> ring(rlk::SCHED_RING);
    rl_status fs = finalize_thin(j, j->stream);
    if (fs) return fs;
    hipError_t e = hipMemcpyAsync(ring.data(), j->at<int64_t>(j->L.sched), ring.size() * 8, hipMemcpyDeviceToHost, j->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(j->stream);
    rl_status st = dev_err(e, "schedule");
    if (st) return st;
    int64_t cnt = std::min<int64_t>(std::min<int64_t>(j->k, cap), rlk::SCHED_RING);
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t kk = j->k - cnt + i;
        if (out) out[i] = ring[kk % rlk::SCHED_RING];
    }
    *n = (int32_t)cnt;
    return RL_OK;
}

rl_status rl_psf_runs(const float* psf, int32_t psf_h, int32_t psf_w, int32_t* runs, float* w,
                      int32_t cap, int32_t* n_runs, int32_t* cls) {
    std::string why;
    rl::CompiledPsf c;
    if (!rl::compile_psf(psf, psf_h, psf_w, &c, &why)) return RL_E_INVAL;
    if (n_runs) *n_runs = (int32_t)c.runs.size();
    if (cls) *cls = c.auto_path;
    if ((int64_t)c.runs.size() > cap) return RL_E_NOMEM;
    for (size_t i = 0; i < c.runs.size(); ++i) {
        if (runs) {
            runs[3 * i + 0] = c.runs[i].dy;
            runs[3 * i + 1] = c.runs[i].x0;
            runs[3 * i + 2] = c.runs[i].x1;
        }
        if (w) w[i] = c.runs[i].w;
    }
    return RL_OK;
}

rl_status rl_debug_spin_limit(int32_t polls, int32_t* previous) {
    const int old = g_spin_limit.exchange(polls);
    if (previous) *previous = old;
    return RL_OK;
}

rl_status rl_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_tmu);
    g_timing = on != 0;
    return RL_OK;
}

rl_status rl_timing_read(const char* name, int64_t* launches, double* total_ms) {
    if (!name || !launches || !total_ms) return RL_E_INVAL;
    std::lock_guard<std::mutex> g(g_tmu);
    int64_t n = 0;
    double tot = 0;
    for (TimedLaunch& t : g_timed) {
        if (t.name != name) continue;
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return dev_err(e, "timing");
        float ms = 0;
        e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess) return dev_err(e, "timing");
        ++n;
        tot += ms;
    }
    *launches = n;
    *total_ms = tot;
    return RL_OK;
}

rl_status rl_timing_reset(void) {
    std::lock_guard<std::mutex> g(g_tmu);
    for (TimedLaunch& t : g_timed) {
        (void)hipEventSynchronize(t.b);
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_timed.clear();
    return RL_OK;
}


rl_status rl_autotune_workspace_bytes(const rl_params* p, size_t* bytes) {
    std::string why;
    if (!bytes) return RL_E_INVAL;
    rl_status st = validate_params(p, &why);
    if (st) return st;
    rl::CompiledPsf c;
    if (!rl::compile_psf(p->psf, p->psf_h, p->psf_w, &c, &why)) return RL_E_INVAL;
    Config base;
    if ((st = choose_config_raw(p, c, &base, &why))) return st;
    size_t mx = make_layout(p, base).total;
    for (const TuneEntry& e : tune_candidates(p, base)) {
        rl_params q = with_entry(p, e);
        Config cfg;
        if (choose_config_raw(&q, c, &cfg, &why) != RL_OK) continue;
        mx = std::max(mx, make_layout(&q, cfg).total);
    }
    *bytes = mx;
    return RL_OK;
}

rl_status rl_autotune(const rl_params* p, void* ws, size_t ws_bytes, int32_t n_iter,
                      int32_t* best_schedule, rl_tuning* best, double* best_ms) {
    std::string why;
    if (!best || n_iter < 1) return RL_E_INVAL;
    rl_status st = validate_params(p, &why);
    if (st) return st;
    rl::CompiledPsf c;
    if (!rl::compile_psf(p->psf, p->psf_h, p->psf_w, &c, &why)) return RL_E_INVAL;
    Config base;
    if ((st = choose_config_raw(p, c, &base, &why))) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(p->stream);
    hipEvent_t a, b;
    if ((st = dev_err(hipEventCreate(&a), "event"))) return st;
    if ((st = dev_err(hipEventCreate(&b), "event"))) { (void)hipEventDestroy(a); return st; }
    double bt = 1e300;
    TuneEntry bestt{};
    bool found = false;
    for (const TuneEntry& e : tune_candidates(p, base)) {
        rl_params q = with_entry(p, e);
        Config cfg;
        if (choose_config_raw(&q, c, &cfg, &why) != RL_OK) continue;  // not applicable
        rl_job* j = nullptr;
        if (rl_init(&q, ws, ws_bytes, &j) != RL_OK) continue;
        // the warm-up covers one full timed chunk, so graph capture is not timed
        st = rl_iterate(j, n_iter);
        if (st == RL_OK) st = dev_err(hipEventRecord(a, s), "event");
        if (st == RL_OK) st = rl_iterate(j, n_iter);
        if (st == RL_OK) st = dev_err(hipEventRecord(b, s), "event");
        if (st == RL_OK) st = dev_err(hipEventSynchronize(b), "event");
        float ms = 0;
        if (st == RL_OK) st = dev_err(hipEventElapsedTime(&ms, a, b), "event");
        rl_destroy(j);
        if (st) break;
        const double per = ms / n_iter;
        if (per < bt) {
            bt = per;
            bestt = e;
            found = true;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st) return st;
    if (!found) return RL_E_UNSUPPORTED;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(p, c)] = bestt;
        ++g_tune_gen;
    }
    *best = bestt.t;
    if (best_schedule) *best_schedule = bestt.schedule;
    if (best_ms) *best_ms = bt;
    return RL_OK;
}

rl_status rl_tune_lookup(const rl_params* p, int32_t* schedule, rl_tuning* out) {
    std::string why;
    if (!p || !out) return RL_E_INVAL;
    rl::CompiledPsf c;
    if (!rl::compile_psf(p->psf, p->psf_h, p->psf_w, &c, &why)) return RL_E_INVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(p, c));
    if (it == g_tune.end()) return RL_E_STATE;
    *out = it->second.t;
    if (schedule) *schedule = it->second.schedule;
    return RL_OK;
}

rl_status rl_tune_cache_save(const char* path) {
    if (!path) return RL_E_INVAL;
    std::ofstream o(path);
    if (!o) return RL_E_INVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    o << "# rl tuning cache: path kh kw taps runs bucket thin schedule -> "
         "schedule strip seg lines_per_wg graph_iters\n";
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        const rl_tuning& t = kv.second.t;
        o << k.path << ' ' << k.kh << ' ' << k.kw << ' ' << k.taps << ' ' << k.runs << ' '
          << k.bucket << ' ' << k.thin << ' ' << k.schedule << ' ' << kv.second.schedule << ' '
          << t.strip << ' ' << t.seg << ' ' << t.lines_per_wg << ' ' << t.graph_iters << '\n';
    }
    return o ? RL_OK : RL_E_INVAL;
}

rl_status rl_tune_cache_load(const char* path) {
    if (!path) return RL_E_INVAL;
    std::ifstream in(path);
    if (!in) return RL_E_INVAL;
    std::map<TuneKey, TuneEntry> loaded;
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ss(line);
        TuneKey k{};
        TuneEntry e{};
        if (!(ss >> k.path >> k.kh >> k.kw >> k.taps >> k.runs >> k.bucket >> k.thin >> k.schedule >>
              e.schedule >> e.t.strip >> e.t.seg >> e.t.lines_per_wg >> e.t.graph_iters))
            return RL_E_INVAL;
        if (e.schedule < RL_SCHED_AUTO || e.schedule > RL_SCHED_FUSED || e.t.strip < 0 ||
            e.t.seg < 0 || e.t.lines_per_wg < 0 || e.t.graph_iters < 0)
            return RL_E_INVAL;
        loaded[k] = e;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : loaded) g_tune[kv.first] = kv.second;
    ++g_tune_gen;
    return RL_OK;
}

rl_status rl_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    ++g_tune_gen;
    return RL_OK;
}

rl_status rl_job_describe(rl_job* j, rl_job_info* info) {
    if (!j || !info) return RL_E_INVAL;
    if (!j->live) return RL_E_STATE;
    std::memset(info, 0, sizeof *info);
    const Config& c = j->cfg;
    info->path = c.path;
    info->schedule = c.sched;
    if (c.kind == KIND_RESIDENT) {
        info->tile_h = c.orient == rlk::ORIENT_ROWS ? c.lines_per_wg : c.line_n;
        info->tile_w = c.orient == rlk::ORIENT_ROWS ? c.line_n : c.lines_per_wg;
        info->strip = c.seg;
        info->n_spans = 1;
        info->n_taps = j->psf.n_taps;
    } else {
        info->tile_h = c.orient == rlk::ORIENT_ROWS ? c.TA : c.TB;
        info->tile_w = c.orient == rlk::ORIENT_ROWS ? c.TB : c.TA;
        info->strip = c.S;
        info->n_spans = (int32_t)c.conv.spans.size();
        info->n_taps = j->psf.n_taps;
        info->lmax = c.kind == KIND_SPAN ? c.lmax : 0;
        info->halo_y0 = c.orient == rlk::ORIENT_ROWS ? c.conv.lane_min : c.conv.c_min;
        info->halo_y1 = c.orient == rlk::ORIENT_ROWS ? c.conv.lane_max : c.conv.c_max;
        info->halo_x0 = c.orient == rlk::ORIENT_ROWS ? c.conv.c_min : c.conv.lane_min;
        info->halo_x1 = c.orient == rlk::ORIENT_ROWS ? c.conv.c_max : c.conv.lane_max;
    }
    info->ws_bytes = (int64_t)j->L.total;
    return RL_OK;
}

}  // extern "C"

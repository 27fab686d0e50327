// PSF compiler (host).  See psf_compile.hpp.
#include "psf_compile.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "rl.h"

namespace rl {

static uint32_t bits_of(float v) {
    uint32_t b;
    std::memcpy(&b, &v, sizeof b);
    return b;
}

bool compile_psf(const float* psf, int kh, int kw, CompiledPsf* out, std::string* why) {
    if (!psf || kh < 1 || kw < 1 || kh > 127 || kw > 127) {
        if (why) *why = "PSF size must be in [1, 127] x [1, 127]";
        return false;
    }
    CompiledPsf c;
    c.kh = kh;
    c.kw = kw;
    const int oy = kh / 2, ox = kw / 2;
    for (int i = 0; i < kh * kw; ++i) {
        float v = psf[i];
        if (!std::isfinite(v) || v < 0.f) {
            if (why) *why = "PSF entries must be finite and non-negative";
            return false;
        }
        if (v != 0.f) ++c.n_taps;
        c.sum += (double)v;
    }
    if (!(c.sum > 0.0)) {
        if (why) *why = "PSF must have a positive sum";
        return false;
    }
    // canonical run list: per row, maximal spans of bit-identical non-zero weights
    for (int i = 0; i < kh; ++i) {
        int j = 0;
        while (j < kw) {
            float v = psf[i * kw + j];
            if (v == 0.f) { ++j; continue; }
            int j1 = j;
            while (j1 + 1 < kw && psf[i * kw + j1 + 1] != 0.f &&
                   bits_of(psf[i * kw + j1 + 1]) == bits_of(v))
                ++j1;
            c.runs.push_back(Run{i - oy, j - ox, j1 - ox, v});
            j = j1 + 1;
        }
    }
    // axis box: all taps in one row (or one column), contiguous, bit-identical, >= 2 taps
    if (c.n_taps >= 2) {
        if (c.runs.size() == 1) {
            const Run& r = c.runs[0];
            c.is_axis_box = true;
            c.box_orient = Orient::Rows;
            c.box_len = r.x1 - r.x0 + 1;
            c.box_w = r.w;
            c.box_c0 = -r.x1;  // conv in correlation form: offsets -x1 .. -x0
        } else {
            // one column?
            int col = -1;
            bool ok = true;
            for (const Run& r : c.runs) {
                if (r.x0 != r.x1) { ok = false; break; }
                if (col < 0) col = r.x0 + ox;
                else if (col != r.x0 + ox) { ok = false; break; }
                if (bits_of(r.w) != bits_of(c.runs[0].w)) { ok = false; break; }
            }
            if (ok) {
                for (size_t q = 1; q < c.runs.size(); ++q)
                    if (c.runs[q].dy != c.runs[q - 1].dy + 1) { ok = false; break; }
            }
            if (ok) {
                c.is_axis_box = true;
                c.box_orient = Orient::Cols;
                c.box_len = (int)c.runs.size();
                c.box_w = c.runs[0].w;
                c.box_c0 = -c.runs.back().dy;
            }
        }
    }
    // rectangle: one run per row, consecutive rows, equal column span and weight bits
    if (!c.is_axis_box && c.runs.size() >= 2) {
        const Run& r0 = c.runs[0];
        bool ok = r0.x1 > r0.x0;
        for (size_t q = 1; ok && q < c.runs.size(); ++q) {
            const Run& r = c.runs[q];
            ok = r.dy == c.runs[q - 1].dy + 1 && r.x0 == r0.x0 && r.x1 == r0.x1 &&
                 bits_of(r.w) == bits_of(r0.w);
        }
        c.is_rect = ok;
    }
    if (c.n_taps == 1) c.auto_path = RL_PATH_DIRECT;  // bit-exact identity for a delta
    else if (c.is_axis_box) c.auto_path = RL_PATH_BOX_AXIS;
    else if (c.is_rect) c.auto_path = RL_PATH_BOX_RECT;
    else c.auto_path = RL_PATH_RUNS;
    *out = std::move(c);
    return true;
}

// Correlation-form offset of tap (i, j): conv (u*h) reads u at (y - (i-oy), x - (j-ox));
// the adjoint (h^* * r) reads r at (y + (i-oy), x + (j-ox)).
static inline void tap_offset(int i, int j, int oy, int ox, bool adjoint, int* sy, int* sx) {
    if (adjoint) { *sy = i - oy; *sx = j - ox; }
    else { *sy = oy - i; *sx = ox - j; }
}

OpTable build_op_table(const float* psf, int kh, int kw, bool adjoint, Orient o,
                       bool split_uniform, int lmax) {
    const int oy = kh / 2, ox = kw / 2;
    // Lines are PSF rows (Orient::Rows) or columns (Orient::Cols), visited in ascending lane
    // offset, and the taps of a line in ascending position: tap (i, j) sits at lane offset /
    // position (sy, sx) of tap_offset, which ascend with i and j for the adjoint and descend
    // for conv, so conv walks both indices backwards.  No sorting and no per-line containers.
    const bool rows = o == Orient::Rows;
    const int nl = rows ? kh : kw, np = rows ? kw : kh;
    OpTable t;
    bool first = true;
    std::vector<std::pair<int, float>> taps;
    taps.reserve((size_t)np);
    std::vector<Span> pieces;
    for (int li = 0; li < nl; ++li) {
        const int idx = adjoint ? li : nl - 1 - li;
        taps.clear();
        for (int pi = 0; pi < np; ++pi) {
            const int pidx = adjoint ? pi : np - 1 - pi;
            const int i = rows ? idx : pidx, j = rows ? pidx : idx;
            const float v = psf[i * kw + j];
            if (v == 0.f) continue;
            int sy, sx;
            tap_offset(i, j, oy, ox, adjoint, &sy, &sx);
            taps.push_back({rows ? sx : sy, v});
        }
        if (taps.empty()) continue;
        int lane;
        {
            int sy, sx;
            tap_offset(rows ? idx : 0, rows ? 0 : idx, oy, ox, adjoint, &sy, &sx);
            lane = rows ? sy : sx;
        }
        pieces.clear();
        size_t q = 0;
        while (q < taps.size()) {
            size_t q1 = q;
            while (q1 + 1 < taps.size() && taps[q1 + 1].first == taps[q1].first + 1 &&
                   (!split_uniform || bits_of(taps[q1 + 1].second) == bits_of(taps[q].second)))
                ++q1;
            // taps q..q1 are one contiguous span; cut into pieces of <= lmax
            size_t s = q;
            while (s <= q1) {
                size_t e = q1;
                if (lmax > 0 && e - s + 1 > (size_t)lmax) e = s + lmax - 1;
                Span sp{};
                sp.lane_off = lane;
                sp.c0 = taps[s].first;
                sp.len = (int32_t)(e - s + 1);
                sp.woff = (int32_t)t.w.size();
                sp.w0 = taps[s].second;
                sp.uniform = 1;
                for (size_t z = s; z <= e; ++z) {
                    t.w.push_back(taps[z].second);
                    if (bits_of(taps[z].second) != bits_of(taps[s].second)) sp.uniform = 0;
                }
                pieces.push_back(sp);
                s = e + 1;
            }
            q = q1 + 1;
        }
        pieces.back().row_end = 1;
        for (const Span& sp : pieces) {
            if (first) {
                t.lane_min = t.lane_max = sp.lane_off;
                t.c_min = sp.c0;
                t.c_max = sp.c0 + sp.len - 1;
                first = false;
            }
            t.lane_min = std::min(t.lane_min, sp.lane_off);
            t.lane_max = std::max(t.lane_max, sp.lane_off);
            t.c_min = std::min(t.c_min, sp.c0);
            t.c_max = std::max(t.c_max, sp.c0 + sp.len - 1);
            t.spans.push_back(sp);
        }
    }
    return t;
}

OpTable build_tap_table(const float* psf, int kh, int kw, bool adjoint) {
    const int oy = kh / 2, ox = kw / 2;
    OpTable t;
    bool first = true;
    for (int i = 0; i < kh; ++i) {
        int last = -1;
        for (int j = 0; j < kw; ++j) {
            float v = psf[i * kw + j];
            if (v == 0.f) continue;
            int sy, sx;
            tap_offset(i, j, oy, ox, adjoint, &sy, &sx);
            Span sp{};
            sp.lane_off = sy;
            sp.c0 = sx;
            sp.len = 1;
            sp.woff = (int32_t)t.w.size();
            sp.w0 = v;
            sp.uniform = 1;
            t.w.push_back(v);
            if (first) {
                t.lane_min = t.lane_max = sy;
                t.c_min = t.c_max = sx;
                first = false;
            }
            t.lane_min = std::min(t.lane_min, sy);
            t.lane_max = std::max(t.lane_max, sy);
            t.c_min = std::min(t.c_min, sx);
            t.c_max = std::max(t.c_max, sx);
            t.spans.push_back(sp);
            last = (int)t.spans.size() - 1;
        }
        if (last >= 0) t.spans[last].row_end = 1;  // one PSF row = one partial sum
    }
    return t;
}

}  // namespace rl

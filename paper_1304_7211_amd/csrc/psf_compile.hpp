// PSF compiler: turns a float32 PSF into the tables the kernels consume.
//
// The paper's fast convolutions (Section 3) all come from looking at the PSF's structure:
// a 1 x M box slides along scan-lines (box filter), a convex uniform shape slides by adding
// one boundary line and removing another (generic box filter), a sparse PSF is summed over
// a list of its support pixels (list filter).  This compiler finds that structure once per
// job on the host.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace rl {

enum class Orient : int32_t { Rows = 0, Cols = 1 };

// One integer run of the PSF (paper notation: a row of the PSF split into maximal spans of
// bit-identical non-zero weights).  dy = i - oy, x0/x1 = j - ox of the first/last tap.
struct Run {
    int32_t dy, x0, x1;
    float w;
};

// A span of an operator in correlation form along the chosen orientation:
//   out(a, b) += sum_{t < len} wt[woff + t] * src(a + lane_off, b + c0 + t)
// where, for Orient::Rows, a = row and b = column (spans lie along rows), and for
// Orient::Cols, a = column and b = row (spans lie along columns).
// `uniform` spans have all weights equal to w0 (a run of the generic box filter).
// `row_end` marks the last piece of one PSF line (the unit of partial summation).
struct Span {
    int32_t lane_off, c0, len, woff;
    float w0;
    int32_t uniform, row_end, pad;
};

struct OpTable {
    std::vector<Span> spans;
    std::vector<float> w;
    int32_t lane_min = 0, lane_max = 0;  // extent of lane_off
    int32_t c_min = 0, c_max = 0;        // extent of c0 .. c0+len-1
};

struct CompiledPsf {
    int32_t kh = 0, kw = 0, n_taps = 0;
    double sum = 0.0;
    std::vector<Run> runs;  // row runs, the canonical run list
    int32_t auto_path = 0;  // RL_PATH_* chosen for RL_PATH_AUTO
    // axis box description (valid when is_axis_box)
    bool is_axis_box = false;
    Orient box_orient = Orient::Rows;
    int32_t box_len = 0, box_c0 = 0;  // correlation-form offset of the first tap (conv)
    float box_w = 0.f;
    // full uniform rectangle of at least 2 x 2 taps (every tap of a kh x kw block present
    // and bit-identical); the block may sit anywhere in the PSF array
    bool is_rect = false;
};

// Validates (finite, >= 0, positive sum) and compiles.  Returns false with a reason.
bool compile_psf(const float* psf, int kh, int kw, CompiledPsf* out, std::string* why);

// Operator tables for conv (forward, u*h) or corr (adjoint, h^* * r) in the given
// orientation.  `split_uniform` splits lines into runs of bit-identical weights (for the
// sliding kernels); otherwise a line is split only at zero taps (for the span kernels).
// Pieces longer than lmax are cut into pieces of at most lmax taps (lmax <= 0: no limit).
OpTable build_op_table(const float* psf, int kh, int kw, bool adjoint, Orient o,
                       bool split_uniform, int lmax);

// Per-tap table (one span of length 1 per non-zero tap, ascending PSF row then column).
OpTable build_tap_table(const float* psf, int kh, int kw, bool adjoint);

}  // namespace rl

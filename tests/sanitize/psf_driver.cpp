// Test driver: runs the library's host-side PSF compiler (psf_compile.cpp) on PSFs read
// from stdin, for a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Prints
// the class and the canonical run list of each PSF (compared with the oracle-side run-list
// definition by the test), and checks every operator table the kernels could be given:
// both operators, both orientations, split or not, every piece limit, and the per-tap
// table.  Test infrastructure only.
//
// stdin: a count, then per PSF "kh kw" and kh*kw values.
// stdout: per PSF "psf <i> <valid> <auto_path> <n_runs>", then "run dy x0 x1 w" lines
// (w as a hexadecimal float); a line "fail ..." for any broken table invariant.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "psf_compile.hpp"

static int check_table(const rl::OpTable& t, int n_taps, int lmax, const char* what) {
    long taps = 0;
    int bad = 0;
    for (const rl::Span& s : t.spans) {
        taps += s.len;
        if (s.len < 1 || (lmax > 0 && s.len > lmax)) bad = 1;
        if (s.woff < 0 || (size_t)(s.woff + s.len) > t.w.size()) bad = 1;
        if (s.lane_off < t.lane_min || s.lane_off > t.lane_max) bad = 1;
        if (s.c0 < t.c_min || s.c0 + s.len - 1 > t.c_max) bad = 1;
        for (int q = 0; q < s.len && !bad; ++q)
            if (!(t.w[s.woff + q] > 0.f) || !std::isfinite(t.w[s.woff + q])) bad = 1;
    }
    if (taps != n_taps) bad = 1;
    if (bad) std::printf("fail %s taps=%ld want=%d\n", what, taps, n_taps);
    return bad;
}

int main() {
    int count = 0;
    if (std::scanf("%d", &count) != 1) return 2;
    int failures = 0;
    for (int i = 0; i < count; ++i) {
        int kh = 0, kw = 0;
        if (std::scanf("%d %d", &kh, &kw) != 2) return 2;
        std::vector<float> h((size_t)kh * kw);
        for (float& v : h)
            if (std::scanf("%f", &v) != 1) return 2;
        rl::CompiledPsf c;
        std::string why;
        const bool ok = rl::compile_psf(h.data(), kh, kw, &c, &why);
        std::printf("psf %d %d %d %zu\n", i, ok ? 1 : 0, ok ? c.auto_path : -1,
                    ok ? c.runs.size() : (size_t)0);
        if (!ok) continue;
        for (const rl::Run& r : c.runs) std::printf("run %d %d %d %a\n", r.dy, r.x0, r.x1, r.w);
        for (int adj = 0; adj < 2; ++adj)
            for (int o = 0; o < 2; ++o)
                for (int split = 0; split < 2; ++split)
                    for (int lmax : {0, 1, 4, 8, 16}) {
                        rl::OpTable t = rl::build_op_table(h.data(), kh, kw, adj != 0,
                                                           o ? rl::Orient::Cols : rl::Orient::Rows,
                                                           split != 0, lmax);
                        failures += check_table(t, c.n_taps, lmax, "op_table");
                    }
        for (int adj = 0; adj < 2; ++adj)
            failures += check_table(rl::build_tap_table(h.data(), kh, kw, adj != 0), c.n_taps, 1,
                                    "tap_table");
    }
    return failures ? 1 : 0;
}

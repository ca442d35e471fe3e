// Test-only host build of the regularized far-field header (no GPU code runs): lets the
// CPU test suite compare the one-function form (Taylor coefficients of R and the
// cluster stream W) against the oracle.
#include "reg_math.hpp"

#include <vector>

template <int P> static void run_p(const double *mom, const double *d, double eps, double u[3]) {
    using E = stk::RegEval<P>;
    std::vector<double> W(E::WS, 0.0);
    for (int a = 0; a < E::NB; ++a) stk::reg_stream_fill(mom, 12, P, a, W.data());
    const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
    E::run(d, R2, W.data(), u);
}

extern "C" {
// mom: (nidx(p), 12) moments of one cluster; d = x - y_c
void hc_reg_far(const double *mom, int p, const double *d, double eps, double *u) {
    switch (p) {
        case 0: run_p<0>(mom, d, eps, u); break;
        case 1: run_p<1>(mom, d, eps, u); break;
        case 2: run_p<2>(mom, d, eps, u); break;
        case 3: run_p<3>(mom, d, eps, u); break;
        case 4: run_p<4>(mom, d, eps, u); break;
        case 5: run_p<5>(mom, d, eps, u); break;
        case 6: run_p<6>(mom, d, eps, u); break;
        case 7: run_p<7>(mom, d, eps, u); break;
        case 8: run_p<8>(mom, d, eps, u); break;
        case 9: run_p<9>(mom, d, eps, u); break;
        case 10: run_p<10>(mom, d, eps, u); break;
    }
}
// W_i^q of one multi-index (for the term-by-term check)
void hc_reg_stream(const double *mom, int p, const int *q, double *out) { stk::reg_stream(mom, 12, p, q, out); }
// 1 if the stream positions of W^q (orders 2 .. p + 3) and V^q (order p + 1) cover
// [0, reg_stream_len(p)) exactly once each
int hc_reg_layout_ok(int p) {
    const int len = stk::reg_stream_len(p);
    std::vector<int> seen(len, 0);
    for (int a = stk::nidx(1); a < stk::nidx(p + 3); ++a) {
        int q[3];
        stk::kof(a, q);
        const int n = q[0] + q[1] + q[2], s = stk::reg_spos(p, a), w = n == stk::reg_vorder(p) ? 6 : 3;
        for (int c = 0; c < w; ++c) {
            if (s + c < 0 || s + c >= len) return 0;
            seen[s + c]++;
        }
    }
    for (int v : seen)
        if (v != 1) return 0;
    return 1;
}
}

// Test-only host build of the far-field arithmetic header (no GPU code runs):
// lets the CPU test suite compare the 12-channel scaled form against the oracle.
#include "stk_math.hpp"

#include <cmath>
#include <vector>

// variant: 0 = FP64, 1 = FP32
template <int P, typename T>
static void run_pt(const double *d, double rho, const double *W, double u[3]) {
    const double R = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const T dh[3] = {T(d[0] / R), T(d[1] / R), T(d[2] / R)};
    const int ng = stk::nidx(P + 1);
    std::vector<T> Wt(6 * ng);
    for (int i = 0; i < 6 * ng; ++i) Wt[i] = T(W[i]);
    T accG[3], accF[3], ut[3];
    stk::FarEval<P, T>::run(dh, T(rho / R), Wt.data(), accG, accF);
    stk::far_velocity(accG, accF, T(1.0 / R), ut);
    for (int i = 0; i < 3; ++i) u[i] = double(ut[i]);
}

static int g_variant = 0;

template <int P> static void run_p(const double *d, double rho, const double *W, double u[3]) {
    switch (g_variant) {
        case 0: run_pt<P, double>(d, rho, W, u); break;
        default: run_pt<P, float>(d, rho, W, u); break;
    }
}

extern "C" {
void hc_set_variant(int v) { g_variant = v; }

// 1 if the stream positions of G^a and E^a (||a|| <= p + 1) cover [0, 6 nidx(p + 1))
// exactly once each
int hc_stream_ok(int p) {
    const int ng = stk::nidx(p + 1);
    std::vector<int> seen(6 * ng, 0);
    for (int a = 0; a < ng; ++a) {
        int q[3], pg, pe;
        stk::kof(a, q);
        stk::stream_pos(p, q, pg, pe);
        for (int c = 0; c < 3; ++c) {
            if (pg + c < 0 || pg + c >= 6 * ng || pe + c < 0 || pe + c >= 6 * ng) return 0;
            seen[pg + c]++;
            seen[pe + c]++;
        }
    }
    for (int v : seen)
        if (v != 1) return 0;
    return stk::stream_off(p, p + 3, 0) == 6 * ng;
}
int hc_gidx(int k1, int k2, int k3) { return stk::gidx(k1, k2, k3); }
void hc_kof(int a, int *k) { stk::kof(a, k); }
double hc_rho(double r) { return stk::rho_of(r); }

// mom: (nm, 12) moments of one cluster; d = x - y_c; r = cluster radius
void hc_far(const double *mom, int p, const double *d, double r, double *u) {
    const int ng = stk::nidx(p + 1);
    const double rho = stk::rho_of(r);
    std::vector<double> W(ng * 6);
    for (int a = 0; a < ng; ++a) {
        int q[3];
        stk::kof(a, q);
        double ge[6];
        stk::phi_ge(mom, 12, p, q, ge);
        const double s = std::pow(rho, -(q[0] + q[1] + q[2]));
        int pg, pe;
        stk::stream_pos(p, q, pg, pe);
        for (int c = 0; c < 3; ++c) {
            W[pg + c] = ge[c] * s;
            W[pe + c] = ge[3 + c] * s / rho;
        }
    }
    switch (p) {
        case 0: run_p<0>(d, rho, W.data(), u); break;
        case 1: run_p<1>(d, rho, W.data(), u); break;
        case 2: run_p<2>(d, rho, W.data(), u); break;
        case 3: run_p<3>(d, rho, W.data(), u); break;
        case 4: run_p<4>(d, rho, W.data(), u); break;
        case 5: run_p<5>(d, rho, W.data(), u); break;
        case 6: run_p<6>(d, rho, W.data(), u); break;
        case 7: run_p<7>(d, rho, W.data(), u); break;
        case 8: run_p<8>(d, rho, W.data(), u); break;
        case 9: run_p<9>(d, rho, W.data(), u); break;
        case 10: run_p<10>(d, rho, W.data(), u); break;
    }
}
}

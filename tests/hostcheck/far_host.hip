// Test-only host build of the far-field arithmetic header (no GPU code runs):
// lets the CPU test suite compare the 12-channel scaled form against the oracle.
#include "stk_math.hpp"

#include <cmath>
#include <vector>

template <int P> static void run_p(const double *d, double rho, const double *W, double u[3]) {
    const double R = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double dh[3] = {d[0] / R, d[1] / R, d[2] / R};
    const int ng = stk::nidx(P + 1);
    double accG[3], accF[3];
    stk::FarEval<P, double>::run(dh, rho / R, W, W + 3 * ng, accG, accF);
    stk::far_velocity(accG, accF, 1.0 / R, u);
}

extern "C" {
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
        for (int c = 0; c < 3; ++c) {
            W[3 * a + c] = ge[c] * s;
            W[3 * ng + 3 * a + c] = ge[3 + c] * s / rho;
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

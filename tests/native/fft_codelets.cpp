// Host check of the FFT codelets and plans of fft_device.h: every codelet,
// forward and inverse, against the DFT by its definition in double, and the
// pass plan of every transform length the canvas edges use.  Prints one line
// per check; exit status 1 if any fails.
#include <cmath>
#include <cstdio>
#include <complex>
#include <vector>

#include "fft_device.h"

using namespace regdock;

template <int R, bool INV>
static double codelet_error() {
    double worst = 0.0;
    unsigned seed = 12345u + 17u * R + (INV ? 1u : 0u);
    auto rnd = [&]() {
        seed = seed * 1664525u + 1013904223u;
        return (double)(seed >> 8) / (double)(1u << 24) - 0.5;
    };
    for (int trial = 0; trial < 20; ++trial) {
        float2 v[R];
        std::complex<double> x[R];
        for (int j = 0; j < R; ++j) {
            v[j] = make_float2((float)rnd(), (float)rnd());
            x[j] = std::complex<double>(v[j].x, v[j].y);
        }
        Dft<R, INV>::run(v);
        const double sg = INV ? 1.0 : -1.0;
        for (int k = 0; k < R; ++k) {
            std::complex<double> X = 0.0;
            for (int j = 0; j < R; ++j) X += x[j] * std::polar(1.0, sg * 2.0 * M_PI * (double)j * k / R);
            worst = std::fmax(worst, std::abs(X - std::complex<double>(v[k].x, v[k].y)));
        }
    }
    return worst;
}

template <int R>
static int check() {
    const double ef = codelet_error<R, false>(), ei = codelet_error<R, true>();
    // float32 inputs of magnitude <= 0.5: a few ulps of sqrt(R)
    const double bar = 8.0 * 6e-8 * std::sqrt((double)R) * R;
    const bool ok = ef <= bar && ei <= bar;
    std::printf("codelet %2d: forward %.2e inverse %.2e (bar %.2e) %s\n", R, ef, ei, bar, ok ? "ok" : "FAIL");
    return ok ? 0 : 1;
}

int main() {
    int bad = 0;
    bad += check<2>() + check<3>() + check<4>() + check<5>() + check<8>() + check<16>();
    bad += check<6>() + check<9>() + check<10>() + check<12>() + check<15>();
    // the fused plane passes' edges take at most two LDS passes per
    // transform; the split passes' edges (192, 256, 360) at most three
    const int edges[] = {16, 32, 48, 60, 64, 80, 96, 120, 128, 160, 180, 192, 256, 360};
    for (int n : edges)
        for (int L : {n, n / 2}) {
            const int max_passes = n <= 180 ? 2 : 3;
            int prod = 1, np = fft_npass(L);
            std::printf("plan %3d:", L);
            for (int p = 0; p < np; ++p) {
                std::printf(" %d", fft_radix(L, p));
                prod *= fft_radix(L, p);
            }
            const bool ok = prod == L && np <= max_passes && fft_supported(L);
            std::printf(" (%d passes) %s\n", np, ok ? "ok" : "FAIL");
            bad += ok ? 0 : 1;
        }
    return bad ? 1 : 0;
}

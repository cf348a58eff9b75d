// Host-side check of the in-register DFTs and the four-step passes of
// fft.h against a direct O(N^2) double-precision DFT.  Threads of one line
// are emulated one after the other; the LDS buffer is a plain array, and a
// lane pair's swap (pass B with L = 2) is emulated by handing each lane its
// partner's values.  Also checks that out(t, i) covers every index once.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2308_10674_amd/csrc/fft.h"

using namespace ptyc;

static double direct_err(const std::vector<cf>& x, const std::vector<cf>& X, int dir) {
    const int n = (int)x.size();
    double num = 0, den = 0;
    for (int k = 0; k < n; ++k) {
        double re = 0, im = 0;
        for (int j = 0; j < n; ++j) {
            double a = dir * 2.0 * M_PI * (double)((long)j * k % n) / n;
            re += x[j].x * std::cos(a) - x[j].y * std::sin(a);
            im += x[j].x * std::sin(a) + x[j].y * std::cos(a);
        }
        num += (re - X[k].x) * (re - X[k].x) + (im - X[k].y) * (im - X[k].y);
        den += re * re + im * im;
    }
    return std::sqrt(num / den);
}

template <int R>
static int check_small() {
    std::mt19937 g(R);
    std::normal_distribution<float> d;
    std::vector<cf> x(R), X(R);
    for (auto& v : x) v = cf{d(g), d(g)};
    cf v[R];
    for (int i = 0; i < R; ++i) v[i] = x[i];
    dft<R, -1>(v);
    for (int i = 0; i < R; ++i) X[i] = v[i];
    double ef = direct_err(x, X, -1);
    for (int i = 0; i < R; ++i) v[i] = x[i];
    dft<R, +1>(v);
    for (int i = 0; i < R; ++i) X[i] = v[i];
    double eb = direct_err(x, X, +1);
    std::printf("dft%-3d fwd %.2e inv %.2e\n", R, ef, eb);
    return (ef < 1e-6 && eb < 1e-6) ? 0 : 1;
}

template <int N>
static int check_line() {
    constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2;
    std::vector<cf> tw(N);
    for (int m = 0; m < N; ++m)
        tw[m] = cf{(float)std::cos(-2.0 * M_PI * m / N), (float)std::sin(-2.0 * M_PI * m / N)};
    std::mt19937 g(N);
    std::normal_distribution<float> d;
    std::vector<cf> x(N), X(N), y(N);
    for (auto& v : x) v = cf{d(g), d(g)};
    std::vector<cf> z(Lds<N>::LINE);
    std::vector<std::vector<cf>> regs(N2, std::vector<cf>(N1));
    for (int t = 0; t < N2; ++t) {
        for (int n1 = 0; n1 < N1; ++n1) regs[t][n1] = x[N2 * n1 + t];
        cf w[N1];
        twiddles_a<N, -1>(w, t, tw.data());
        passA_to_lds<N, -1>(regs[t].data(), z.data(), t, w);
    }
    if constexpr (Fact<N>::L == 1) {
        for (int t = 0; t < N2; ++t) passB1_from_lds<N, -1>(regs[t].data(), z.data(), t);
    } else {
        // lane pairs: every lane's local part first, then each combines with
        // its partner's local result (what the lane swap delivers on the GPU)
        for (int t = 0; t < N2; ++t) passB2_local<N, -1>(regs[t].data(), z.data(), t);
        auto local = regs;
        for (int t = 0; t < N2; ++t) passB2_combine<N>(regs[t].data(), local[t ^ 1].data(), t);
    }
    for (int t = 0; t < N2; ++t)
        for (int i = 0; i < N1; ++i) X[Fact<N>::out(t, i)] = regs[t][i];
    {
        std::vector<int> seen(N, 0);
        for (int t = 0; t < N2; ++t)
            for (int i = 0; i < N1; ++i) ++seen[Fact<N>::out(t, i)];
        for (int k = 0; k < N; ++k)
            if (seen[k] != 1) {
                std::printf("line%-4d out() covers index %d %d times\n", N, k, seen[k]);
                return 1;
            }
    }
    double ef = direct_err(x, X, -1);
    // inverse back from the pass-B distribution
    if constexpr (Fact<N>::L == 1) {
        for (int t = 0; t < N2; ++t) {
            cf w[N1];
            twiddles_binv<N, +1>(w, t, tw.data());
            passB1inv_to_lds<N, +1>(regs[t].data(), z.data(), t, w);
        }
    } else {
        auto held = regs;
        for (int t = 0; t < N2; ++t) {
            passB2inv_combine<N, +1>(regs[t].data(), held[t ^ 1].data(), t);
            cf w[N1];
            twiddles_binv<N, +1>(w, t, tw.data());
            passB2inv_local_to_lds<N, +1>(regs[t].data(), z.data(), t, w);
        }
    }
    double eb = 0, den = 0;
    for (int t = 0; t < N2; ++t) {
        passAinv_from_lds<N, +1>(regs[t].data(), z.data(), t);
        for (int n1 = 0; n1 < N1; ++n1) {
            cf r = regs[t][n1];
            cf o = x[N2 * n1 + t];
            eb += (r.x / N - o.x) * (r.x / N - o.x) + (r.y / N - o.y) * (r.y / N - o.y);
            den += o.x * o.x + o.y * o.y;
        }
    }
    eb = std::sqrt(eb / den);
    std::printf("line%-4d fwd %.2e roundtrip %.2e\n", N, ef, eb);
    return (ef < 2e-6 && eb < 2e-6) ? 0 : 1;
}

int main() {
    int bad = 0;
    bad += check_small<2>() + check_small<4>() + check_small<8>() + check_small<16>();
    bad += check_line<16>() + check_line<32>() + check_line<64>() + check_line<128>() + check_line<256>();
    std::printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}

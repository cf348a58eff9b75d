// Complex FP32 arithmetic and small in-register DFTs for the ePIE kernels.
//
// A length-N transform (N = N1 * N2) is computed by the four-step
// factorisation: with n = N2*n1 + n2 and k = k1 + N1*k2,
//   X[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) W_N^(n2 k1) sum_n1 x[N2 n1 + n2] W_N1^(n1 k1)
// so a group of N2 threads first runs N2 DFTs of length N1 in registers
// (pass A), multiplies by W_N^(n2 k1), exchanges through LDS and runs N1
// DFTs of length N2 (pass B).  The inverse runs the same passes backwards
// (B^-1 then A^-1) and ends in the distribution the forward pass started
// from.  The small DFTs below use exact mathematical constants; the N-point
// twiddles come from a table computed in double precision on the host.
#pragma once

#include <hip/hip_runtime.h>

namespace ptyc {

struct __align__(8) cf {
    float x, y;
};

__host__ __device__ inline cf mk(float x, float y) { return cf{x, y}; }
__host__ __device__ inline cf operator+(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cf operator-(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cf operator*(float s, cf a) { return cf{s * a.x, s * a.y}; }
// The library is compiled without floating-point contraction, so which
// multiplications fuse with an addition is fixed here, in the source, and
// every kernel that uses these helpers rounds the same way whatever code
// surrounds them (the launch forms and tile variants give the same bits).
__host__ __device__ inline float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ inline cf cmul(cf a, cf b) {
    return cf{fma_(a.x, b.x, -(a.y * b.y)), fma_(a.x, b.y, a.y * b.x)};
}
// conj(a) * b
__host__ __device__ inline cf cmulc(cf a, cf b) {
    return cf{fma_(a.x, b.x, a.y * b.y), fma_(a.x, b.y, -(a.y * b.x))};
}
// y + s x
__host__ __device__ inline cf axpy(float s, cf x, cf y) { return cf{fma_(s, x.x, y.x), fma_(s, x.y, y.y)}; }
__host__ __device__ inline float norm2(cf a) { return fma_(a.x, a.x, a.y * a.y); }

// multiply by DIR*i (DIR = -1 forward, +1 inverse): W_4^1 of that direction
template <int DIR>
__host__ __device__ inline cf rot(cf v) {
    return DIR < 0 ? cf{v.y, -v.x} : cf{-v.y, v.x};
}

// multiply by the constant (c + DIR*i*s)
template <int DIR>
__host__ __device__ inline cf twc(cf v, float c, float s) {
    const float sd = DIR < 0 ? -s : s;
    return cf{fma_(v.x, c, -(v.y * sd)), fma_(v.x, sd, v.y * c)};
}

// cos and sin of pi/8 and pi/4 (mathematical constants)
constexpr float kC8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float kS8 = 0.38268343236508977173f;   // sin(pi/8)
constexpr float kR2 = 0.70710678118654752440f;   // cos(pi/4) = sin(pi/4)

template <int DIR>
__host__ __device__ inline void dft2(cf& a, cf& b) {
    cf t = a - b;
    a = a + b;
    b = t;
}

// v[0..3] -> natural-order DFT of length 4
template <int DIR>
__host__ __device__ inline void dft4(cf& v0, cf& v1, cf& v2, cf& v3) {
    cf t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = rot<DIR>(v1 - v3);
    v0 = t0 + t2;
    v2 = t0 - t2;
    v1 = t1 + t3;
    v3 = t1 - t3;
}

// natural-order DFT of length 8 (radix-2 split of two length-4 DFTs)
template <int DIR>
__host__ __device__ inline void dft8(cf* v) {
    cf e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cf o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = twc<DIR>(o1, kR2, kR2);       // W_8^1
    o2 = rot<DIR>(o2);                 // W_8^2
    o3 = twc<DIR>(o3, -kR2, kR2);      // W_8^3
    v[0] = e0 + o0; v[4] = e0 - o0;
    v[1] = e1 + o1; v[5] = e1 - o1;
    v[2] = e2 + o2; v[6] = e2 - o2;
    v[3] = e3 + o3; v[7] = e3 - o3;
}

// natural-order DFT of length 16 (four-step 4 x 4)
template <int DIR>
__host__ __device__ inline void dft16(cf* v) {
    cf y[16];
    // DFTs of length 4 over n1 for each n2: inputs x[4 n1 + n2]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cf a = v[n2], b = v[4 + n2], c = v[8 + n2], d = v[12 + n2];
        dft4<DIR>(a, b, c, d);
        y[0 * 4 + n2] = a;   // y[k1*4 + n2]
        y[1 * 4 + n2] = b;
        y[2 * 4 + n2] = c;
        y[3 * 4 + n2] = d;
    }
    // twiddles W_16^(n2 k1)
    y[1 * 4 + 1] = twc<DIR>(y[1 * 4 + 1], kC8, kS8);    // m = 1
    y[1 * 4 + 2] = twc<DIR>(y[1 * 4 + 2], kR2, kR2);    // m = 2
    y[1 * 4 + 3] = twc<DIR>(y[1 * 4 + 3], kS8, kC8);    // m = 3
    y[2 * 4 + 1] = twc<DIR>(y[2 * 4 + 1], kR2, kR2);    // m = 2
    y[2 * 4 + 2] = rot<DIR>(y[2 * 4 + 2]);              // m = 4
    y[2 * 4 + 3] = twc<DIR>(y[2 * 4 + 3], -kR2, kR2);   // m = 6
    y[3 * 4 + 1] = twc<DIR>(y[3 * 4 + 1], kS8, kC8);    // m = 3
    y[3 * 4 + 2] = twc<DIR>(y[3 * 4 + 2], -kR2, kR2);   // m = 6
    y[3 * 4 + 3] = twc<DIR>(y[3 * 4 + 3], -kC8, -kS8);  // m = 9
    // DFTs of length 4 over n2 for each k1: output X[k1 + 4 k2]
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cf a = y[k1 * 4 + 0], b = y[k1 * 4 + 1], c = y[k1 * 4 + 2], d = y[k1 * 4 + 3];
        dft4<DIR>(a, b, c, d);
        v[k1 + 0] = a;
        v[k1 + 4] = b;
        v[k1 + 8] = c;
        v[k1 + 12] = d;
    }
}

template <int R, int DIR>
__host__ __device__ inline void dft(cf* v) {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
    if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
    else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<DIR>(v);
    else dft16<DIR>(v);
}

// Factorisation N = N1 * N2 used for each supported pattern size.
// T = N2 threads cooperate on one length-N transform; each holds N1 points.
// L = 1: pass B runs N1/N2 DFTs of length N2 in each thread (N1 >= N2).
// L = 2: N2 = 2 N1 and every DFT of length N2 of pass B is shared by a pair
// of lanes (t, t ^ 1): each runs a length-N1 DFT of the even or the odd
// inputs, the odd lane twiddles by W_N2^k, and the pair swaps halves
// (X[k] = E[k] + W^k O[k], X[k + N1] = E[k] - W^k O[k]).  Fewer points per
// thread means twice the threads per line, which is what a batch of a few
// dozen patterns needs to fill the chip.
// out(t, i): the index of the spectrum value thread t holds in v[i] after
// pass B (and must hold before the inverse of pass B).
template <int N> struct Fact;
template <int N1_, int N2_> struct FactL1 {
    static constexpr int N1 = N1_, N2 = N2_, L = 1;
    static_assert(N1 % N2 == 0, "pass B groups");
    __host__ __device__ static inline int out(int t, int i) { return (t + N2 * (i / N2)) + N1 * (i % N2); }
};
template <int N1_> struct FactL2 {
    static constexpr int N1 = N1_, N2 = 2 * N1_, L = 2;
    static_assert(N2 == 8 || N2 == 16, "the pair twiddles W_N2^k are taken from W_16");
    __host__ __device__ static inline int out(int t, int i) { return (t >> 1) + N1 * i + N1 * N1 * (t & 1); }
};
template <> struct Fact<16>  : FactL1<4, 4> {};
template <> struct Fact<32>  : FactL2<4> {};
template <> struct Fact<64>  : FactL1<8, 8> {};
template <> struct Fact<128> : FactL2<8> {};
template <> struct Fact<256> : FactL1<16, 16> {};

// multiply by W_16^k of direction DIR, k < 8 (exact constants)
template <int DIR>
__host__ __device__ inline cf w16(cf v, int k) {
    switch (k) {
        case 1: return twc<DIR>(v, kC8, kS8);
        case 2: return twc<DIR>(v, kR2, kR2);
        case 3: return twc<DIR>(v, kS8, kC8);
        case 4: return rot<DIR>(v);
        case 5: return twc<DIR>(v, -kS8, kC8);
        case 6: return twc<DIR>(v, -kR2, kR2);
        case 7: return twc<DIR>(v, -kC8, kS8);
        default: return v;
    }
}

// LDS exchange buffer of one length-N line: Z[k1][n2] at k1*(N2+1) + n2,
// padded to an odd number of complex slots per line.
template <int N>
struct Lds {
    static constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2;
    static constexpr int RAW = N1 * (N2 + 1);
    static constexpr int LINE = (RAW % 2 == 0) ? RAW + 1 : RAW;
    __host__ __device__ static inline int at(int k1, int n2) { return k1 * (N2 + 1) + n2; }
};

// The W_N twiddles one thread applies, taken from tw[m] = exp(-2 pi i m / N),
// m < N, into registers ahead of the pass (so a kernel can issue these
// loads before its other memory traffic): N1 per thread for pass A
// (w[k1] = W_N^(DIR t k1)) and N1 for the inverse of pass B (w[i] = the
// factor of the i-th element the thread writes).
template <int N, int DIR>
__host__ __device__ inline void twiddles_a(cf* w, int t, const cf* __restrict__ tw) {
#pragma unroll
    for (int k1 = 0; k1 < Fact<N>::N1; ++k1) {
        cf x = tw[t * k1];
        if (DIR > 0) x.y = -x.y;
        w[k1] = x;
    }
}

template <int N, int DIR>
__host__ __device__ inline void twiddles_binv(cf* w, int t, const cf* __restrict__ tw) {
    constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2;
    if constexpr (Fact<N>::L == 1) {
#pragma unroll
        for (int m = 0; m < N1 / N2; ++m)
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) {
                cf x = tw[n2 * (t + N2 * m)];
                if (DIR > 0) x.y = -x.y;
                w[m * N2 + n2] = x;
            }
    } else {
        const int k1 = t >> 1, h = t & 1;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            cf x = tw[(2 * m + h) * k1];
            if (DIR > 0) x.y = -x.y;
            w[m] = x;
        }
    }
}

// Pass A of a transform in direction DIR.  In: v[n1] = x[N2 n1 + t].
// Out: Z[k1][t] = W_N^(DIR t k1) * sum_n1 x[N2 n1 + t] W_N1^(DIR n1 k1);
// w = twiddles_a<N, DIR>.
template <int N, int DIR>
__host__ __device__ inline void passA_to_lds(cf* v, cf* z, int t, const cf* w) {
    constexpr int N1 = Fact<N>::N1;
    dft<N1, DIR>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) z[Lds<N>::at(k1, t)] = (k1 == 0) ? v[k1] : cmul(v[k1], w[k1]);
}

// Pass B with L = 1.  Thread t handles k1 = t + N2 m, m < N1/N2.
// Out: v[m N2 + k2] = X[(t + N2 m) + N1 k2].
template <int N, int DIR>
__host__ __device__ inline void passB1_from_lds(cf* v, const cf* z, int t) {
    constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2;
#pragma unroll
    for (int m = 0; m < N1 / N2; ++m) {
        cf u[N2];
        const int k1 = t + N2 * m;
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) u[n2] = z[Lds<N>::at(k1, n2)];
        dft<N2, DIR>(u);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) v[m * N2 + k2] = u[k2];
    }
}

// Inverse of pass B with L = 1: from v[m N2 + k2] = X[(t + N2 m) + N1 k2]
// to Z[k1][n2] = W_N^(DIR n2 k1) * sum_k2 X[k1 + N1 k2] W_N2^(DIR n2 k2) for
// the transform direction DIR (the conjugate of the forward direction);
// w = twiddles_binv<N, DIR>.
template <int N, int DIR>
__host__ __device__ inline void passB1inv_to_lds(cf* v, cf* z, int t, const cf* w) {
    constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2;
#pragma unroll
    for (int m = 0; m < N1 / N2; ++m) {
        cf u[N2];
        const int k1 = t + N2 * m;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) u[k2] = v[m * N2 + k2];
        dft<N2, DIR>(u);
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) z[Lds<N>::at(k1, n2)] = cmul(u[n2], w[m * N2 + n2]);
    }
}

// Pass B with L = 2, the part each lane does alone: thread t = 2 k1 + h
// reads Z[k1][2 m + h], m < N1, runs the length-N1 DFT (E for h = 0, O for
// h = 1) and the odd lane multiplies by W_N2^k.
template <int N, int DIR>
__host__ __device__ inline void passB2_local(cf* v, const cf* z, int t) {
    constexpr int N1 = Fact<N>::N1;
    const int k1 = t >> 1, h = t & 1;
#pragma unroll
    for (int m = 0; m < N1; ++m) v[m] = z[Lds<N>::at(k1, 2 * m + h)];
    dft<N1, DIR>(v);
    if (h) {
#pragma unroll
        for (int k = 1; k < N1; ++k) v[k] = w16<DIR>(v[k], k * (16 / Fact<N>::N2));   // W_N2^k
    }
}

// The pair's combination, p = the partner lane's v: the even lane keeps
// E + W O = X[k1 + N1 k], the odd lane E - W O = X[k1 + N1 (k + N1)].
template <int N>
__host__ __device__ inline void passB2_combine(cf* v, const cf* p, int t) {
    const float sg = (t & 1) ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < Fact<N>::N1; ++i) v[i] = p[i] + sg * v[i];
}

// Inverse of pass B with L = 2, first the pair step: with p = the partner's
// v (the even lane holds X[k1 + N1 k], the odd lane X[k1 + N1 (k + N1)]),
// the even lane forms X[k] + X[k + N1] and the odd lane
// (X[k] - X[k + N1]) W_N2^(DIR k).
template <int N, int DIR>
__host__ __device__ inline void passB2inv_combine(cf* v, const cf* p, int t) {
    const float sg = (t & 1) ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < Fact<N>::N1; ++i) v[i] = p[i] + sg * v[i];
    if (t & 1) {
#pragma unroll
        for (int k = 1; k < Fact<N>::N1; ++k) v[k] = w16<DIR>(v[k], k * (16 / Fact<N>::N2));   // W_N2^k
    }
}

// ... then each lane alone: the length-N1 DFT gives Z'[k1][2 m + h], which
// is twiddled by W_N^(DIR n2 k1) into the LDS line (w = twiddles_binv).
template <int N, int DIR>
__host__ __device__ inline void passB2inv_local_to_lds(cf* v, cf* z, int t, const cf* w) {
    constexpr int N1 = Fact<N>::N1;
    const int k1 = t >> 1, h = t & 1;
    dft<N1, DIR>(v);
#pragma unroll
    for (int m = 0; m < N1; ++m) z[Lds<N>::at(k1, 2 * m + h)] = cmul(v[m], w[m]);
}

// Inverse of pass A: thread t = n2 reads Z[k1][t], k1 < N1, and ends with
// v[n1] = x[N2 n1 + t].
template <int N, int DIR>
__host__ __device__ inline void passAinv_from_lds(cf* v, const cf* z, int t) {
    constexpr int N1 = Fact<N>::N1;
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = z[Lds<N>::at(k1, t)];
    dft<N1, DIR>(v);
}

// Device forms of pass B and its inverse.  XOR is the lane distance of the
// two threads t and t ^ 1 of a line (1 when t is the fastest thread index,
// the column tile width when the columns are).
template <int XOR>
__device__ inline cf lane_swap(cf v) {
    static_assert(XOR > 0 && XOR < 64 && (XOR & (XOR - 1)) == 0, "lane distance");
    if constexpr (XOR == 1 || XOR == 2) {
        // neighbours within a quad: a DPP quad permutation ([1,0,3,2] or
        // [2,3,0,1]), a modifier of a VALU move instead of a trip through
        // the LDS crossbar
        constexpr int ctrl = XOR == 1 ? 0xB1 : 0x4E;
        return cf{__int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.x), ctrl, 0xF, 0xF, false)),
                  __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.y), ctrl, 0xF, 0xF, false))};
    } else {
        return cf{__shfl_xor(v.x, XOR, 64), __shfl_xor(v.y, XOR, 64)};
    }
}

template <int N, int DIR, int XOR>
__device__ inline void passB_from_lds(cf* v, const cf* z, int t) {
    if constexpr (Fact<N>::L == 1) {
        passB1_from_lds<N, DIR>(v, z, t);
    } else {
        passB2_local<N, DIR>(v, z, t);
        cf p[Fact<N>::N1];
#pragma unroll
        for (int i = 0; i < Fact<N>::N1; ++i) p[i] = lane_swap<XOR>(v[i]);
        passB2_combine<N>(v, p, t);
    }
}

template <int N, int DIR, int XOR>
__device__ inline void passBinv_to_lds(cf* v, cf* z, int t, const cf* w) {
    if constexpr (Fact<N>::L == 1) {
        passB1inv_to_lds<N, DIR>(v, z, t, w);
    } else {
        cf p[Fact<N>::N1];
#pragma unroll
        for (int i = 0; i < Fact<N>::N1; ++i) p[i] = lane_swap<XOR>(v[i]);
        passB2inv_combine<N, DIR>(v, p, t);
        passB2inv_local_to_lds<N, DIR>(v, z, t, w);
    }
}

}  // namespace ptyc

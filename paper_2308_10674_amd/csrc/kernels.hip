// HIP kernels of the ePIE position update for gfx950.
//
// One batch of positions with pairwise disjoint windows runs in four
// launches (the stage split lets an N x N spectrum span several workgroups):
//   rows_fwd   psi = P * S_j O, 1D FFT of every row           -> scratch
//   cols       1D FFT of every column, modulus replacement with sqrt(I_j)
//              and the error partial, inverse 1D FFT of the column -> scratch
//   rows_inv   inverse 1D FFT of every row, scale 1/N^2, Delta = psi' - psi,
//              object step into O and probe increment into dprobe
//   probe      P += beta/|B| * sum of the batch's increments (slot order),
//              and the partial maxima of |P|^2 for the next batch
// The method is the ePIE update of Maiden & Rodenburg 2009 as used in the
// paper's "ePIE Implementation" section; the batch semantics (shared probe
// inside a batch, batch-mean probe step) make batch members commute.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ptyc {

namespace {

constexpr int kWave = 64;

__device__ inline float wave_max(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// block-wide max; every thread gets the result
template <int NT>
__device__ inline float block_max(float v, float* sh) {
    v = wave_max(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float m = sh[0];
#pragma unroll
    for (int i = 1; i < NT / kWave; ++i) m = fmaxf(m, sh[i]);
    __syncthreads();
    return m;
}

// block-wide sum in a fixed order; the result is valid in thread 0
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / kWave; ++i) s += sh[i];
    }
    return s;
}

// rows per row-stage workgroup / columns per column-stage workgroup
template <int N> struct Tile;
template <> struct Tile<16>  { static constexpr int RB = 16, CB = 16; };
template <> struct Tile<32>  { static constexpr int RB = 32, CB = 32; };
template <> struct Tile<64>  { static constexpr int RB = 32, CB = 32; };
template <> struct Tile<128> { static constexpr int RB = 32, CB = 32; };
template <> struct Tile<256> { static constexpr int RB = 16, CB = 16; };

template <int N> struct Geo {
    static constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2, T = N2;
    static constexpr int RB = Tile<N>::RB, CB = Tile<N>::CB;
    static constexpr int G = N / RB;          // row blocks per position
    static constexpr int GC = N / CB;         // column blocks per position
    static constexpr int NT_ROW = RB * T;     // threads per row-stage workgroup
    static constexpr int NT_COL = CB * T;     // threads per column-stage workgroup
    static constexpr int NT_PROBE = 256;
    static constexpr int PB = (N * N + NT_PROBE - 1) / NT_PROBE;  // probe blocks
};

// ---------------------------------------------------------------- stage 1
template <int N>
__global__ __launch_bounds__(Geo<N>::NT_ROW) void k_rows_fwd(BatchArgs a) {
    using g = Geo<N>;
    __shared__ cf lds[g::RB * Lds<N>::LINE];
    __shared__ float red[g::NT_ROW / kWave];
    const int slot = blockIdx.x / g::G, rb = blockIdx.x % g::G;
    const int64_t j = a.order[a.off + slot];
    const int2 p0 = a.pos[j];
    const int t = threadIdx.x % g::T, rl = threadIdx.x / g::T;
    const int r = rb * g::RB + rl;
    const cf* orow = a.obj + (size_t)(p0.x + r) * a.w + p0.y;
    const cf* prow = a.probe + (size_t)r * N;
    cf v[g::N1];
    float m = 0.f;
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) {
        const int col = g::N2 * n1 + t;
        const cf o = orow[col];
        m = fmaxf(m, norm2(o));
        v[n1] = cmul(prow[col], o);
    }
    cf* z = lds + rl * Lds<N>::LINE;
    passA_to_lds<N, -1>(v, z, t, a.tw);
    __syncthreads();
    passB_from_lds<N, -1>(v, z, t);
    cf* srow = a.scratch + (size_t)slot * N * N + (size_t)r * N;
#pragma unroll
    for (int mm = 0; mm < g::N1 / g::N2; ++mm)
#pragma unroll
        for (int k2 = 0; k2 < g::N2; ++k2) srow[(t + g::N2 * mm) + g::N1 * k2] = v[mm * g::N2 + k2];
    m = block_max<g::NT_ROW>(m, red);
    if (threadIdx.x == 0) a.winmax[slot * g::G + rb] = m;
}

// ---------------------------------------------------------------- stage 2
template <int N>
__global__ __launch_bounds__(Geo<N>::NT_COL) void k_cols(BatchArgs a) {
    using g = Geo<N>;
    __shared__ cf lds[g::CB * Lds<N>::LINE];
    __shared__ double red[g::NT_COL / kWave];
    const int slot = blockIdx.x / g::GC, cb = blockIdx.x % g::GC;
    const int64_t j = a.order[a.off + slot];
    const int cl = threadIdx.x % g::CB, t = threadIdx.x / g::CB;
    const int c = cb * g::CB + cl;
    cf* base = a.scratch + (size_t)slot * N * N + c;
    cf v[g::N1];
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) v[n1] = base[(size_t)(g::N2 * n1 + t) * N];
    cf* z = lds + cl * Lds<N>::LINE;
    passA_to_lds<N, -1>(v, z, t, a.tw);
    __syncthreads();
    passB_from_lds<N, -1>(v, z, t);
    // modulus replacement Psi' = sqrt(I) sgn(Psi), running error
    const float* amp = a.sqrt_i + (size_t)j * N * N + c;
    float e = 0.f;
#pragma unroll
    for (int mm = 0; mm < g::N1 / g::N2; ++mm)
#pragma unroll
        for (int k2 = 0; k2 < g::N2; ++k2) {
            const int row = (t + g::N2 * mm) + g::N1 * k2;
            const float s = amp[(size_t)row * N];
            const cf zz = v[mm * g::N2 + k2];
            const float mag = sqrtf(norm2(zz));
            const float d = mag - s;
            e += d * d;
            const float f = mag > 0.f ? s / mag : 0.f;
            v[mm * g::N2 + k2] = f * zz;
        }
    __syncthreads();
    passBinv_to_lds<N, +1>(v, z, t, a.tw);
    __syncthreads();
    passAinv_from_lds<N, +1>(v, z, t);
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) base[(size_t)(g::N2 * n1 + t) * N] = v[n1];
    const double tot = block_sum<g::NT_COL>((double)e, red);
    if (threadIdx.x == 0) a.err_part[(a.off + slot) * g::GC + cb] = tot;
}

// ---------------------------------------------------------------- stage 3
template <int N>
__global__ __launch_bounds__(Geo<N>::NT_ROW) void k_rows_inv(BatchArgs a) {
    using g = Geo<N>;
    __shared__ cf lds[g::RB * Lds<N>::LINE];
    __shared__ float red[g::NT_ROW / kWave];
    const int slot = blockIdx.x / g::G, rb = blockIdx.x % g::G;
    const int64_t j = a.order[a.off + slot];
    const int2 p0 = a.pos[j];
    const int t = threadIdx.x % g::T, rl = threadIdx.x / g::T;
    const int r = rb * g::RB + rl;
    // max |P|^2 over the probe blocks, max |S_j O|^2 over the row blocks
    float pm = 0.f;
    for (int i = threadIdx.x; i < a.npmax; i += g::NT_ROW) pm = fmaxf(pm, a.pmax_part[i]);
    pm = block_max<g::NT_ROW>(pm, red);
    float om = 0.f;
    for (int i = threadIdx.x; i < g::G; i += g::NT_ROW) om = fmaxf(om, a.winmax[slot * g::G + i]);
    om = block_max<g::NT_ROW>(om, red);
    const float ostep = a.alpha / pm;
    const float pstep = 1.f / om;

    const cf* srow = a.scratch + (size_t)slot * N * N + (size_t)r * N;
    cf v[g::N1];
#pragma unroll
    for (int mm = 0; mm < g::N1 / g::N2; ++mm)
#pragma unroll
        for (int k2 = 0; k2 < g::N2; ++k2) v[mm * g::N2 + k2] = srow[(t + g::N2 * mm) + g::N1 * k2];
    cf* z = lds + rl * Lds<N>::LINE;
    passBinv_to_lds<N, +1>(v, z, t, a.tw);
    __syncthreads();
    passAinv_from_lds<N, +1>(v, z, t);
    constexpr float inv = 1.0f / (float)(N * N);
    cf* orow = a.obj + (size_t)(p0.x + r) * a.w + p0.y;
    const cf* prow = a.probe + (size_t)r * N;
    cf* drow = a.dprobe + (size_t)slot * N * N + (size_t)r * N;
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) {
        const int col = g::N2 * n1 + t;
        const cf o = orow[col];
        const cf p = prow[col];
        const cf delta = inv * v[n1] - cmul(p, o);
        orow[col] = o + ostep * cmulc(p, delta);
        drow[col] = pstep * cmulc(o, delta);
    }
}

// ---------------------------------------------------------------- stage 4
template <int N>
__global__ __launch_bounds__(Geo<N>::NT_PROBE) void k_probe(BatchArgs a) {
    using g = Geo<N>;
    __shared__ float red[g::NT_PROBE / kWave];
    const int e = blockIdx.x * g::NT_PROBE + threadIdx.x;
    float m = 0.f;
    if (e < N * N) {
        cf p = a.probe[e];
        if (a.bsize > 0) {
            cf acc = a.dprobe[e];
            for (int s = 1; s < a.bsize; ++s) acc = acc + a.dprobe[(size_t)s * N * N + e];
            p = p + (a.beta / (float)a.bsize) * acc;
            a.probe[e] = p;
        }
        m = norm2(p);
    }
    m = block_max<g::NT_PROBE>(m, red);
    if (threadIdx.x == 0) a.pmax_part[blockIdx.x] = m;
}

// ---------------------------------------------------------------- ingest
template <int N>
__global__ __launch_bounds__(256) void k_ingest(const float* __restrict__ src, float* dst,
                                                double* sum_i, int is_sqrt, int centred,
                                                int* bad) {
    __shared__ double red[256 / kWave];
    const size_t i = blockIdx.x;
    const float* s = src + i * N * N;
    float* d = dst + i * N * N;
    double acc = 0.0;
    int badl = 0;
    for (int e = threadIdx.x; e < N * N; e += 256) {
        const float x = s[e];
        if (!(x >= 0.f) || !isfinite(x)) badl = 1;
        const float amp = is_sqrt ? x : sqrtf(x);
        acc += is_sqrt ? (double)x * (double)x : (double)x;
        int r = e / N, c = e % N;
        if (centred) {
            r = (r + N / 2) % N;
            c = (c + N / 2) % N;
        }
        d[r * N + c] = amp;
    }
    if (badl) atomicOr(bad, 1);
    const double tot = block_sum<256>(acc, red);
    if (threadIdx.x == 0) sum_i[i] = tot;
}

// ---------------------------------------------------------------- error
__global__ __launch_bounds__(256) void k_err_reduce(const double* err_part, int64_t n_part,
                                                    const int64_t* order, int64_t order_len,
                                                    const double* sum_i, double* out) {
    __shared__ double red[256 / kWave];
    double num = 0.0, den = 0.0;
    for (int64_t i = threadIdx.x; i < n_part; i += 256) num += err_part[i];
    for (int64_t i = threadIdx.x; i < order_len; i += 256) den += sum_i[order[i]];
    num = block_sum<256>(num, red);
    __syncthreads();
    den = block_sum<256>(den, red);
    if (threadIdx.x == 0) *out = den > 0.0 ? num / den : 0.0;
}

template <int N>
hipError_t batch_n(const BatchArgs& a, hipStream_t s) {
    using g = Geo<N>;
    if (a.bsize > 0) {
        hipLaunchKernelGGL(k_rows_fwd<N>, dim3(g::G * a.bsize), dim3(g::NT_ROW), 0, s, a);
        hipLaunchKernelGGL(k_cols<N>, dim3(g::GC * a.bsize), dim3(g::NT_COL), 0, s, a);
        hipLaunchKernelGGL(k_rows_inv<N>, dim3(g::G * a.bsize), dim3(g::NT_ROW), 0, s, a);
    }
    hipLaunchKernelGGL(k_probe<N>, dim3(g::PB), dim3(g::NT_PROBE), 0, s, a);
    return hipGetLastError();
}

template <int N>
hipError_t probe_n(const BatchArgs& a, hipStream_t s) {
    using g = Geo<N>;
    hipLaunchKernelGGL(k_probe<N>, dim3(g::PB), dim3(g::NT_PROBE), 0, s, a);
    return hipGetLastError();
}

template <int N>
hipError_t ingest_n(const float* src, float* dst, double* sum_i, int64_t count, bool is_sqrt,
                    bool centred, int* bad, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ingest<N>, dim3((unsigned)count), dim3(256), 0, s, src, dst, sum_i,
                       (int)is_sqrt, (int)centred, bad);
    return hipGetLastError();
}

template <int N>
Shape shape_n() {
    using g = Geo<N>;
    return Shape{g::G, g::GC, g::PB};
}

}  // namespace

bool supported_n(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }

Shape shape_for(int n) {
    switch (n) {
        case 16: return shape_n<16>();
        case 32: return shape_n<32>();
        case 64: return shape_n<64>();
        case 128: return shape_n<128>();
        case 256: return shape_n<256>();
    }
    return Shape{0, 0, 0};
}

hipError_t launch_batch(int n, const BatchArgs& a, hipStream_t s) {
    switch (n) {
        case 16: return batch_n<16>(a, s);
        case 32: return batch_n<32>(a, s);
        case 64: return batch_n<64>(a, s);
        case 128: return batch_n<128>(a, s);
        case 256: return batch_n<256>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_probe_reduce(int n, const BatchArgs& a, hipStream_t s) {
    switch (n) {
        case 16: return probe_n<16>(a, s);
        case 32: return probe_n<32>(a, s);
        case 64: return probe_n<64>(a, s);
        case 128: return probe_n<128>(a, s);
        case 256: return probe_n<256>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ingest(int n, const float* src, float* dst, double* sum_i, int64_t count,
                         bool is_sqrt, bool centred, int* bad, hipStream_t s) {
    switch (n) {
        case 16: return ingest_n<16>(src, dst, sum_i, count, is_sqrt, centred, bad, s);
        case 32: return ingest_n<32>(src, dst, sum_i, count, is_sqrt, centred, bad, s);
        case 64: return ingest_n<64>(src, dst, sum_i, count, is_sqrt, centred, bad, s);
        case 128: return ingest_n<128>(src, dst, sum_i, count, is_sqrt, centred, bad, s);
        case 256: return ingest_n<256>(src, dst, sum_i, count, is_sqrt, centred, bad, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_err_reduce(const double* err_part, int64_t n_part, const int64_t* order,
                             int64_t order_len, const double* sum_i, double* err_out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_err_reduce, dim3(1), dim3(256), 0, s, err_part, n_part, order, order_len,
                       sum_i, err_out);
    return hipGetLastError();
}

}  // namespace ptyc

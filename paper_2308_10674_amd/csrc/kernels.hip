// HIP kernels of the ePIE position update for gfx950.
//
// One batch of positions with pairwise disjoint windows is updated in three
// stages (an N x N spectrum spans several workgroups, so the 2D transform is
// split into a row pass and a column pass with an exchange buffer between):
//   rows_fwd   psi = P * S_j O and the 1D FFT of each row       -> scratch
//   cols       1D FFT of each column, modulus replacement with sqrt(I_j)
//              and the error partial, inverse 1D FFT of the column -> scratch
//   rows_inv   inverse 1D FFT of each row, psi' = ... / N^2, Delta = psi' - psi,
//              object step into O; one workgroup owns a block of probe rows
//              for every position of the batch and sums their increments
//              conj(S_j O) Delta / max|S_j O|^2 in slot order, then writes
//              P_{b+1} = P_b + beta/|B| * sum and the block's max |P_{b+1}|^2
// The method is the ePIE update (Maiden & Rodenburg 2009) that the paper's
// "ePIE Implementation" section uses; inside a batch every position sees the
// same probe and the probe moves by the batch mean of the increments, so the
// members of a batch commute.
//
// Launch forms: per batch, three kernel launches (k_rows_fwd, k_cols,
// k_rows_inv); or one cooperative kernel per sweep (k_sweep) that runs the
// same stage functions separated by grid-wide barriers.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace ptyc {

namespace {

constexpr int kWave = 64;

// Cross-lane reductions.  Inside a row of 16 lanes they use DPP operand
// controls (a VALU modifier, no trip through the LDS unit): the quad
// permutations [1,0,3,2] and [2,3,0,1], then the half-row and the row
// mirrors.  Each step combines a lane with a partner holding the same
// number of inputs, so after the four steps every lane of the row holds the
// row's result, computed the same way in every lane.  The four rows are
// then combined through readlane (uniform results) in a fixed order.
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane_of(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_of(double v, int lane) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// max over aligned groups of G lanes (G = 2, 4, 8, 16 or 32); every lane of
// a group gets the group's result
template <int G>
__device__ inline float group_max(float v) {
    static_assert(G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group size");
    v = fmaxf(v, dpp<kDppQuadXor1>(v));
    if constexpr (G >= 4) v = fmaxf(v, dpp<kDppQuadXor2>(v));
    if constexpr (G >= 8) v = fmaxf(v, dpp<kDppRowHalfMirror>(v));
    if constexpr (G >= 16) v = fmaxf(v, dpp<kDppRowMirror>(v));
    if constexpr (G >= 32) v = fmaxf(v, __shfl_xor(v, 16, kWave));
    if constexpr (G == 64) v = fmaxf(v, __shfl_xor(v, 32, kWave));
    return v;
}

// max over the wave (uniform result)
__device__ inline float wave_max(float v) {
    v = group_max<16>(v);
    return fmaxf(fmaxf(lane_of(v, 0), lane_of(v, 16)), fmaxf(lane_of(v, 32), lane_of(v, 48)));
}

// sum over the wave in a fixed order (uniform result)
__device__ inline double wave_sum(double v) {
    v += dpp<kDppQuadXor1>(v);
    v += dpp<kDppQuadXor2>(v);
    v += dpp<kDppRowHalfMirror>(v);
    v += dpp<kDppRowMirror>(v);
    return (lane_of(v, 0) + lane_of(v, 16)) + (lane_of(v, 32) + lane_of(v, 48));
}

// The N2 threads of one transform line are lanes of one wave, so the LDS
// exchange between the passes of a line needs only a wave-level ordering:
// a wave's LDS operations execute in issue order, and the fences keep the
// compiler from moving them across this point.
__device__ __forceinline__ void line_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- tiles
// Forward row stage: RB rows of one position per workgroup; column stage: CB
// columns.  Small tiles spread a position over many compute units (a batch
// holds only a few dozen positions, so the stages are latency-bound).  At
// 128 px (16 threads per line) 4 rows (one wave per workgroup) and 16
// columns measured best; 8 or 32 columns per workgroup were slower.
#ifndef PTYC_RB64
#define PTYC_RB64 16
#endif
#ifndef PTYC_CB64
#define PTYC_CB64 16
#endif
#ifndef PTYC_RB128
#define PTYC_RB128 4
#endif
#ifndef PTYC_CB128
#define PTYC_CB128 16
#endif
#ifndef PTYC_RB256
#define PTYC_RB256 16
#endif
#ifndef PTYC_CB256
#define PTYC_CB256 16
#endif
template <int N> struct Tile;
template <> struct Tile<16>  { static constexpr int RB = 16, CB = 16; };
template <> struct Tile<32>  { static constexpr int RB = 32, CB = 32; };
template <> struct Tile<64>  { static constexpr int RB = PTYC_RB64, CB = PTYC_CB64; };
template <> struct Tile<128> { static constexpr int RB = PTYC_RB128, CB = PTYC_CB128; };
template <> struct Tile<256> { static constexpr int RB = PTYC_RB256, CB = PTYC_CB256; };

// Inverse row stage: R rows for S slots at a time (S*R*N2 threads); for the
// probe step thread i < R*N owns element i of the block's R rows.  At 128 px
// S = 40 holds the largest colour batches of a dense raster (36) in one
// round; at 256 px one round of 36 or 40 slots measured no faster than two
// rounds of 32 for the few batches larger than 32.
#ifndef PTYC_IR128
#define PTYC_IR128 1
#endif
#ifndef PTYC_IS128
#define PTYC_IS128 40
#endif
#ifndef PTYC_IR256
#define PTYC_IR256 1
#endif
#ifndef PTYC_IS256
#define PTYC_IS256 32
#endif
template <int N> struct ITile;
template <> struct ITile<16>  { static constexpr int R = 4, S = 4; };
template <> struct ITile<32>  { static constexpr int R = 4, S = 8; };
template <> struct ITile<64>  { static constexpr int R = 4, S = 8; };
template <> struct ITile<128> { static constexpr int R = PTYC_IR128, S = PTYC_IS128; };
template <> struct ITile<256> { static constexpr int R = PTYC_IR256, S = PTYC_IS256; };

// Tile variants of the per-batch kernels among which ptyc_tune chooses at
// run time; variant 0 is the default (the macros above).  The variants only
// group rows, columns and slots into workgroups differently: every row's
// and column's arithmetic, the order of the slot sum and the layouts of the
// partial maxima are the same, so all variants produce the same object and
// probe bit for bit.
struct TileV {
    int rb, cb, r, s;
};
template <int N> struct Variants;
template <> struct Variants<16> {
    static constexpr int K = 1;
    static constexpr TileV v[K] = {{Tile<16>::RB, Tile<16>::CB, ITile<16>::R, ITile<16>::S}};
};
template <> struct Variants<32> {
    static constexpr int K = 1;
    static constexpr TileV v[K] = {{Tile<32>::RB, Tile<32>::CB, ITile<32>::R, ITile<32>::S}};
};
template <> struct Variants<64> {
    static constexpr int K = 2;
    static constexpr TileV v[K] = {{Tile<64>::RB, Tile<64>::CB, ITile<64>::R, ITile<64>::S}, {32, 32, 4, 8}};
};
template <> struct Variants<128> {
    static constexpr int K = 5;
    static constexpr TileV v[K] = {
        {Tile<128>::RB, Tile<128>::CB, ITile<128>::R, ITile<128>::S}, {8, 16, 1, 40}, {16, 16, 1, 40},
        {4, 16, 1, 32}, {8, 16, 1, 32}};
};
template <> struct Variants<256> {
    static constexpr int K = 3;
    static constexpr TileV v[K] = {
        {Tile<256>::RB, Tile<256>::CB, ITile<256>::R, ITile<256>::S}, {8, 16, 1, 32}, {16, 32, 1, 32}};
};

// Tiles of the persistent form: one workgroup size for all stages (B rows
// or columns in the forward stages; R rows for S slots in the inverse stage).
template <int N> struct PTile;
template <> struct PTile<16>  { static constexpr int B = 16, R = 4, S = 4; };
template <> struct PTile<32>  { static constexpr int B = 32, R = 4, S = 8; };
template <> struct PTile<64>  { static constexpr int B = 32, R = 4, S = 8; };
template <> struct PTile<128> { static constexpr int B = 32, R = 2, S = 16; };
template <> struct PTile<256> { static constexpr int B = 16, R = 1, S = 16; };

template <int N, int RB> struct RowG {
    static constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2, T = N2;
    static constexpr int G = N / RB, NT = RB * T;
    static_assert(N % RB == 0 && NT % kWave == 0 && G * (NT / kWave) == N * N2 / kWave, "row tile");
};
template <int N, int CB> struct ColG {
    static constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2, T = N2;
    static constexpr int GC = N / CB, NT = CB * T;
    static_assert(N % CB == 0 && NT % kWave == 0, "column tile");
    // a lane pair of pass B (L = 2) is CB lanes apart and must share a wave
    static_assert(Fact<N>::L == 1 || 2 * CB <= kWave, "column tile too wide for lane pairs");
};
// OWN: probe elements of the block each thread owns (element k NT + tid),
// so a tile may hold more probe rows than it has threads per row group.
template <int N, int R_ = ITile<N>::R, int S_ = ITile<N>::S> struct InvG {
    static constexpr int N1 = Fact<N>::N1, N2 = Fact<N>::N2, T = N2;
    static constexpr int R = R_, S = S_;
    static constexpr int NT = S * R * T, GI = N / R;
    static constexpr int OWN = (R * N + NT - 1) / NT;
    static_assert(NT % kWave == 0 && N % R == 0 && (R * N) % kWave == 0, "inverse tile");
    static_assert(R * N <= NT || (R * N) % NT == 0, "owned probe elements");
};

// The maxima travel between stages as per-wave partials: the forward row
// stage leaves kWinParts entries of max |S_j O|^2 per position (N / RB
// workgroups of RB N2 / 64 waves, whatever RB), the inverse row stage
// kProbeParts entries of max |P|^2 (N / R workgroups of R N / 64 owner
// waves, whatever R); both counts are the same in every launch form.
template <int N> constexpr int kWinParts = N * Fact<N>::N2 / kWave;
// The column stage leaves its error sum as per-wave partials too: kColParts
// entries per position (N / CB workgroups of CB N2 / 64 waves, whatever CB).
template <int N> constexpr int kColParts = N * Fact<N>::N2 / kWave;
template <int N> constexpr int kProbeParts = N * N / kWave;

// Stores of the bulk data that the next kernel reads on other XCDs (the
// spectrum exchange and the object window): written through this XCD's L2
// (an agent-scope relaxed store, i.e. a plain store with the agent
// coherence bit), so no dirty lines are left for the write-back at the end
// of the kernel.  The stored value is unchanged.
__device__ __forceinline__ void store_through(cf* p, cf v) {
    unsigned long long bits;
    __builtin_memcpy(&bits, &v, sizeof(bits));
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), bits, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Access to data that another workgroup of the same kernel writes.  In the
// per-batch kernels (COH = false) a kernel boundary separates producer and
// consumer, so plain loads are coherent; only the bulk stores are written
// through (above).  The persistent kernels (COH = true) have no kernel
// boundary between stages: every such load is a device-scope relaxed load
// (it misses the caches that may hold a stale line) and every such store a
// device-scope relaxed store (written through), so their barriers need no
// cache write-back or invalidation, only the wait for their own stores.
template <bool COH>
__device__ __forceinline__ cf ldc(const cf* p) {
    if constexpr (COH) {
        const unsigned long long b = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cf v;
        __builtin_memcpy(&v, &b, sizeof(v));
        return v;
    } else {
        return *p;
    }
}
template <bool COH>
__device__ __forceinline__ float ldc(const float* p) {
    if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool COH>
__device__ __forceinline__ double ldc(const double* p) {
    if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
// a store of a small result (probe, partial maxima, error partials)
template <bool COH>
__device__ __forceinline__ void stc(cf* p, cf v) {
    if constexpr (COH) store_through(p, v);
    else *p = v;
}
template <bool COH>
__device__ __forceinline__ void stc(float* p, float v) {
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool COH>
__device__ __forceinline__ void stc(double* p, double v) {
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// ---------------------------------------------------------------- stage 1
// psi = P * S_j O for rows rb*RB .. rb*RB+RB-1 of slot `slot`, 1D FFT of
// each row, spectrum rows to scratch; partial max |S_j O|^2 to winmax, one
// entry per wave (no workgroup barrier: a maximum is exact in any order).
template <int N, int RB, bool COH = false>
__device__ __forceinline__ void stage_rows_fwd(const BatchArgs& a, int slot, int rb, cf* lds) {
    using g = RowG<N, RB>;
    const int t = threadIdx.x % g::T, rl = threadIdx.x / g::T;
    cf w[g::N1];
    twiddles_a<N, -1>(w, t, a.tw);
    const OrderEntry e = a.order[a.off + slot];
    const int r = rb * RB + rl;
    const cf* orow = a.obj + (size_t)(e.row + r) * a.w + e.col;
    const cf* prow = a.probe + (size_t)r * N;
    cf v[g::N1];
    float m = 0.f;
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) {
        const int col = g::N2 * n1 + t;
        const cf o = ldc<COH>(&orow[col]);
        m = fmaxf(m, norm2(o));
        v[n1] = cmul(ldc<COH>(&prow[col]), o);
    }
    cf* z = lds + rl * Lds<N>::LINE;
    passA_to_lds<N, -1>(v, z, t, w);
    line_sync();   // row rl's threads are consecutive lanes of one wave
    passB_from_lds<N, -1, 1>(v, z, t);
    cf* srow = a.scratch + (size_t)slot * N * N + (size_t)r * N;
#pragma unroll
    for (int i = 0; i < g::N1; ++i) store_through(&srow[Fact<N>::out(t, i)], v[i]);
    m = wave_max(m);
    if (threadIdx.x % kWave == 0)
        stc<COH>(&a.winmax[slot * kWinParts<N> + rb * (g::NT / kWave) + threadIdx.x / kWave], m);
}

// ---------------------------------------------------------------- stage 2
// Columns cb*CB .. of slot `slot`: 1D FFT, Psi' = sqrt(I_j) sgn(Psi) with
// the error partial, inverse 1D FFT (unscaled), back to scratch.
template <int N, int CB, int MODE = kModeEpie, bool COH = false>
__device__ __forceinline__ void stage_cols(const BatchArgs& a, int slot, int cb, cf* lds) {
    using g = ColG<N, CB>;
    const int cl = threadIdx.x % CB, t = threadIdx.x / CB;
    // twiddles first: the first pass then waits for them and the spectrum
    // only, not for sqrt(I) (loads complete in issue order)
    cf wa[g::N1], wb[g::N1];
    twiddles_a<N, -1>(wa, t, a.tw);
    const int64_t j = a.order[a.off + slot].j;
    const int c = cb * CB + cl;
    cf* base = a.scratch + (size_t)slot * N * N + c;
    const float* ampb = a.sqrt_i + (size_t)j * N * N + amp_at(N, 0, c);   // row r at ampb[r * kAmpBlock]
    cf v[g::N1];
    float amp[g::N1];
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) v[n1] = ldc<COH>(&base[(size_t)(g::N2 * n1 + t) * N]);
    bool valid[g::N1];
#pragma unroll
    for (int i = 0; i < g::N1; ++i) {
        const int row = Fact<N>::out(t, i);
        amp[i] = ampb[(size_t)row * kAmpBlock];
        valid[i] = a.mask == nullptr || a.mask[row * N + c] != 0;
    }
    twiddles_binv<N, +1>(wb, t, a.tw);
    cf* z = lds + cl * Lds<N>::LINE;
    passA_to_lds<N, -1>(v, z, t, wa);
    __syncthreads();
    passB_from_lds<N, -1, CB>(v, z, t);
    float e = 0.f;
#pragma unroll
    for (int i = 0; i < g::N1; ++i) {
        const float s = amp[i];
        const cf zz = v[i];
        const float mag = sqrtf(norm2(zz));
        const float d = mag - s;
        if (!valid[i]) {
            // a masked detector pixel: no measurement, so the model's value
            // stays (ePIE) and it carries no loss (gradient)
            if (MODE == kModeGrad) v[i] = cf{0.f, 0.f};
            continue;
        }
        e += d * d;
        if (MODE == kModeEpie) {
            // Psi' = sqrt(I) sgn(Psi)
            const float f = mag > 0.f ? s / mag : 0.f;
            v[i] = f * zz;
        } else if (MODE == kModeGrad) {
            // dL/dPsi (PyTorch convention) = 2 (|Psi| - sqrt(I)) sgn(Psi), times the upstream scale
            const float f = mag > 0.f ? (2.f * a.gscale) * (d / mag) : 0.f;
            v[i] = f * zz;
        }
    }
    if (MODE != kModeLoss) {
        __syncthreads();
        passBinv_to_lds<N, +1, CB>(v, z, t, wb);
        __syncthreads();
        passAinv_from_lds<N, +1>(v, z, t);
#pragma unroll
        for (int n1 = 0; n1 < g::N1; ++n1) store_through(&base[(size_t)(g::N2 * n1 + t) * N], v[n1]);
    }
    // one partial per wave (no workgroup barrier at the end of the stage)
    static_assert((g::NT % kWave) == 0 && g::GC * (g::NT / kWave) == kColParts<N>, "error partials");
    const double tot = wave_sum((double)e);
    if (threadIdx.x % kWave == 0)
        stc<COH>(&a.err_part[(a.off + slot) * kColParts<N> + cb * (g::NT / kWave) + threadIdx.x / kWave], tot);
}

// ---------------------------------------------------------------- stage 3
// Probe rows rb*R .. rb*R+R-1, for every slot of the batch (S at a time):
// inverse 1D FFT of the slot's spectrum row, Delta = psi'/N^2 - P S_j O,
// object step alpha conj(P) Delta / max|P|^2, probe increment
// conj(S_j O) Delta / max|S_j O|^2 summed over slots in slot order, then
// P_{b+1} written for the block.  bsize == 0 only refreshes the block's
// max |P|^2.  lds: S R lines of Lds<N>::LINE (a line holds its slot row's
// transform, then that row's probe increments, which the slot sum reads),
// then the block's R probe rows (R N), read by every slot's threads instead
// of a register copy per slot, then the twiddle table (N) that the slots'
// inverse passes read (one load of it per workgroup instead of one set per
// thread).
template <int N, int R, int S, bool COH = false>
__device__ __forceinline__ void stage_rows_inv(const BatchArgs& a, int rb, cf* lds) {
    using g = InvG<N, R, S>;
    const int t = threadIdx.x % g::T;
    const int rl = (threadIdx.x / g::T) % g::R;
    const int sl = threadIdx.x / (g::T * g::R);
    const int r = rb * g::R + rl;
    // the elements this thread owns in the probe block: element
    // e = k NT + threadIdx.x of the block's R rows (if e < R N)
    constexpr int OWN = g::OWN;
    cf p_own[OWN], acc[OWN];
    cf* const pl = lds + g::S * g::R * Lds<N>::LINE;   // the block's probe rows
    cf* const twl = pl + g::R * N;                     // the twiddle table
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
        const int e = k * g::NT + (int)threadIdx.x;
        const size_t own = (size_t)rb * g::R * N + e;
        p_own[k] = e < g::R * N ? ldc<COH>(&a.probe[own]) : cf{0.f, 0.f};
        if (e < g::R * N) pl[e] = p_own[k];
        acc[k] = cf{0.f, 0.f};
    }
    for (int e = (int)threadIdx.x; e < N; e += g::NT) twl[e] = a.tw[e];
    if (a.bsize > 0) {
        __syncthreads();
        const cf* prl = pl + rl * N;
        // every wave reduces all partial maxima itself (no barrier)
        float pm = 0.f;
#pragma unroll
        for (int k = 0; k < (kProbeParts<N> + kWave - 1) / kWave; ++k) {
            const int i = k * kWave + (int)(threadIdx.x % kWave);
            if (i < kProbeParts<N>) pm = fmaxf(pm, ldc<COH>(&a.pmax_in[i]));
        }
        pm = wave_max(pm);
        const float ostep = a.alpha / pm;
        cf* z = lds + (sl * g::R + rl) * Lds<N>::LINE;
        for (int g0 = 0; g0 < a.bsize; g0 += g::S) {
            const int slot = g0 + sl;
            const bool act = slot < a.bsize;
            cf v[g::N1], o[g::N1];
            cf* orow = nullptr;
            float om = 1.f;
            if (act) {
                const OrderEntry e = a.order[a.off + slot];
                const cf* srow = a.scratch + (size_t)slot * N * N + (size_t)r * N;
                orow = a.obj + (size_t)(e.row + r) * a.w + e.col;
#pragma unroll
                for (int i = 0; i < g::N1; ++i) v[i] = ldc<COH>(&srow[Fact<N>::out(t, i)]);
#pragma unroll
                for (int n1 = 0; n1 < g::N1; ++n1) o[n1] = ldc<COH>(&orow[g::N2 * n1 + t]);
            } else {
#pragma unroll
                for (int n1 = 0; n1 < g::N1; ++n1) {
                    v[n1] = cf{0.f, 0.f};
                    o[n1] = cf{0.f, 0.f};
                }
            }
            // max |S_j O|^2 from the forward stage's per-wave partials,
            // loaded now and reduced by the slot's own threads after the
            // transform, so the transform does not wait for these loads
            // and the object row's (an idle slot reads slot 0's partials,
            // which exist, and discards the result)
            constexpr int GT = g::T * g::R;
            constexpr int kWm = (kWinParts<N> + GT - 1) / GT;
            float wpart[kWm];
            const int ws = act ? slot : 0;
#pragma unroll
            for (int k = 0; k < kWm; ++k) {
                const int i = k * GT + (int)(threadIdx.x % GT);
                wpart[k] = i < kWinParts<N> ? ldc<COH>(&a.winmax[ws * kWinParts<N> + i]) : 0.f;
            }
            {
                cf wb[g::N1];
                twiddles_binv<N, +1>(wb, t, twl);
                passBinv_to_lds<N, +1, 1>(v, z, t, wb);
            }
            line_sync();   // the line's threads are consecutive lanes of one wave
            passAinv_from_lds<N, +1>(v, z, t);
            float wm = 0.f;
#pragma unroll
            for (int k = 0; k < kWm; ++k) wm = fmaxf(wm, wpart[k]);
            wm = group_max<GT>(wm);
            if (act) om = wm;
            constexpr float inv = 1.0f / (float)(N * N);
            const float pstep = 1.f / om;
            line_sync();   // the increments overwrite what the line's lanes just read
            if (act) {
#pragma unroll
                for (int n1 = 0; n1 < g::N1; ++n1) {
                    const int col = g::N2 * n1 + t;
                    const cf pv = prl[col];
                    const cf delta = inv * v[n1] - cmul(pv, o[n1]);
                    store_through(&orow[col], axpy(ostep, cmulc(pv, delta), o[n1]));
                    z[col] = pstep * cmulc(o[n1], delta);
                }
            }
            __syncthreads();
            // slot order: this group's slots ascending, after the earlier groups
            const int nact = min(g::S, a.bsize - g0);
#pragma unroll
            for (int k = 0; k < OWN; ++k) {
                const int e = k * g::NT + (int)threadIdx.x;
                if (e >= g::R * N) continue;
                // the same sequential sum, with eight loads in flight at a time
                const cf* col = lds + (e / N) * Lds<N>::LINE + e % N;
                constexpr int kSlotStride = g::R * Lds<N>::LINE;
                int q = 0;
                for (; q + 8 <= nact; q += 8) {
                    cf tq[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) tq[u] = col[(q + u) * kSlotStride];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[k] = acc[k] + tq[u];
                }
                for (; q < nact; ++q) acc[k] = acc[k] + col[q * kSlotStride];
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
        const int e = k * g::NT + (int)threadIdx.x;
        const bool owner = e < g::R * N;
        const size_t own = (size_t)rb * g::R * N + e;
        cf pn = p_own[k];
        if (a.bsize > 0 && owner) {
            pn = axpy(a.beta / (float)a.bsize, acc[k], p_own[k]);
            stc<COH>(&a.probe[own], pn);
        }
        // one partial per 64 consecutive elements of the block, from the
        // wave that owns them (waves past R*N own none)
        const float m = wave_max(norm2(pn));
        if (threadIdx.x % kWave == 0 && owner) stc<COH>(&a.pmax_out[(rb * g::R * N + e) / kWave], m);
    }
}

// ---------------------------------------------------------------- per-batch launches
template <int N> constexpr int kRowNT = RowG<N, Tile<N>::RB>::NT;
template <int N> constexpr int kColNT = ColG<N, Tile<N>::CB>::NT;
template <int N> constexpr int kSweepNT = RowG<N, PTile<N>::B>::NT;

// A graph node does not know its batch's extent when it is built: it reads
// the offset and size from the device offsets array (uniform loads).
__device__ __forceinline__ BatchArgs resolved(const BatchArgs& a) {
    BatchArgs r = a;
    if (a.boffs) {
        r.off = a.boffs[a.batch];
        r.bsize = (int)(a.boffs[a.batch + 1] - r.off);
    }
    return r;
}

// DEV: the batch's extent comes from device memory (graph nodes; their grids
// cover the largest batch, so surplus workgroups return at once).  Without
// it the extent is an argument and every caller sizes the grid to the batch
// exactly, so the kernel starts its loads without the branch and the check.
template <int N, int RB = Tile<N>::RB, bool DEV = false>
__global__ __launch_bounds__((RowG<N, RB>::NT)) void k_rows_fwd(BatchArgs a) {
    using g = RowG<N, RB>;
    __shared__ cf lds[RB * Lds<N>::LINE];
    const BatchArgs b = DEV ? resolved(a) : a;
    const int slot = blockIdx.x / g::G;
    if (DEV && slot >= b.bsize) return;   // a grid sized for a larger batch (whole workgroup)
    stage_rows_fwd<N, RB>(b, slot, blockIdx.x % g::G, lds);
}

template <int N, int CB = Tile<N>::CB, bool DEV = false>
__global__ __launch_bounds__((ColG<N, CB>::NT)) void k_cols(BatchArgs a) {
    using g = ColG<N, CB>;
    __shared__ cf lds[CB * Lds<N>::LINE];
    const BatchArgs b = DEV ? resolved(a) : a;
    const int slot = blockIdx.x / g::GC;
    if (DEV && slot >= b.bsize) return;
    stage_cols<N, CB>(b, slot, blockIdx.x % g::GC, lds);
}

template <int N, int R = ITile<N>::R, int S = ITile<N>::S, bool DEV = false>
__global__ __launch_bounds__((InvG<N, R, S>::NT)) void k_rows_inv(BatchArgs a) {
    using g = InvG<N, R, S>;
    __shared__ cf lds[g::S * g::R * Lds<N>::LINE + g::R * N + N];
    stage_rows_inv<N, g::R, g::S>(DEV ? resolved(a) : a, blockIdx.x, lds);
}

// Several reconstructions at once: workgroup b belongs to descriptor i with
// start[i] <= b < start[i+1]; the descriptor is uniform, so it lives in
// scalar registers.
struct MultiArgs {
    const BatchArgs* tab;
    int count;
    int start[kMultiMax + 1];
};

__device__ inline int multi_find(const MultiArgs& m) {
    int i = 0;
    while (i + 1 < m.count && (int)blockIdx.x >= m.start[i + 1]) ++i;
    return i;
}

template <int N>
__global__ __launch_bounds__(kRowNT<N>) void k_rows_fwd_multi(MultiArgs m) {
    constexpr int RB = Tile<N>::RB;
    using g = RowG<N, RB>;
    __shared__ cf lds[RB * Lds<N>::LINE];
    const int i = multi_find(m);
    const BatchArgs a = m.tab[i];
    const int local = (int)blockIdx.x - m.start[i];
    stage_rows_fwd<N, RB>(a, local / g::G, local % g::G, lds);
}

template <int N>
__global__ __launch_bounds__(kColNT<N>) void k_cols_multi(MultiArgs m) {
    constexpr int CB = Tile<N>::CB;
    using g = ColG<N, CB>;
    __shared__ cf lds[CB * Lds<N>::LINE];
    const int i = multi_find(m);
    const BatchArgs a = m.tab[i];
    const int local = (int)blockIdx.x - m.start[i];
    stage_cols<N, CB>(a, local / g::GC, local % g::GC, lds);
}

template <int N>
__global__ __launch_bounds__((InvG<N>::NT)) void k_rows_inv_multi(MultiArgs m) {
    using g = InvG<N>;
    __shared__ cf lds[g::S * g::R * Lds<N>::LINE + g::R * N + N];
    const int i = (int)blockIdx.x / g::GI;
    const BatchArgs a = m.tab[i];
    stage_rows_inv<N, g::R, g::S>(a, (int)blockIdx.x % g::GI, lds);
}

// Mixed pattern sizes in one launch per stage.  Every size in {64, 128,
// 256} gets a tile with the same workgroup size (kMixFwdNT threads, one
// wave, in the forward row stage, kMixRowNT in the column stage, kMixInvNT
// in the inverse stage), so one kernel
// serves all of them; a workgroup finds its descriptor and branches (the
// descriptor is uniform) to the stage of that size.  The tiles change how
// rows, columns and slots are grouped into workgroups, not the arithmetic
// of any element, and the partial-maximum layouts do not depend on the
// tile: the results equal those of the per-size kernels.
constexpr int kMixRowNT = 256, kMixFwdNT = 64, kMixInvNT = 512;
// The inverse stage has a second tile with fewer slots (S2, R2 rows each)
// for scans whose batches are small (spiral scans: a handful of positions
// per batch), so fewer lanes transform idle slots; BatchArgs::itile selects
// it.
template <int N> struct MixTile;
// RF: rows per workgroup of the forward stage (one wave), RB: columns per
// workgroup of the column stage.
template <> struct MixTile<64>  { static constexpr int RF = 8, RB = 32, R = 4, S = 16, R2 = 8, S2 = 8; };
template <> struct MixTile<128> { static constexpr int RF = 4, RB = 16, R = 1, S = 32, R2 = 4, S2 = 8; };
template <> struct MixTile<256> { static constexpr int RF = 4, RB = 16, R = 1, S = 32, R2 = 4, S2 = 8; };
template <int N> constexpr int kMixRowLds = MixTile<N>::RB * Lds<N>::LINE;
template <int N> constexpr int kMixFwdLds = MixTile<N>::RF * Lds<N>::LINE;
template <int N> constexpr int kMixInvLds =
    MixTile<N>::S * MixTile<N>::R * Lds<N>::LINE + (MixTile<N>::R > MixTile<N>::R2 ? MixTile<N>::R : MixTile<N>::R2) * N + N;
constexpr int cmax3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }
constexpr int kMixRowLdsMax = cmax3(kMixRowLds<64>, kMixRowLds<128>, kMixRowLds<256>);
constexpr int kMixFwdLdsMax = cmax3(kMixFwdLds<64>, kMixFwdLds<128>, kMixFwdLds<256>);
constexpr int kMixInvLdsMax = cmax3(kMixInvLds<64>, kMixInvLds<128>, kMixInvLds<256>);

template <int N>
__device__ __forceinline__ void mix_rows_fwd(const BatchArgs& a, int local, cf* lds) {
    using g = RowG<N, MixTile<N>::RF>;
    static_assert(g::NT == kMixFwdNT, "mixed row tile");
    stage_rows_fwd<N, MixTile<N>::RF>(a, local / g::G, local % g::G, lds);
}

template <int N>
__device__ __forceinline__ void mix_cols(const BatchArgs& a, int local, cf* lds) {
    using g = ColG<N, MixTile<N>::RB>;
    static_assert(g::NT == kMixRowNT, "mixed column tile");
    stage_cols<N, MixTile<N>::RB>(a, local / g::GC, local % g::GC, lds);
}

template <int N>
__device__ __forceinline__ void mix_rows_inv(const BatchArgs& a, int local, cf* lds) {
    using g = InvG<N, MixTile<N>::R, MixTile<N>::S>;
    using g2 = InvG<N, MixTile<N>::R2, MixTile<N>::S2>;
    static_assert(g::NT == kMixInvNT && g2::NT == kMixInvNT, "mixed inverse tile");
    static_assert(g2::S * g2::R <= g::S * g::R, "the small-batch tile fits the LDS of the default one");
    if (a.itile)
        stage_rows_inv<N, g2::R, g2::S>(a, local, lds);
    else
        stage_rows_inv<N, g::R, g::S>(a, local, lds);
}

__global__ __launch_bounds__(kMixFwdNT) void k_rows_fwd_mix(MultiArgs m) {
    __shared__ cf lds[kMixFwdLdsMax];
    const int i = multi_find(m);
    const BatchArgs a = m.tab[i];
    const int local = (int)blockIdx.x - m.start[i];
    switch (a.n) {
        case 64: mix_rows_fwd<64>(a, local, lds); break;
        case 128: mix_rows_fwd<128>(a, local, lds); break;
        case 256: mix_rows_fwd<256>(a, local, lds); break;
    }
}

__global__ __launch_bounds__(kMixRowNT) void k_cols_mix(MultiArgs m) {
    __shared__ cf lds[kMixRowLdsMax];
    const int i = multi_find(m);
    const BatchArgs a = m.tab[i];
    const int local = (int)blockIdx.x - m.start[i];
    switch (a.n) {
        case 64: mix_cols<64>(a, local, lds); break;
        case 128: mix_cols<128>(a, local, lds); break;
        case 256: mix_cols<256>(a, local, lds); break;
    }
}

__global__ __launch_bounds__(kMixInvNT) void k_rows_inv_mix(MultiArgs m) {
    __shared__ cf lds[kMixInvLdsMax];
    const int i = multi_find(m);
    const BatchArgs a = m.tab[i];
    const int local = (int)blockIdx.x - m.start[i];
    switch (a.n) {
        case 64: mix_rows_inv<64>(a, local, lds); break;
        case 128: mix_rows_inv<128>(a, local, lds); break;
        case 256: mix_rows_inv<256>(a, local, lds); break;
    }
}

// Mean of K equally shaped complex arrays, written back to all of them
// (summed in list order, so the result does not depend on the launch).
struct MeanArgs {
    cf* ptr[kMultiMax];
    int k;
    int64_t count;
};

__global__ __launch_bounds__(256) void k_mean(MeanArgs m) {
    const float inv = 1.f / (float)m.k;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m.count; e += (int64_t)gridDim.x * 256) {
        cf acc = m.ptr[0][e];
        for (int i = 1; i < m.k; ++i) acc = acc + m.ptr[i][e];
        acc = inv * acc;
        for (int i = 0; i < m.k; ++i) m.ptr[i][e] = acc;
    }
}

// The column stage of the amplitude loss (kModeLoss: loss partials only) or
// of its gradient (kModeGrad: also g_Psi, transformed back along columns).
template <int N, int MODE>
__global__ __launch_bounds__(kColNT<N>) void k_cols_mode(BatchArgs a) {
    constexpr int CB = Tile<N>::CB;
    using g = ColG<N, CB>;
    __shared__ cf lds[CB * Lds<N>::LINE];
    stage_cols<N, CB, MODE>(a, blockIdx.x / g::GC, blockIdx.x % g::GC, lds);
}

// ---------------------------------------------------------------- amplitude-loss adjoint
// dL/dpsi of every position of a minibatch at once.  A workgroup takes AR
// rows of the slots of one group of kAdjGroup consecutive slots, kAdjLanes
// slots at a time (one 64-thread lane set per slot): the inverse row FFT of
// the column stage's output gives F^H g_Psi (unscaled, = dL/dpsi); the
// position's contribution conj(P) dL/dpsi to dL/dO on its window replaces
// the slot's spectrum rows (windows may overlap: the object tiles sum them
// afterwards), and conj(S_j O) dL/dpsi is added to the lane set's running
// dL/dP rows, which are combined in lane order at the end into the group's
// partial sum part[group] (summed over the groups in order afterwards).
template <int N> struct AdjG {
    static constexpr int T = Fact<N>::N2, AR = kWave / T;   // one wave per slot and row block
    using rg = RowG<N, AR>;
    static constexpr int G = rg::G, NT = kAdjLanes * kWave;
};

template <int N>
__global__ __launch_bounds__(kAdjLanes * kWave) void k_rows_adj(BatchArgs a, cf* part) {
    using ag = AdjG<N>;
    using g = typename ag::rg;
    constexpr int AR = ag::AR;
    __shared__ cf lds[kAdjLanes * AR * Lds<N>::LINE];
    static_assert(Lds<N>::LINE >= N, "the lines hold the lane sets' partial sums afterwards");
    cf* red = lds;   // after the loop: lane set k > 0's dL/dP rows at [(k - 1) AR + row] N
    const int grp = blockIdx.x / ag::G, rb = blockIdx.x % ag::G;
    const int t = threadIdx.x % g::T, rl = (threadIdx.x / g::T) % AR, ln = threadIdx.x / kWave;
    const int r = rb * AR + rl;
    cf wb[g::N1];
    twiddles_binv<N, +1>(wb, t, a.tw);
    const cf* prow = a.probe + (size_t)r * N;
    cf p[g::N1], acc[g::N1];
#pragma unroll
    for (int n1 = 0; n1 < g::N1; ++n1) {
        p[n1] = prow[g::N2 * n1 + t];
        acc[n1] = cf{0.f, 0.f};
    }
    cf* z = lds + (ln * AR + rl) * Lds<N>::LINE;
    const int s1 = min(a.bsize, (grp + 1) * kAdjGroup);
    for (int slot = grp * kAdjGroup + ln; slot < s1; slot += kAdjLanes) {
        cf* srow = a.scratch + (size_t)slot * N * N + (size_t)r * N;
        cf v[g::N1], o[g::N1];
#pragma unroll
        for (int i = 0; i < g::N1; ++i) v[i] = srow[Fact<N>::out(t, i)];
        const OrderEntry e = a.order[a.off + slot];
        const cf* orow = a.obj + (size_t)(e.row + r) * a.w + e.col;
#pragma unroll
        for (int n1 = 0; n1 < g::N1; ++n1) o[n1] = orow[g::N2 * n1 + t];
        passBinv_to_lds<N, +1, 1>(v, z, t, wb);
        line_sync();   // the line's threads are consecutive lanes of one wave
        passAinv_from_lds<N, +1>(v, z, t);
        // the row's spectrum was read by this wave before the transform, so
        // the contribution may replace it
#pragma unroll
        for (int n1 = 0; n1 < g::N1; ++n1) {
            const int col = g::N2 * n1 + t;
            srow[col] = cmulc(p[n1], v[n1]);
            acc[n1] = acc[n1] + cmulc(o[n1], v[n1]);
        }
        line_sync();   // the next slot's transform reuses the line
    }
    __syncthreads();   // every lane set is done with its lines
    if (ln > 0) {
#pragma unroll
        for (int n1 = 0; n1 < g::N1; ++n1) red[((ln - 1) * AR + rl) * N + g::N2 * n1 + t] = acc[n1];
    }
    __syncthreads();
    if (ln == 0) {
        cf* prt = part + (size_t)grp * N * N + (size_t)r * N;
#pragma unroll
        for (int n1 = 0; n1 < g::N1; ++n1) {
            const int col = g::N2 * n1 + t;
            cf sum = acc[n1];
#pragma unroll
            for (int k = 1; k < kAdjLanes; ++k) sum = sum + red[((k - 1) * AR + rl) * N + col];
            prt[col] = sum;
        }
    }
}

// dL/dP: the groups' partial sums added in group order, eight loads in
// flight at a time (block blk of 256 elements)
__device__ inline void probe_grad_sum(const cf* part, int64_t nn, int parts, cf* gprobe, int blk) {
    const int64_t el = (int64_t)blk * 256 + threadIdx.x;
    if (el >= nn) return;
    cf acc = cf{0.f, 0.f};
    int q = 0;
    for (; q + 8 <= parts; q += 8) {
        cf tq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) tq[u] = part[(size_t)(q + u) * nn + el];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = acc + tq[u];
    }
    for (; q < parts; ++q) acc = acc + part[(size_t)q * nn + el];
    gprobe[el] = acc;
}

// dL/dO by object tiles of kGradTR x kGradTC pixels, one workgroup per
// tile (tile tid): each pixel of the tile gets the sum of the contributions
// of the windows that cover it, over the slots listed for the tile
// (ascending), and every pixel is written (zero where no window reaches).
__device__ inline void obj_grad_gather(const cf* co_slot, const OrderEntry* order, int n, int64_t h, int64_t w,
                                       int tiles_x, const int* tile_off, const int* tile_slot, cf* gobj, int tid) {
    constexpr int kRowsPerPass = 256 / kGradTC, KR = kGradTR / kRowsPerPass, U = 8;
    const int64_t y0 = (int64_t)(tid / tiles_x) * kGradTR, x0 = (int64_t)(tid % tiles_x) * kGradTC;
    const int cx = (int)threadIdx.x % kGradTC, ry = (int)threadIdx.x / kGradTC;
    const int64_t x = x0 + cx;
    const int64_t nn = (int64_t)n * n;
    cf acc[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) acc[k] = cf{0.f, 0.f};
    const int q1 = tile_off[tid + 1];
    // U slots at a time, so their loads are in flight together; the sum
    // still runs over the slots in ascending order (a pixel outside a
    // window adds zero, which changes no sum)
    for (int q0 = tile_off[tid]; q0 < q1; q0 += U) {
        cf c[U][KR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool live = q0 + u < q1;
            const int s = live ? tile_slot[q0 + u] : 0;
            const OrderEntry e = order[s];
            const int64_t dx = x - e.col;
            const bool in_x = live && dx >= 0 && dx < n;
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int64_t dy = y0 + ry + (int64_t)k * kRowsPerPass - e.row;
                c[u][k] = in_x && dy >= 0 && dy < n ? co_slot[(size_t)s * nn + dy * n + dx] : cf{0.f, 0.f};
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < KR; ++k) acc[k] = acc[k] + c[u][k];
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int64_t y = y0 + ry + (int64_t)k * kRowsPerPass;
        if (y < h && x < w) gobj[y * w + x] = acc[k];
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(cf* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = cf{0.f, 0.f};
}

// ---------------------------------------------------------------- persistent sweeps
// A persistent kernel runs every batch of one or more sweeps of a scan with
// a fixed set of co-resident workgroups.  The stages of a batch are
// separated by barriers over the workgroups that serve that scan: a
// monotone arrival counter (zeroed before the launch) that each workgroup
// increments once its own device-coherent stores have completed, then
// polls until every workgroup of the scan has arrived.  All data the stages
// pass between workgroups goes through the coherent accesses (COH = true),
// so no cache write-back or invalidation is needed.  Every wait is bounded;
// on expiry (ScanArgs::spin_limit polls) the fault flag is raised and the
// waiting workgroups leave, so the grid always drains.

// Arrival is two-level: workgroup `local` of the gn that share the barrier
// adds one to the counter of its group of kBarGroup consecutive workgroups
// (bar[kBarLine (g + 1)], a memory line of its own); the group's last
// arrival adds one to the top counter bar[0], which every workgroup polls
// until it reaches `target` (the number of group completions so far).  So
// at most kBarGroup atomics, not gn, queue on any one address.
__device__ inline bool group_barrier(unsigned* bar, int local, int gn, unsigned target, unsigned spin_limit,
                                     int* fault, int* ok_sh) {
    // this wave's stores have completed (the coherent ones are written
    // through); the memory clobber keeps the compiler from moving memory
    // accesses across the wait
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const int g = local / kBarGroup;
        const unsigned gsize = (unsigned)min(kBarGroup, gn - g * kBarGroup);
        // the group counter counts every arrival of every barrier, so the
        // arrival that completes a multiple of gsize is the group's last
        // for this barrier (no workgroup passes a barrier before all have
        // arrived at it)
        const unsigned v =
            __hip_atomic_fetch_add(&bar[kBarLine * (g + 1)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((v + 1u) % gsize == 0u) __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        int ok = 1;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            // the bound on every poll, another workgroup's fault every 1024
            if (++spins >= spin_limit ||
                ((spins & 1023u) == 0u && __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        *ok_sh = ok;
    }
    __syncthreads();
    asm volatile("" ::: "memory");
    return *ok_sh != 0;
}

// Running Fourier error of one sweep from its error partials: the same
// summation order as k_err_reduce (256 threads, strided, then block_sum),
// so the value is the one the per-batch launches report.
__device__ inline void sweep_error(const double* err_part, int64_t n_part, const OrderEntry* order,
                                   int64_t order_len, const double* sum_i, double* out, double* red) {
    double num = 0.0, den = 0.0;
    for (int64_t i = threadIdx.x; i < n_part; i += 256) num += ldc<true>(&err_part[i]);
    for (int64_t i = threadIdx.x; i < order_len; i += 256) den += sum_i[order[i].j];
    num = block_sum<256>(num, red);
    den = block_sum<256>(den, red);
    if (threadIdx.x == 0) *out = den > 0.0 ? num / den : 0.0;
}

// The sweeps of one scan by workgroup `local` of the sc.gn that serve it:
// for every non-empty batch the forward row items, the column items and
// the inverse row items are dealt round-robin to the scan's workgroups,
// with a barrier after each stage; the probe maxima alternate halves after
// every non-empty batch.  ERR: the workgroup with local index 0 reduces
// each sweep's error after its last batch (256 threads).
template <int N, int RB, int CB, int IR, int IS, bool ERR>
__device__ void persist_scan(const ScanArgs& sc, int local, int* fault, cf* lds, double* red,
                             int* ok_sh) {
    using rg = RowG<N, RB>;
    using cg = ColG<N, CB>;
    using ig = InvG<N, IR, IS>;
    BatchArgs a = sc.a;
    unsigned target = 0;
    const unsigned groups = (unsigned)bar_groups(sc.gn);
    for (int sw = 0; sw < sc.n_sweeps; ++sw) {
        a.order = sc.a.order + (size_t)sw * sc.olen;
        const int64_t* offs = sc.offs + (size_t)sw * (sc.nb + 1);
        for (int b = 0; b < sc.nb; ++b) {
            const int64_t off = offs[b];
            const int bs = (int)(offs[b + 1] - off);
            if (bs <= 0) continue;
            a.off = off;
            a.bsize = bs;
            for (int it = local; it < bs * rg::G; it += sc.gn)
                stage_rows_fwd<N, RB, true>(a, it / rg::G, it % rg::G, lds);
            target += groups;
            if (!group_barrier(sc.bar, local, sc.gn, target, sc.spin_limit, fault, ok_sh)) return;
            for (int it = local; it < bs * cg::GC; it += sc.gn)
                stage_cols<N, CB, kModeEpie, true>(a, it / cg::GC, it % cg::GC, lds);
            target += groups;
            if (!group_barrier(sc.bar, local, sc.gn, target, sc.spin_limit, fault, ok_sh)) return;
            for (int it = local; it < ig::GI; it += sc.gn) stage_rows_inv<N, IR, IS, true>(a, it, lds);
            target += groups;
            if (!group_barrier(sc.bar, local, sc.gn, target, sc.spin_limit, fault, ok_sh)) return;
            // the maxima just written are those of the next batch's probe
            float* const next_in = a.pmax_out;
            a.pmax_out = const_cast<float*>(a.pmax_in);
            a.pmax_in = next_in;
        }
        if constexpr (ERR) {
            // the next sweep overwrites the partials only after its first
            // barrier, which this workgroup reaches after the reduction
            if (sc.err && local == 0) sweep_error(a.err_part, sc.olen * kColParts<N>, a.order, sc.olen, sc.sum_i,
                                                  sc.err + sw, red);
        }
    }
}

// One scan, every workgroup of the launch (the "persistent" launch form).
template <int N>
__global__ __launch_bounds__(kSweepNT<N>) void k_sweep(ScanArgs sc, int* fault) {
    constexpr int TB = PTile<N>::B;
    using rg = RowG<N, TB>;
    using cg = ColG<N, TB>;
    using ig = InvG<N, PTile<N>::R, PTile<N>::S>;
    static_assert(rg::NT == cg::NT && rg::NT == ig::NT, "one workgroup size for every stage");
    constexpr int NT = rg::NT;
    constexpr int LINES = TB > ig::S * ig::R + ig::R + 1 ? TB : ig::S * ig::R + ig::R + 1;
    __shared__ cf lds[LINES * Lds<N>::LINE];
    __shared__ double redd[NT / kWave];
    __shared__ int ok_sh;
    sc.gn = (int)gridDim.x;
    persist_scan<N, TB, TB, ig::R, ig::S, false>(sc, (int)blockIdx.x, fault, lds, redd, &ok_sh);
}

// Several independent scans in one launch (pattern sizes 64, 128, 256):
// workgroups sc.g0 .. sc.g0 + sc.gn - 1 serve scan sc, each scan advancing
// through its own batches at its own pace (its barriers count only its own
// workgroups).  One workgroup size (kMP threads) for every size and stage;
// the tiles group rows, columns and slots differently from the per-batch
// kernels but compute every element the same way, so each scan's object
// and probe equal those of its own per-batch sweeps bit for bit.
constexpr int kMP = 256;
template <int N> struct MPTile;
template <> struct MPTile<64>  { static constexpr int RB = 32, CB = 32, R0 = 4, S0 = 8, R1 = 2, S1 = 16; };
template <> struct MPTile<128> { static constexpr int RB = 16, CB = 16, R0 = 1, S0 = 16, R1 = 2, S1 = 8; };
template <> struct MPTile<256> { static constexpr int RB = 16, CB = 16, R0 = 1, S0 = 16, R1 = 1, S1 = 16; };
template <int N> constexpr int kMPLines =
    cmax3(MPTile<N>::RB, MPTile<N>::S0 * MPTile<N>::R0 + MPTile<N>::R0 + 1, MPTile<N>::S1 * MPTile<N>::R1 + MPTile<N>::R1 + 1) *
    Lds<N>::LINE;
constexpr int kMPLds = cmax3(kMPLines<64>, kMPLines<128>, kMPLines<256>);

template <int N>
__device__ __forceinline__ void multi_scan(const ScanArgs& sc, int local, int* fault, cf* lds, double* red,
                                           int* ok_sh) {
    using t = MPTile<N>;
    static_assert(RowG<N, t::RB>::NT == kMP && ColG<N, t::CB>::NT == kMP, "multi-scan row and column tiles");
    static_assert(InvG<N, t::R0, t::S0>::NT == kMP && InvG<N, t::R1, t::S1>::NT == kMP, "multi-scan inverse tiles");
    if (sc.inv_tile == 0)
        persist_scan<N, t::RB, t::CB, t::R0, t::S0, true>(sc, local, fault, lds, red, ok_sh);
    else
        persist_scan<N, t::RB, t::CB, t::R1, t::S1, true>(sc, local, fault, lds, red, ok_sh);
}

__global__ __launch_bounds__(kMP) void k_multi_persist(const ScanArgs* scans, int count, int* fault) {
    __shared__ cf lds[kMPLds];
    __shared__ double red[kMP / kWave];
    __shared__ int ok_sh;
    int i = 0;
    while (i + 1 < count && (int)blockIdx.x >= scans[i + 1].g0) ++i;
    const ScanArgs sc = scans[i];
    const int local = (int)blockIdx.x - sc.g0;
    if (local < 0 || local >= sc.gn) return;
    switch (sc.a.n) {
        case 64: multi_scan<64>(sc, local, fault, lds, red, &ok_sh); break;
        case 128: multi_scan<128>(sc, local, fault, lds, red, &ok_sh); break;
        case 256: multi_scan<256>(sc, local, fault, lds, red, &ok_sh); break;
    }
}

// ---------------------------------------------------------------- sequential sweep
// Strict (sequential) ePIE in one workgroup: the probe lives in LDS for the
// whole sweep and is updated after every position, the N x N spectrum of
// the current position stays in LDS between its row and column passes,
// and the workgroup walks the order one position after another.  N x N2
// threads: thread group l of N2 threads transforms row l in the row passes
// and column l in the column pass, with the same passes, twiddles and
// update expressions as the per-batch kernels, so a sweep gives the bytes
// of the batch form with batches of one.  OL: the whole object is held in
// LDS for the sweep (copied in at the start, out at the end) when it fits
// beside the rest (kStrictObj<N> complex values), so a position's window
// never waits for device memory; the next position's sqrt(I) is loaded
// while the current one is transformed.
template <int N> constexpr int kStrictNT = N * Fact<N>::N2;
template <int N> constexpr int kStrictTP = N + 1;
template <int N> constexpr int kStrictNW = kStrictNT<N> / kWave > 0 ? kStrictNT<N> / kWave : 1;
// LDS of the kernel without the object, and what is left of the 160 KiB for it
template <int N> constexpr int kStrictLdsBase =
    (int)sizeof(cf) * (N * N + N * kStrictTP<N> + N * Lds<N>::LINE) + kStrictNW<N> * (2 * 4 + 8) + 64;
template <int N> constexpr int kStrictObj = (160 * 1024 - kStrictLdsBase<N>) / (int)sizeof(cf);

template <int N, bool OL>
__global__ __launch_bounds__(kStrictNT<N>) void k_strict(BatchArgs a, int count) {
    using F = Fact<N>;
    constexpr int N1 = F::N1, N2 = F::N2, NT = kStrictNT<N>, TP = kStrictTP<N>, NW = kStrictNW<N>;
    static_assert(kWave % N2 == 0, "a transform line lies within one wave");
    __shared__ cf P[N * N];
    __shared__ cf tile[N * TP];
    __shared__ cf line[N * Lds<N>::LINE];
    __shared__ float part[2][NW];
    __shared__ double dsum[NW];
    __shared__ cf objl[OL ? kStrictObj<N> : 1];
    const int t = threadIdx.x % N2, l = threadIdx.x / N2;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    cf* z = line + l * Lds<N>::LINE;
    cf wa[N1], wb[N1];
    twiddles_a<N, -1>(wa, t, a.tw);
    twiddles_binv<N, +1>(wb, t, a.tw);
    const int64_t hw = a.h * a.w;
    if constexpr (OL) {
        for (int64_t e = threadIdx.x; e < hw; e += NT) objl[e] = a.obj[e];
    }
    cf* const obase = OL ? objl : a.obj;
    // block maximum of per-thread values (uniform result); slot k of part
    auto block_max = [&](float m, int k) {
        m = wave_max(m);
        if (lane == 0) part[k][wid] = m;
        __syncthreads();
        float r = part[k][0];
#pragma unroll
        for (int i = 1; i < NW; ++i) r = fmaxf(r, part[k][i]);
        return r;
    };
    // the probe row elements this thread owns in the row passes
    float pm0 = 0.f;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        const int e = l * N + N2 * n1 + t;
        const cf p = a.probe[e];
        P[e] = p;
        pm0 = fmaxf(pm0, norm2(p));
    }
    float pm = block_max(pm0, 0);
    constexpr float inv = 1.0f / (float)(N * N);
    // sqrt(I) of column l of a position, in the order the column pass holds it
    auto load_amp = [&](int64_t j, float* amp) {
        const float* ampb = a.sqrt_i + (size_t)j * N * N + amp_at(N, 0, l);
#pragma unroll
        for (int i = 0; i < N1; ++i) amp[i] = ampb[(size_t)F::out(t, i) * kAmpBlock];
    };
    float amp[N1];
    OrderEntry e = a.order[a.off];
    load_amp(e.j, amp);
    for (int k = 0; k < count; ++k) {
        cf* orow = obase + (size_t)(e.row + l) * a.w + e.col;
        cf o[N1], v[N1], p[N1];
        float m = 0.f;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const int col = N2 * n1 + t;
            o[n1] = orow[col];
            p[n1] = P[l * N + col];
            m = fmaxf(m, norm2(o[n1]));
            v[n1] = cmul(p[n1], o[n1]);
        }
        // the next position's sqrt(I), in flight during this one (issued
        // after the object rows, whose wait therefore does not include it)
        const OrderEntry en = a.order[a.off + (k + 1 < count ? k + 1 : k)];
        float amp_next[N1];
        load_amp(en.j, amp_next);
        bool valid[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) valid[i] = a.mask == nullptr || a.mask[F::out(t, i) * N + l] != 0;
        // row pass (forward): spectrum row l into the tile
        passA_to_lds<N, -1>(v, z, t, wa);
        line_sync();
        passB_from_lds<N, -1, 1>(v, z, t);
#pragma unroll
        for (int i = 0; i < N1; ++i) tile[l * TP + F::out(t, i)] = v[i];
        const float om = block_max(m, 1);   // its barrier also orders the tile writes
        // column pass: column l, modulus replacement, inverse
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) v[n1] = tile[(N2 * n1 + t) * TP + l];
        passA_to_lds<N, -1>(v, z, t, wa);
        line_sync();
        passB_from_lds<N, -1, 1>(v, z, t);
        float err = 0.f;
#pragma unroll
        for (int i = 0; i < N1; ++i) {
            const cf zz = v[i];
            const float mag = sqrtf(norm2(zz));
            const float d = mag - amp[i];
            if (!valid[i]) continue;
            err += d * d;
            const float f = mag > 0.f ? amp[i] / mag : 0.f;
            v[i] = f * zz;
        }
        line_sync();
        passBinv_to_lds<N, +1, 1>(v, z, t, wb);
        line_sync();
        passAinv_from_lds<N, +1>(v, z, t);
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) tile[(N2 * n1 + t) * TP + l] = v[n1];
        // error of this position (its own slot of the partials)
        const double es = wave_sum((double)err);
        if (lane == 0) dsum[wid] = es;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
#pragma unroll
            for (int i = 0; i < NW; ++i) tot += dsum[i];
            a.err_part[a.off + k] = tot;
        }
        // inverse row pass: row l, then the object and probe steps
#pragma unroll
        for (int i = 0; i < N1; ++i) v[i] = tile[l * TP + F::out(t, i)];
        passBinv_to_lds<N, +1, 1>(v, z, t, wb);
        line_sync();
        passAinv_from_lds<N, +1>(v, z, t);
        const float ostep = a.alpha / pm;
        const float pstep = 1.f / om;
        float m2 = 0.f;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const int col = N2 * n1 + t;
            const cf delta = inv * v[n1] - cmul(p[n1], o[n1]);
            orow[col] = axpy(ostep, cmulc(p[n1], delta), o[n1]);
            // a batch of one: the increment sum starts from zero
            const cf acc = cf{0.f, 0.f} + pstep * cmulc(o[n1], delta);
            const cf pn = axpy(a.beta, acc, p[n1]);
            P[l * N + col] = pn;
            m2 = fmaxf(m2, norm2(pn));
        }
        // the next position reads rows of the object this one wrote (this
        // workgroup's own stores, visible to it after the barrier)
        pm = block_max(m2, 0);
        e = en;
#pragma unroll
        for (int i = 0; i < N1; ++i) amp[i] = amp_next[i];
    }
    if constexpr (OL) {
        __syncthreads();
        for (int64_t q = threadIdx.x; q < hw; q += NT) a.obj[q] = objl[q];
    }
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
        const int q = l * N + N2 * n1 + t;
        a.probe[q] = P[q];
    }
}

__global__ __launch_bounds__(256) void k_zero_u32(unsigned* p, int n) {
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- ingest
template <int N>
__global__ __launch_bounds__(256) void k_ingest(const float* __restrict__ src, float* dst, double* sum_i,
                                                IngestSpec sp, int* bad) {
    __shared__ double red[256 / kWave];
    const size_t i = blockIdx.x;
    const float* f = src + i * (size_t)sp.frame_h * sp.frame_w;
    float* d = dst + i * N * N;
    const float rs = sqrtf(sp.scale);
    double acc = 0.0;
    int badl = 0;
    for (int e = threadIdx.x; e < N * N; e += 256) {
        const int r = e / N, c = e % N;   // pixel of the N x N crop
        const float x = f[(size_t)(sp.crop_y + r) * sp.frame_w + sp.crop_x + c];
        // orientation (transpose, then row flip, then column flip), then the
        // optional move of DC from (N/2, N/2) to (0, 0)
        int a = r, b = c;
        if (sp.orient & 1) { const int t = a; a = b; b = t; }
        if (sp.orient & 2) a = N - 1 - a;
        if (sp.orient & 4) b = N - 1 - b;
        if (sp.centred) {
            a = (a + N / 2) % N;
            b = (b + N / 2) % N;
        }
        const bool valid = sp.mask == nullptr || sp.mask[a * N + b] != 0;
        float amp = 0.f;
        if (valid) {
            if (!(x >= 0.f) || !isfinite(x)) badl = 1;
            if (sp.is_sqrt) {
                amp = x * rs;
                acc += (double)amp * (double)amp;
            } else {
                const float v = sp.scale * x;
                amp = sqrtf(v);
                acc += (double)v;
            }
        }
        d[amp_at(N, a, b)] = amp;
    }
    if (badl) atomicOr(bad, 1);
    const double tot = block_sum<256>(acc, red);
    if (threadIdx.x == 0) sum_i[i] = tot;
}

// stored amplitudes of position blockIdx.x back to row-major order
template <int N>
__global__ __launch_bounds__(256) void k_amp_rowmajor(const float* __restrict__ src, float* dst) {
    const float* a = src + (size_t)blockIdx.x * N * N;
    float* d = dst + (size_t)blockIdx.x * N * N;
    for (int e = threadIdx.x; e < N * N; e += 256) d[e] = a[amp_at(N, e / N, e % N)];
}

// ---------------------------------------------------------------- error
__device__ inline void err_reduce(const double* err_part, int64_t n_part, const OrderEntry* order, int64_t order_len,
                                  const double* sum_i, double* out, int raw, double* red) {
    double num = 0.0, den = 0.0;
    // each thread's strided sum in index order, eight loads in flight
    int64_t i = threadIdx.x;
    for (; i + 7 * 256 < n_part; i += 8 * 256) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = err_part[i + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) num += t[u];
    }
    for (; i < n_part; i += 256) num += err_part[i];
    for (int64_t k = threadIdx.x; k < order_len; k += 256) den += sum_i[order[k].j];
    num = block_sum<256>(num, red);
    den = block_sum<256>(den, red);
    if (threadIdx.x == 0) *out = raw ? num : (den > 0.0 ? num / den : 0.0);
}

__global__ __launch_bounds__(256) void k_err_reduce(const double* err_part, int64_t n_part,
                                                    const OrderEntry* order, int64_t order_len,
                                                    const double* sum_i, double* out, int raw) {
    __shared__ double red[256 / kWave];
    err_reduce(err_part, n_part, order, order_len, sum_i, out, raw, red);
}

// The last launch of a loss with gradient, three independent parts by
// workgroup range: the dL/dO tiles, then the dL/dP element blocks, then one
// workgroup summing the loss partials.
__global__ __launch_bounds__(256) void k_grad_finish(GradFinish f) {
    __shared__ double red[256 / kWave];
    const int b = (int)blockIdx.x;
    if (b < f.n_tiles) {
        obj_grad_gather(f.co, f.order, f.n, f.h, f.w, f.tiles_x, f.tile_off, f.tile_slot, f.gobj, b);
    } else if (b < f.n_tiles + f.probe_blocks) {
        probe_grad_sum(f.part, f.nn, f.parts, f.gprobe, b - f.n_tiles);
    } else {
        err_reduce(f.loss_part, f.n_loss_part, nullptr, 0, nullptr, f.loss, 1, red);
    }
}

// ---------------------------------------------------------------- host side
constexpr int mix_tile_rf(int n) {
    return n == 64 ? MixTile<64>::RF : n == 128 ? MixTile<128>::RF : n == 256 ? MixTile<256>::RF : 0;
}
constexpr int mix_tile_rb(int n) {
    return n == 64 ? MixTile<64>::RB : n == 128 ? MixTile<128>::RB : n == 256 ? MixTile<256>::RB : 0;
}
constexpr int mix_tile_r(int n, int itile) {
    if (itile) return n == 64 ? MixTile<64>::R2 : n == 128 ? MixTile<128>::R2 : n == 256 ? MixTile<256>::R2 : 0;
    return n == 64 ? MixTile<64>::R : n == 128 ? MixTile<128>::R : n == 256 ? MixTile<256>::R : 0;
}
template <int N>
Shape shape_n(int form, int variant) {
    if (form == kFormPersistent) return Shape{kWinParts<N>, kColParts<N>, kProbeParts<N>};
    if constexpr (N >= 64) {
        if (form == kFormMixed) return Shape{kWinParts<N>, kColParts<N>, kProbeParts<N>};
    }
    if (variant < 0 || variant >= Variants<N>::K) variant = 0;
    return Shape{kWinParts<N>, kColParts<N>, kProbeParts<N>};
}

template <int N, int V = 0>
hipError_t batch_n(const BatchArgs& a, hipStream_t s, hipEvent_t* ev) {
    constexpr TileV tv = Variants<N>::v[V];
    using rg = RowG<N, tv.rb>;
    using cg = ColG<N, tv.cb>;
    using ig = InvG<N, tv.r, tv.s>;
    constexpr auto kr = k_rows_fwd<N, tv.rb>;
    constexpr auto kc = k_cols<N, tv.cb>;
    constexpr auto ki = k_rows_inv<N, tv.r, tv.s>;
    if (ev) {
        // ev[2k], ev[2k+1]: the start and end of kernel k, taken from its
        // own dispatch (not from markers between launches)
        if (a.bsize > 0) {
            hipExtLaunchKernelGGL(kr, dim3(rg::G * a.bsize), dim3(rg::NT), 0, s, ev[0], ev[1], 0, a);
            hipExtLaunchKernelGGL(kc, dim3(cg::GC * a.bsize), dim3(cg::NT), 0, s, ev[2], ev[3], 0, a);
        }
        hipExtLaunchKernelGGL(ki, dim3(ig::GI), dim3(ig::NT), 0, s, ev[4], ev[5], 0, a);
        return hipGetLastError();
    }
    if (a.bsize > 0) {
        hipLaunchKernelGGL(kr, dim3(rg::G * a.bsize), dim3(rg::NT), 0, s, a);
        hipLaunchKernelGGL(kc, dim3(cg::GC * a.bsize), dim3(cg::NT), 0, s, a);
    }
    hipLaunchKernelGGL(ki, dim3(ig::GI), dim3(ig::NT), 0, s, a);
    return hipGetLastError();
}

template <int N, int V = 0>
hipError_t batch_v(int variant, const BatchArgs& a, hipStream_t s, hipEvent_t* ev) {
    if constexpr (V < Variants<N>::K) {
        if (variant == V) return batch_n<N, V>(a, s, ev);
        return batch_v<N, V + 1>(variant, a, s, ev);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int N, int V = 0>
hipError_t graph_n(const BatchArgs& a, int nb, int max_b, hipGraph_t* out) {
    constexpr TileV tv = Variants<N>::v[V];
    using rg = RowG<N, tv.rb>;
    using cg = ColG<N, tv.cb>;
    using ig = InvG<N, tv.r, tv.s>;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t prev = nullptr;
    auto add = [&](const void* fn, int grid, int nt, BatchArgs* args) {
        void* params[] = {args};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(fn);
        kp.gridDim = dim3(grid);
        kp.blockDim = dim3(nt);
        kp.sharedMemBytes = 0;
        kp.kernelParams = params;
        kp.extra = nullptr;
        hipGraphNode_t node = nullptr;
        hipError_t r = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (r == hipSuccess) prev = node;
        return r;
    };
    for (int b = 0; b < nb && e == hipSuccess; ++b) {
        BatchArgs ab = a;
        ab.batch = b;
        if (b & 1) {   // every node's inverse stage writes the other half (an empty batch refreshes it)
            ab.pmax_in = a.pmax_out;
            ab.pmax_out = const_cast<float*>(a.pmax_in);
        }
        ab.off = 0;
        ab.bsize = 0;
        e = add(reinterpret_cast<const void*>(&k_rows_fwd<N, tv.rb, true>), rg::G * max_b, rg::NT, &ab);
        if (e == hipSuccess)
            e = add(reinterpret_cast<const void*>(&k_cols<N, tv.cb, true>), cg::GC * max_b, cg::NT, &ab);
        if (e == hipSuccess)
            e = add(reinterpret_cast<const void*>(&k_rows_inv<N, tv.r, tv.s, true>), ig::GI, ig::NT, &ab);
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    *out = g;
    return hipSuccess;
}

template <int N, int V = 0>
hipError_t graph_v(int variant, const BatchArgs& a, int nb, int max_b, hipGraph_t* out) {
    if constexpr (V < Variants<N>::K) {
        if (variant == V) return graph_n<N, V>(a, nb, max_b, out);
        return graph_v<N, V + 1>(variant, a, nb, max_b, out);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t batch_multi_n(const BatchArgs* dev_tab, const BatchArgs* host_tab, int count, hipStream_t s) {
    using rg = RowG<N, Tile<N>::RB>;
    using cg = ColG<N, Tile<N>::CB>;
    if (count <= 0 || count > kMultiMax) return hipErrorInvalidValue;
    MultiArgs mr{dev_tab, count, {}}, mc{dev_tab, count, {}};
    mr.start[0] = mc.start[0] = 0;
    for (int i = 0; i < count; ++i) {
        mr.start[i + 1] = mr.start[i] + rg::G * host_tab[i].bsize;
        mc.start[i + 1] = mc.start[i] + cg::GC * host_tab[i].bsize;
    }
    if (mr.start[count] > 0) {
        hipLaunchKernelGGL(k_rows_fwd_multi<N>, dim3(mr.start[count]), dim3(rg::NT), 0, s, mr);
        hipLaunchKernelGGL(k_cols_multi<N>, dim3(mc.start[count]), dim3(cg::NT), 0, s, mc);
    }
    hipLaunchKernelGGL(k_rows_inv_multi<N>, dim3(InvG<N>::GI * count), dim3(InvG<N>::NT), 0, s, mr);
    return hipGetLastError();
}

// refresh the partial maxima of |P|^2 in the layout of `form`
template <int N>
hipError_t probe_n(const BatchArgs& a, int form, hipStream_t s) {
    BatchArgs z = a;
    z.bsize = 0;
    if (form == kFormPersistent) {
        constexpr int R = PTile<N>::R, S = PTile<N>::S;
        using g = InvG<N, R, S>;
        k_rows_inv<N, R, S><<<dim3(g::GI), dim3(g::NT), 0, s>>>(z);
    } else {
        hipLaunchKernelGGL(k_rows_inv<N>, dim3(InvG<N>::GI), dim3(InvG<N>::NT), 0, s, z);
    }
    return hipGetLastError();
}

// The forward stages of the amplitude loss over a.bsize positions at once
// (windows may overlap: nothing is written to the object): exit wave and
// row FFTs, then the column stage computing the loss partials and, with
// grad, g_Psi transformed back to the rows of dL/dpsi in the exchange.
template <int N>
hipError_t loss_fwd_n(const BatchArgs& a, bool grad, hipStream_t s) {
    using rg = RowG<N, Tile<N>::RB>;
    using cg = ColG<N, Tile<N>::CB>;
    if (a.bsize <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows_fwd<N>, dim3(rg::G * a.bsize), dim3(rg::NT), 0, s, a);
    if (grad)
        hipLaunchKernelGGL((k_cols_mode<N, kModeGrad>), dim3(cg::GC * a.bsize), dim3(cg::NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_cols_mode<N, kModeLoss>), dim3(cg::GC * a.bsize), dim3(cg::NT), 0, s, a);
    return hipGetLastError();
}

template <int N>
hipError_t adjoint_rows_n(const BatchArgs& a, cf* part, hipStream_t s) {
    if (a.bsize <= 0) return hipSuccess;
    const int groups = (a.bsize + kAdjGroup - 1) / kAdjGroup;
    hipLaunchKernelGGL(k_rows_adj<N>, dim3(AdjG<N>::G * groups), dim3(AdjG<N>::NT), 0, s, a, part);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_scale_c64(cf* p, int64_t n, const double* scale) {
    const float f = (float)*scale;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = f * p[i];
}

template <int N>
int persistent_capacity_n() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_sweep<N>),
                                                     kSweepNT<N>, 0) != hipSuccess)
        return 0;
    return per * cus;
}

template <int N>
hipError_t sweep_n(const ScanArgs& sc, int max_batch, int capacity, int* fault, hipStream_t s) {
    constexpr int TB = PTile<N>::B;
    const int need = std::max(max_batch * (N / TB), InvG<N, PTile<N>::R, PTile<N>::S>::GI);
    const int grid = std::min(need, capacity);
    // the top counter (the fault flag beside it stays) and the group counters
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, s, sc.bar, 1);
    const int gw = bar_words(grid) - kBarLine;
    hipLaunchKernelGGL(k_zero_u32, dim3((gw + 255) / 256), dim3(256), 0, s, sc.bar + kBarLine, gw);
    ScanArgs aa = sc;
    aa.g0 = 0;
    aa.gn = grid;
    void* args[] = {&aa, &fault};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sweep<N>), dim3(grid), dim3(kSweepNT<N>),
                                      args, 0, s);
}

template <int N>
hipError_t ingest_n(const float* src, float* dst, double* sum_i, int64_t count, const IngestSpec& sp, int* bad,
                    hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ingest<N>, dim3((unsigned)count), dim3(256), 0, s, src, dst, sum_i, sp, bad);
    return hipGetLastError();
}

}  // namespace

#define PTYC_DISPATCH(n, call)                             \
    switch (n) {                                           \
        case 16: { constexpr int N = 16; return call; }   \
        case 32: { constexpr int N = 32; return call; }   \
        case 64: { constexpr int N = 64; return call; }   \
        case 128: { constexpr int N = 128; return call; } \
        case 256: { constexpr int N = 256; return call; } \
    }

bool supported_n(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256; }

Shape shape_for(int n, int form, int variant) {
    PTYC_DISPATCH(n, shape_n<N>(form, variant));
    return Shape{0, 0, 0};
}

int tile_variants(int n) {
    PTYC_DISPATCH(n, Variants<N>::K);
    return 0;
}

hipError_t launch_batch(int n, int variant, const BatchArgs& a, hipStream_t s, hipEvent_t* ev) {
    PTYC_DISPATCH(n, batch_v<N>(variant, a, s, ev));
    return hipErrorInvalidValue;
}

hipError_t launch_probe_reduce(int n, const BatchArgs& a, int form, hipStream_t s) {
    PTYC_DISPATCH(n, probe_n<N>(a, form, s));
    return hipErrorInvalidValue;
}

hipError_t launch_batch_multi(int n, const BatchArgs* dev_tab, const BatchArgs* host_tab, int count,
                              hipStream_t s) {
    PTYC_DISPATCH(n, batch_multi_n<N>(dev_tab, host_tab, count, s));
    return hipErrorInvalidValue;
}

bool mixed_n(int n) { return n == 64 || n == 128 || n == 256; }

hipError_t launch_batch_mixed(const BatchArgs* dev_tab, const BatchArgs* host_tab, int count, hipStream_t s) {
    if (count <= 0 || count > kMultiMax) return hipErrorInvalidValue;
    MultiArgs mf{dev_tab, count, {}}, mr{dev_tab, count, {}}, mi{dev_tab, count, {}};
    mf.start[0] = mr.start[0] = mi.start[0] = 0;
    for (int i = 0; i < count; ++i) {
        const int n = host_tab[i].n;
        if (!mixed_n(n) || host_tab[i].bsize < 0) return hipErrorInvalidValue;
        mf.start[i + 1] = mf.start[i] + n / mix_tile_rf(n) * host_tab[i].bsize;
        mr.start[i + 1] = mr.start[i] + n / mix_tile_rb(n) * host_tab[i].bsize;
        mi.start[i + 1] = mi.start[i] + n / mix_tile_r(n, host_tab[i].itile);
    }
    if (mr.start[count] > 0) {
        hipLaunchKernelGGL(k_rows_fwd_mix, dim3(mf.start[count]), dim3(kMixFwdNT), 0, s, mf);
        hipLaunchKernelGGL(k_cols_mix, dim3(mr.start[count]), dim3(kMixRowNT), 0, s, mr);
    }
    hipLaunchKernelGGL(k_rows_inv_mix, dim3(mi.start[count]), dim3(kMixInvNT), 0, s, mi);
    return hipGetLastError();
}

hipError_t launch_mean(void* const* ptrs, int k, int64_t count_c64, hipStream_t s) {
    if (k <= 0 || k > kMultiMax || count_c64 <= 0) return hipErrorInvalidValue;
    MeanArgs m{};
    for (int i = 0; i < k; ++i) m.ptr[i] = (cf*)ptrs[i];
    m.k = k;
    m.count = count_c64;
    const int64_t blocks = std::min<int64_t>((count_c64 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_mean, dim3((unsigned)blocks), dim3(256), 0, s, m);
    return hipGetLastError();
}

int persistent_capacity(int n) {
    PTYC_DISPATCH(n, persistent_capacity_n<N>());
    return 0;
}

template <int N>
hipError_t strict_n(const BatchArgs& a, int count, hipStream_t s) {
    if constexpr (N <= kStrictMaxN) {
        if (a.h * a.w <= kStrictObj<N>)
            hipLaunchKernelGGL((k_strict<N, true>), dim3(1), dim3(kStrictNT<N>), 0, s, a, count);
        else
            hipLaunchKernelGGL((k_strict<N, false>), dim3(1), dim3(kStrictNT<N>), 0, s, a, count);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_strict(int n, const BatchArgs& a, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    PTYC_DISPATCH(n, strict_n<N>(a, count, s));
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(int n, const ScanArgs& sc, int max_batch, int capacity, int* fault, hipStream_t s) {
    PTYC_DISPATCH(n, sweep_n<N>(sc, max_batch, capacity, fault, s));
    return hipErrorInvalidValue;
}

int multi_capacity() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_multi_persist), kMP, 0) !=
        hipSuccess)
        return 0;
    return per * cus;
}

template <int N>
int multi_need_n(int max_batch, int inv_tile) {
    using t = MPTile<N>;
    const int r = inv_tile ? t::R1 : t::R0;
    return std::max(std::max(max_batch * (N / t::RB), max_batch * (N / t::CB)), N / r);
}

int multi_need(int n, int max_batch, int inv_tile) {
    switch (n) {
        case 64: return multi_need_n<64>(max_batch, inv_tile);
        case 128: return multi_need_n<128>(max_batch, inv_tile);
        case 256: return multi_need_n<256>(max_batch, inv_tile);
    }
    return 0;
}

int multi_col_blocks(int n) {
    switch (n) {
        case 64: return kColParts<64>;
        case 128: return kColParts<128>;
        case 256: return kColParts<256>;
    }
    return 0;
}

hipError_t build_multi_graph(const ScanArgs* dev_scans, int count, int grid, unsigned* bars, int n_bars, int* fault,
                             hipGraph_t* out) {
    if (count <= 0 || count > kMultiMax || grid <= 0 || !out) return hipErrorInvalidValue;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t zero = nullptr, run = nullptr;
    {
        void* params[] = {&bars, &n_bars};
        hipKernelNodeParams kp{};
        kp.func = reinterpret_cast<void*>(&k_zero_u32);
        kp.gridDim = dim3((unsigned)((n_bars + 255) / 256));
        kp.blockDim = dim3(256);
        kp.kernelParams = params;
        e = hipGraphAddKernelNode(&zero, g, nullptr, 0, &kp);
    }
    if (e == hipSuccess) {
        void* params[] = {&dev_scans, &count, &fault};
        hipKernelNodeParams kp{};
        kp.func = reinterpret_cast<void*>(&k_multi_persist);
        kp.gridDim = dim3(grid);
        kp.blockDim = dim3(kMP);
        kp.kernelParams = params;
        e = hipGraphAddKernelNode(&run, g, &zero, 1, &kp);
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    *out = g;
    return hipSuccess;
}

hipError_t launch_multi_persist(const ScanArgs* dev_scans, int count, int grid, unsigned* bars, int n_bars, int* fault,
                                bool coop, hipStream_t s) {
    if (count <= 0 || count > kMultiMax || grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n_bars + 255) / 256)), dim3(256), 0, s, bars, n_bars);
    if (!coop) {
        hipLaunchKernelGGL(k_multi_persist, dim3(grid), dim3(kMP), 0, s, dev_scans, count, fault);
        return hipGetLastError();
    }
    void* args[] = {&dev_scans, &count, &fault};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_multi_persist), dim3(grid), dim3(kMP), args, 0,
                                      s);
}

hipError_t build_sweep_graph(int n, int variant, const BatchArgs& a, int nb, int max_b, hipGraph_t* out) {
    if (nb < 0 || max_b <= 0 || !a.boffs || !out) return hipErrorInvalidValue;
    PTYC_DISPATCH(n, graph_v<N>(variant, a, nb, max_b, out));
    return hipErrorInvalidValue;
}

hipError_t launch_loss_fwd(int n, const BatchArgs& a, bool grad, hipStream_t s) {
    PTYC_DISPATCH(n, loss_fwd_n<N>(a, grad, s));
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_rows(int n, const BatchArgs& a, void* part, hipStream_t s) {
    PTYC_DISPATCH(n, adjoint_rows_n<N>(a, (cf*)part, s));
    return hipErrorInvalidValue;
}

hipError_t launch_grad_finish(GradFinish f, hipStream_t s) {
    f.tiles_x = (int)((f.w + kGradTC - 1) / kGradTC);
    f.n_tiles = f.tiles_x * (int)((f.h + kGradTR - 1) / kGradTR);
    f.probe_blocks = (int)((f.nn + 255) / 256);
    hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)(f.n_tiles + f.probe_blocks + 1)), dim3(256), 0, s, f);
    return hipGetLastError();
}
hipError_t launch_scale(void* p, int64_t count_c64, const double* scale, hipStream_t s) {
    if (count_c64 <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count_c64 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_scale_c64, dim3((unsigned)blocks), dim3(256), 0, s, (cf*)p, count_c64, scale);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, int64_t count_c64, hipStream_t s) {
    if (count_c64 <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count_c64 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (cf*)p, count_c64);
    return hipGetLastError();
}

hipError_t launch_sum_reduce(const double* part, int64_t n_part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_err_reduce, dim3(1), dim3(256), 0, s, part, n_part, (const OrderEntry*)nullptr,
                       (int64_t)0, (const double*)nullptr, out, 1);
    return hipGetLastError();
}

template <int N>
hipError_t amp_rowmajor_n(const float* src, float* dst, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_amp_rowmajor<N>, dim3((unsigned)count), dim3(256), 0, s, src, dst);
    return hipGetLastError();
}

hipError_t launch_amp_rowmajor(int n, const float* src, float* dst, int64_t count, hipStream_t s) {
    PTYC_DISPATCH(n, amp_rowmajor_n<N>(src, dst, count, s));
    return hipErrorInvalidValue;
}

hipError_t launch_ingest(int n, const float* src, float* dst, double* sum_i, int64_t count,
                         const IngestSpec& sp, int* bad, hipStream_t s) {
    PTYC_DISPATCH(n, ingest_n<N>(src, dst, sum_i, count, sp, bad, s));
    return hipErrorInvalidValue;
}

hipError_t launch_err_reduce(const double* err_part, int64_t n_part, const OrderEntry* order,
                             int64_t order_len, const double* sum_i, double* err_out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_err_reduce, dim3(1), dim3(256), 0, s, err_part, n_part, order, order_len,
                       sum_i, err_out, 0);
    return hipGetLastError();
}

}  // namespace ptyc

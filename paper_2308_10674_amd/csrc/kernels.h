// Launch interface between the host engine and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.h"

namespace ptyc {

// One entry of a sweep's order on the device: the position's window corner
// stored beside its index, so a stage reaches both with a single load.
struct OrderEntry {
    int32_t row, col;         // window corner (top-left) in the object
    int64_t j;                // position index (row of sqrt_i, sum_i)
};

// Stored amplitudes sqrt(I) of one position: N x N floats in blocks of
// kAmpBlock columns, block after block; element (row r, column c) at
// amp_at(N, r, c).  A column workgroup of kAmpBlock columns (or a multiple)
// then reads whole 64-byte row segments lying back to back, instead of
// sharing 128-byte lines with the workgroup of the neighbouring columns.
// At N = 16 this is the row-major layout.
constexpr int kAmpBlock = 16;
__host__ __device__ constexpr int amp_at(int n, int r, int c) {
    return ((c / kAmpBlock) * n + r) * kAmpBlock + c % kAmpBlock;
}

// Everything one batch of positions needs.  Device pointers only.
struct BatchArgs {
    cf* obj;                  // [h][w] object, updated in place
    int64_t h, w;
    cf* probe;                // [n][n] probe P_b (read by the stages, written by the reduce)
    const cf* tw;             // [n] exp(-2 pi i m / n)
    const float* sqrt_i;      // [cap][n x n] measured moduli, each position in the amp_at layout
    const int2* pos;          // [cap] window corners (row, col)
    const OrderEntry* order;  // this sweep's order
    int64_t off;              // first order entry of this batch
    int bsize;                // positions in this batch
    cf* scratch;              // [slots][n][n] spectrum exchange between stages
    float* winmax;            // [slots][Shape::row_blocks] partial max |S_j O|^2, one per forward-stage wave
    // partial maxima of |P|^2 per probe row block, double-buffered: the
    // inverse row stage reads those of P_b from pmax_in and writes those of
    // P_{b+1} to pmax_out, so no workgroup can read a partial that another
    // workgroup of the same launch has already replaced
    const float* pmax_in;     // [Shape::probe_blocks]
    float* pmax_out;          // [Shape::probe_blocks]
    double* err_part;         // [order_len][column blocks] error partial sums
    float alpha, beta;
    float gscale;             // upstream scale of the amplitude-loss gradient
    const unsigned char* mask;  // [n][n] 1 = measured detector pixel; nullptr: all measured
    const int64_t* boffs;     // graph nodes: off and bsize are read from boffs[batch], boffs[batch + 1]
    int batch;
    int n;                    // pattern size (read by the mixed-size kernels)
    int itile;                // mixed-size inverse stage: 0 the default tile, 1 the eight-slot tile
};

// How raw detector frames become stored amplitudes.
struct IngestSpec {
    int frame_h, frame_w;     // raw frame size
    int crop_y, crop_x;       // top-left corner of the n x n crop in the frame
    int orient;               // bit 0 transpose, bit 1 flip rows, bit 2 flip columns
    int centred;              // the crop has DC at (n/2, n/2)
    int is_sqrt;              // frames hold amplitudes, not counts
    float scale;              // counts are multiplied by scale
    const unsigned char* mask;  // [n][n] in the stored layout, or nullptr
};

// What the column and inverse-row stages compute.
enum : int { kModeEpie = 0, kModeGrad = 1, kModeLoss = 2 };

// Launch forms of a sweep.
enum : int { kFormBatch = 1, kFormPersistent = 2, kFormGraph = 3, kFormMixed = 4 };

// Work split per pattern size and launch form.
struct Shape {
    int row_blocks;   // winmax entries per slot (per-wave partials)
    int col_blocks;   // column items per position (error partials per position)
    int probe_blocks; // pmax entries (per-wave partials)
};

// One scan as a persistent kernel runs it: every batch of n_sweeps sweeps.
// Software barriers of the persistent kernels: a top counter, then one
// arrival counter per group of kBarGroup workgroups, each in a line of
// kBarLine unsigned (128 bytes); bar_words(gn) unsigned hold a barrier of gn
// workgroups.
constexpr int kBarGroup = 32, kBarLine = 32;
constexpr int bar_groups(int gn) { return (gn + kBarGroup - 1) / kBarGroup; }
constexpr int bar_words(int gn) { return kBarLine * (1 + bar_groups(gn)); }
// polls of a barrier wait before it gives up (about 0.1 s)
constexpr unsigned kSpinLimitDefault = 1u << 22;

struct ScanArgs {
    BatchArgs a;              // the scan's buffers; a.order holds the n_sweeps orders, olen entries each;
                              // a.pmax_in / a.pmax_out: the probe maxima halves at the start
    const int64_t* offs;      // [n_sweeps][nb + 1] batch offsets into each sweep's order (device)
    int64_t olen;             // positions per sweep
    int nb;                   // batches per sweep
    int n_sweeps;
    int g0, gn;               // workgroups g0 .. g0 + gn - 1 of the launch serve this scan
    int inv_tile;             // inverse-stage tile of the multi-scan kernel (0 or 1)
    unsigned* bar;            // barrier counters of those workgroups (bar_words(gn) unsigned), zero at the launch
    double* err;              // nullptr, or [n_sweeps] running Fourier error of each sweep (multi-scan kernel)
    unsigned spin_limit;      // polls a barrier wait may take before it raises the fault flag
    const double* sum_i;      // [positions] sum of I per position (the error's denominator)
};

bool supported_n(int n);
// variant: the per-batch tile variant (batch and graph forms; see tile_variants)
Shape shape_for(int n, int form, int variant = 0);
// number of tile variants of the per-batch kernels at pattern size n
int tile_variants(int n);

// ev: NULL, or six events: the start and end of each of the three kernels
// of the batch, taken from the kernel dispatches themselves
hipError_t launch_batch(int n, int variant, const BatchArgs& a, hipStream_t s, hipEvent_t* ev = nullptr);
// the partial maxima of |P|^2 of the current probe (no update), into a.pmax_out
hipError_t launch_probe_reduce(int n, const BatchArgs& a, int form, hipStream_t s);
// one batch of each of `count` independent reconstructions with pattern
// size n (three launches): dev_tab on the device, host_tab the same
// descriptors on the host (for the grid layout); count <= kMultiMax
constexpr int kMultiMax = 64;
// pattern sizes the mixed-size kernels serve (64, 128, 256)
bool mixed_n(int n);
// one batch of each of `count` independent reconstructions of any sizes
// that mixed_n accepts, three launches in all (the layout of kFormMixed)
hipError_t launch_batch_mixed(const BatchArgs* dev_tab, const BatchArgs* host_tab, int count, hipStream_t s);
hipError_t launch_batch_multi(int n, const BatchArgs* dev_tab, const BatchArgs* host_tab, int count,
                              hipStream_t s);
// Sequential ePIE of `count` positions a.order[a.off ..] in one workgroup
// (pattern sizes up to kStrictMaxN): the probe stays on chip and is updated
// after every position; one error partial per position at
// a.err_part[a.off + k]; a.probe holds the final probe afterwards (its
// partial maxima are not refreshed).
constexpr int kStrictMaxN = 64;
hipError_t launch_strict(int n, const BatchArgs& a, int count, hipStream_t s);
int persistent_capacity(int n);  // co-resident workgroups of the sweep kernel
// One scan's sweeps as one cooperative launch of at most `capacity`
// workgroups (the persistent form); sc.bar (bar_words(capacity) unsigned,
// the fault flag at sc.bar[1]) has its counters zeroed first.
// The kernel swaps the probe maxima halves after every non-empty batch.
hipError_t launch_sweep(int n, const ScanArgs& sc, int max_batch, int capacity, int* fault, hipStream_t s);
// Several scans (pattern sizes 64, 128, 256) as one persistent launch of
// `grid` workgroups: dev_scans[i] on the device (the same descriptors as
// host_scans, whose g0 / gn tile 0 .. grid - 1 in ascending order), their
// arrival counters inside the n_bars counters at bars (all zeroed first by
// a kernel).  coop: a
// cooperative launch (grid must not exceed multi_capacity()); otherwise a
// plain launch, which stream capture accepts.
int multi_capacity();
// workgroups a scan of pattern size n can keep busy in its largest stage
int multi_need(int n, int max_batch, int inv_tile);
// error partials per position of the multi-scan kernel at pattern size n
int multi_col_blocks(int n);
hipError_t launch_multi_persist(const ScanArgs* dev_scans, int count, int grid, unsigned* bars, int n_bars, int* fault,
                                bool coop, hipStream_t s);
// the same launch (counter reset, then the persistent kernel as a plain
// launch of `grid` workgroups) as a two-node graph
hipError_t build_multi_graph(const ScanArgs* dev_scans, int count, int grid, unsigned* bars, int n_bars, int* fault,
                             hipGraph_t* out);
// One sweep of nb batches as a graph of 3 nb kernel nodes in a chain.  The
// nodes read their batch's offset and size from a.boffs (a.boffs[b] ..
// a.boffs[b + 1] in a.order) when they run, and their grids cover max_b
// slots, so the instantiated graph serves every sweep with nb batches of at
// most max_b positions over the same buffers.  Batch 0 reads the probe
// maxima from a.pmax_in; the halves alternate from node to node (every
// node, empty or not, writes the other half), so after the graph the
// current maxima are in a.pmax_in when nb is even, else in a.pmax_out.
hipError_t build_sweep_graph(int n, int variant, const BatchArgs& a, int nb, int max_b, hipGraph_t* out);
// Amplitude loss, forward stages over a.bsize positions a.order[a.off ..]
// (windows may overlap), slot k's spectrum at a.scratch + k N^2; loss
// partials into a.err_part; grad: the column stage leaves dL/dpsi's row
// transforms in the exchange for launch_adjoint_rows.
hipError_t launch_loss_fwd(int n, const BatchArgs& a, bool grad, hipStream_t s);
// The adjoint over the same a.bsize positions after launch_loss_fwd(grad):
// the inverse row transforms give dL/dpsi of every position; its
// contribution conj(P) dL/dpsi to dL/dO replaces the position's spectrum in
// a.scratch, and the sums of conj(S_j O) dL/dpsi over each group of
// kAdjGroup consecutive positions go to part ([groups][n][n] complex64,
// groups = ceil(bsize / kAdjGroup)).
constexpr int kAdjGroup = 16, kAdjLanes = 4;
hipError_t launch_adjoint_rows(int n, const BatchArgs& a, void* part, hipStream_t s);
// The last launch of a loss with gradient.  dL/dP = the `parts` partial
// sums of dL/dP (nn complex64 each, at part) added in order, into gprobe;
// dL/dO over the whole h x w object by tiles of kGradTR x kGradTC pixels
// (row-major tile index t, ceil(w / kGradTC) tiles per row): tile t sums the
// contributions co of the slots tile_slot[tile_off[t] .. tile_off[t + 1])
// (ascending; slot k's contribution is n x n at co + k n^2 over the window
// at order[k]) and writes every pixel of the tile to gobj; the loss = the
// n_loss_part partials at loss_part summed as launch_sum_reduce does, into
// the device double *loss.  tiles_x, n_tiles and probe_blocks are filled in
// by the launcher.
constexpr int kGradTR = 16, kGradTC = 64;
struct GradFinish {
    const cf* co;
    const OrderEntry* order;
    int n;
    int64_t h, w;
    const int* tile_off;
    const int* tile_slot;
    cf* gobj;
    const cf* part;
    int64_t nn;
    int parts;
    cf* gprobe;
    const double* loss_part;
    int64_t n_loss_part;
    double* loss;
    int tiles_x, n_tiles, probe_blocks;
};
hipError_t launch_grad_finish(GradFinish f, hipStream_t s);
// multiply count complex values in place by the device scalar *scale
hipError_t launch_scale(void* p, int64_t count_c64, const double* scale, hipStream_t s);
hipError_t launch_fill_zero(void* p, int64_t count_c64, hipStream_t s);
// replace each of the k arrays (count_c64 complex values each) by their mean
hipError_t launch_mean(void* const* ptrs, int k, int64_t count_c64, hipStream_t s);
hipError_t launch_sum_reduce(const double* part, int64_t n_part, double* out, hipStream_t s);
hipError_t launch_ingest(int n, const float* src, float* sqrt_i_dst, double* sum_i_dst,
                         int64_t count, const IngestSpec& spec, int* bad_flag, hipStream_t s);
// count positions' stored amplitudes (amp_at layout) to row-major n x n
// arrays at dst (device memory)
hipError_t launch_amp_rowmajor(int n, const float* src, float* dst, int64_t count, hipStream_t s);
hipError_t launch_err_reduce(const double* err_part, int64_t n_part, const OrderEntry* order,
                             int64_t order_len, const double* sum_i, double* err_out,
                             hipStream_t s);

}  // namespace ptyc

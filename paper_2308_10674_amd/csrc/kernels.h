// Launch interface between the host engine and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.h"

namespace ptyc {

// Everything one batch of positions needs.  Device pointers only.
struct BatchArgs {
    cf* obj;                  // [h][w] object, updated in place
    int64_t h, w;
    cf* probe;                // [n][n] probe P_b (read by the stages, written by the reduce)
    const cf* tw;             // [n] exp(-2 pi i m / n)
    const float* sqrt_i;      // [cap][n][n] measured moduli
    const int2* pos;          // [cap] window corners (row, col)
    const int64_t* order;     // this sweep's position order
    int64_t off;              // first order entry of this batch
    int bsize;                // positions in this batch
    cf* scratch;              // [slots][n][n] spectrum exchange between stages
    cf* dprobe;               // [slots][n][n] per-position probe increments
    float* winmax;            // [slots][row blocks] partial max |S_j O|^2
    float* pmax_part;         // [probe blocks] partial max |P|^2 of the current probe
    int npmax;                // number of probe blocks
    double* err_part;         // [order_len][column blocks] error partial sums
    float alpha, beta;
};

// Tile shapes per pattern size: rows per row-stage workgroup, columns per
// column-stage workgroup (each workgroup has rows*N2 or cols*N2 threads).
struct Shape {
    int row_blocks;   // workgroups per position in the row stages
    int col_blocks;   // workgroups per position in the column stage
    int probe_blocks; // workgroups of the probe reduction
};

bool supported_n(int n);
Shape shape_for(int n);

hipError_t launch_batch(int n, const BatchArgs& a, hipStream_t s);
hipError_t launch_probe_reduce(int n, const BatchArgs& a, hipStream_t s);  // bsize 0: max only
hipError_t launch_ingest(int n, const float* src, float* sqrt_i_dst, double* sum_i_dst,
                         int64_t count, bool is_sqrt, bool centred, int* bad_flag,
                         hipStream_t s);
hipError_t launch_err_reduce(const double* err_part, int64_t n_part, const int64_t* order,
                             int64_t order_len, const double* sum_i, double* err_out,
                             hipStream_t s);

}  // namespace ptyc

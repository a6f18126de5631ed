// Internal interface between the HIP kernels (scf_kernels.hip) and the host runtime
// (scf_runtime.hip) of libscf.  Not installed; the public ABI is include/scf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scf {

// Per-channel constants, one table entry per channel, read by every kernel.
// Device region of a channel, in floats from the workspace base:
//   off + b*18*plane     population buffer b in {0,1}: [k][i][y][pitch], k = A,B; i = 0..8
//   off + 36*plane       density field [k][y][pitch]
//   off + 38*plane       (masked channels) solid-neighbourhood codes, uint16 [y][pitch]
struct Chan {
    int32_t nx, ny, pitch, x0, x1, xs;   // xs = x0/2: liquid-reservoir centre (scan start)
    int32_t row_base;                    // first entry of this channel in the packed row list
    int32_t masked;                      // 1: solid nodes from the mask codes, 0: wall rows
    int64_t off;                         // float offset of population buffer 0
    int64_t plane;                       // ny * pitch
    int64_t moff;                        // float offset of the code field (masked channels)
    float G;                             // bulk coupling (D2Q9 weights)
    float gw[2];                         // wall couplings
    float omega[2];                      // 1/tau_k
    float tm[2];                         // tau_k / m_k
    float wm[2];                         // m_k / tau_k
    float c1[2];                         // (1 - alpha_k) / 5: axis rest coefficient
    float c0[2];                         // alpha_k: rest-direction coefficient (used at init)
    float inv_m[2];                      // 1 / m_k
    float pad1;
};

// One row of one channel, for the per-row kernels (two-kernel step, observe, init, copies).
struct RowRef {
    int32_t chan, y;
};

// Per-row partial sums written by the observe pass.
struct RowPartial {
    double mass[2];
    int32_t bad;
    int32_t pad[3];
};

// Observation record (layout of scf_obs in include/scf.h).
struct ObsRec {
    int64_t t;
    double mass[2];
    double z, precursor, precursor_lo, precursor_hi;
    int32_t flags;
    int32_t reserved;
};

struct TileDesc {
    int32_t chan, xb, yb, ye;   // strip [xb, xb+bx) x rows [yb, ye)
    int32_t down;               // 0: rows walked upward from yb, 1: downward from ye-1
    int32_t w;                  // output columns of the strip (two-step tiles)
    int32_t pad[2];
};

// Kernel launchers (all asynchronous on `stream`; return hipSuccess or the launch error).
// launch_init builds the masked channels' codes, then the initial populations.
hipError_t launch_init(const Chan* chans, const RowRef* rows, int nrows, float* ws, hipStream_t s);
// Fused steps: with `first` non-NULL (persistent schedules) the launch has exactly `grid` blocks
// and block b runs tiles [first[b], first[b+1]); otherwise blocks stride over the whole list.
hipError_t launch_step_fused(int bx, bool masked, const Chan* chans, const TileDesc* tiles,
                             int ntiles, const int32_t* first, int grid, float* ws, int src,
                             hipStream_t s);
// Two time steps in one pass; each tile carries its output width w <= bx - 6 (see k_step_fused2).
hipError_t launch_step_fused2(int bx, bool masked, const Chan* chans, const TileDesc* tiles,
                              int ntiles, const int32_t* first, int grid, float* ws, int src,
                              hipStream_t s);
// Blocks of the fused step (fuse 1 or 2) that one CU holds at once; 0 if the query fails.
int resident_blocks_per_cu(int bx, bool masked, int fuse);
hipError_t launch_step_two_kernel(const Chan* chans, const RowRef* rows, int nrows, float* ws,
                                  int src, hipStream_t s);
hipError_t launch_observe(const Chan* chans, const RowRef* rows, int nrows, int nchan, float* ws,
                          int src, RowPartial* partials, ObsRec* now, ObsRec* ring,
                          int32_t* counter, int max_samples, int record, hipStream_t s);
hipError_t launch_pull_out(const Chan* chans, const RowRef* rows, int nrows, float* ws, int src,
                           hipStream_t s);

}  // namespace scf

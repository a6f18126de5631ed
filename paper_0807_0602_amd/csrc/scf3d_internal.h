// Internal interface between the 3-D kernels (scf3d_kernels.hip) and their host runtime
// (scf3d_runtime.hip).  Not installed; the public ABI is include/scf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace scf {
int set_error(int code, const std::string& msg);   // shared error text (scf_runtime.hip)
}

namespace scf3 {

// One 3-D channel.  Device region, in floats from the workspace base:
//   off + b*38*plane    population buffer b in {0,1}: [k][i][z][y][pitch], k = A,B; i = 0..18
//   off + 76*plane      density field [k][z][y][pitch]
struct Chan3 {
    int32_t nx, ny, nz, pitch, x0, x1, walls_y, walls_z;
    int64_t off;     // float offset of population buffer 0
    int64_t plane;   // nz * ny * pitch
    float G, gw[2], omega[2], tm[2], wm[2], inv_m[2];
    float pad;
};

struct Part3 {
    double mass[2];
    int32_t bad, pad;
};

// Observation record (layout of scf3_obs in include/scf.h).
struct Obs3 {
    int64_t t;
    double mass[2];
    double z;
    int32_t flags, reserved;
};

// `h` is the host copy of the device table entry `c` (launch geometry).
hipError_t launch_init(const Chan3& h, const Chan3* c, float* ws, hipStream_t s);
hipError_t launch_step(const Chan3& h, const Chan3* c, float* ws, int src, hipStream_t s);
// One fused launch per step: 64 x 4 (x, z) tiles walking `cy` rows of y.
hipError_t launch_step_fused(const Chan3& h, const Chan3* c, float* ws, int src, int cy, hipStream_t s);
hipError_t launch_observe(const Chan3& h, const Chan3* c, float* ws, int src, Part3* parts, Obs3* out,
                          hipStream_t s);
hipError_t launch_pull_out(const Chan3& h, const Chan3* c, float* ws, int src, hipStream_t s);

}  // namespace scf3

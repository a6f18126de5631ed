// HIP kernels for gfx950 of the three-dimensional (D3Q19) binary Shan-Chen capillary: the 3-D
// extension the paper names as future work (Conclusions), with the step of Sec. 2 written for
// D3Q19: equilibrium w_i n (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) with w = 1/3, 1/18 (axis),
// 1/36 (edge); bulk force -G psi_k sum_i w_i psi_kbar(x + c_i) c_i (psi = n, 0 on solids); wall
// force -G_kw n_k sum_i w_i s(x + c_i) c_i; common velocity U and shifted equilibrium; BGK;
// pull streaming with half-way bounce-back.  The z-projection of these weights is D2Q9 with rest
// fraction 4/9, so z-independent states follow the 2-D model.
//
// The fused step (k3_fused) walks y-slices of x-z tiles with the densities in an LDS ring; the
// two-kernel variant (k3_density, k3_collide) writes a density field and reads it back.
// Storage: FP32, f[k][i][z][y][pitch], x fastest, pitch = nx rounded up to 64.
#include "scf3d_internal.h"

// Every multiply-add is written out (no implicit contraction), as in the 2-D kernels.
#pragma clang fp contract(off)

namespace scf3 {
namespace {

constexpr int kThreads = 256;

// D3Q19 velocities: rest, six axis links, twelve edge links.
__constant__ int kCX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int kCY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int kCZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__constant__ int kOpp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

// Interaction weights of the links (rest excluded): 1/18 (axis), 1/36 (edge).
constexpr float kWA = 1.0f / 18.0f;
constexpr float kWE = 1.0f / 36.0f;
// 3 w_i for the odd part of the equilibrium: 1/6 (axis) and 1/12 (edge), with 1/6 carried as
// two terms (a single rounded constant would bias the equilibrium momentum at every step).
constexpr float kSixthHi = 1.0f / 6.0f;
constexpr float kSixthLo = (float)(1.0 / 6.0 - (double)kSixthHi);

__device__ __forceinline__ float sixth(float v) { return __builtin_fmaf(v, kSixthHi, v * kSixthLo); }

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ bool solid(const Chan3& c, int x, int y, int z) {
    if ((unsigned)(x - c.x0) >= (unsigned)(c.x1 - c.x0)) return false;
    return (c.walls_y && (y == 0 || y == c.ny - 1)) || (c.walls_z && (z == 0 || z == c.nz - 1));
}

__device__ __forceinline__ int64_t idx(const Chan3& c, int x, int y, int z) {
    return ((int64_t)z * c.ny + y) * c.pitch + x;
}

// Populations f_i(x, t) of both components streaming into (x, y, z) from buffer g.
__device__ __forceinline__ void pull(const float* __restrict__ g, const Chan3& c, int x, int y, int z,
                                     float f[38]) {
    const int64_t own = idx(c, x, y, z);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int xs = wrapc(x - kCX[i], c.nx), ys = wrapc(y - kCY[i], c.ny), zs = wrapc(z - kCZ[i], c.nz);
        int pi = i;
        int64_t src = idx(c, xs, ys, zs);
        if (i > 0 && solid(c, xs, ys, zs)) {
            pi = kOpp[i];
            src = own;
        }
        f[i] = g[pi * c.plane + src];
        f[19 + i] = g[(19 + pi) * c.plane + src];
    }
}

__device__ __forceinline__ float sum19(const float* f) {
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 19; ++i) s += f[i];
    return s;
}

__global__ void __launch_bounds__(kThreads)
k3_density(const Chan3* __restrict__ cp, float* __restrict__ ws, int src) {
    const Chan3 c = *cp;
    const int x = blockIdx.x * kThreads + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= c.nx) return;
    const float* __restrict__ g = ws + c.off + (int64_t)src * 38 * c.plane;
    float* __restrict__ dn = ws + c.off + 76 * c.plane;
    float nA = 0.0f, nB = 0.0f;
    if (!solid(c, x, y, z)) {
        float f[38];
        pull(g, c, x, y, z, f);
        nA = sum19(f);
        nB = sum19(f + 19);
    }
    dn[idx(c, x, y, z)] = nA;
    dn[c.plane + idx(c, x, y, z)] = nB;
}

// Deviation-form BGK of one component: D_i = (w_i n - f_i) + n w_i (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)
// for i > 0, D_0 = -sum D_i; f*_i = f_i + omega D_i.
__device__ __forceinline__ void relax(const float* f, float n, float ux, float uy, float uz, float om,
                                      float* __restrict__ out, int64_t P, int64_t at) {
    const float usq = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
    float D[19];
    float sumD = 0.0f;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const float cu = (float)kCX[i] * ux + (float)kCY[i] * uy + (float)kCZ[i] * uz;
        const bool axis = i < 7;
        const float w = axis ? kWA : kWE;
        const float odd = axis ? sixth(cu) : 0.5f * sixth(cu);            // 3 w_i c.u
        const float even = w * __builtin_fmaf(4.5f * cu, cu, -1.5f * usq);  // w_i (9/2 cu^2 - 3/2 u^2)
        D[i] = __builtin_fmaf(n, odd + even, w * n - f[i]);
        sumD += D[i];
    }
    D[0] = -sumD;
#pragma unroll
    for (int i = 0; i < 19; ++i) out[i * P + at] = __builtin_fmaf(om, D[i], f[i]);
}

__global__ void __launch_bounds__(kThreads)
k3_collide(const Chan3* __restrict__ cp, float* __restrict__ ws, int src) {
    const Chan3 c = *cp;
    const int x = blockIdx.x * kThreads + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= c.nx || solid(c, x, y, z)) return;
    const float* __restrict__ g = ws + c.off + (int64_t)src * 38 * c.plane;
    float* __restrict__ d = ws + c.off + (int64_t)(src ^ 1) * 38 * c.plane;
    const float* __restrict__ nAf = ws + c.off + 76 * c.plane;
    const float* __restrict__ nBf = nAf + c.plane;
    float f[38];
    pull(g, c, x, y, z, f);
    const float nA = sum19(f), nB = sum19(f + 19);
    float jA[3] = {0.0f, 0.0f, 0.0f}, jB[3] = {0.0f, 0.0f, 0.0f};
    float sA[3] = {0.0f, 0.0f, 0.0f}, sB[3] = {0.0f, 0.0f, 0.0f}, sw[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const float cx = (float)kCX[i], cy = (float)kCY[i], cz = (float)kCZ[i];
        jA[0] += cx * f[i]; jA[1] += cy * f[i]; jA[2] += cz * f[i];
        jB[0] += cx * f[19 + i]; jB[1] += cy * f[19 + i]; jB[2] += cz * f[19 + i];
        const int xn = wrapc(x + kCX[i], c.nx), yn = wrapc(y + kCY[i], c.ny), zn = wrapc(z + kCZ[i], c.nz);
        const int64_t nb = idx(c, xn, yn, zn);
        const float w = i < 7 ? kWA : kWE;
        const float a = w * nAf[nb], b = w * nBf[nb];
        const float s = solid(c, xn, yn, zn) ? w : 0.0f;
        sA[0] += a * cx; sA[1] += a * cy; sA[2] += a * cz;
        sB[0] += b * cx; sB[1] += b * cy; sB[2] += b * cz;
        sw[0] += s * cx; sw[1] += s * cy; sw[2] += s * cz;
    }
    // accelerations a_k = F_k / n_k
    float aA[3], aB[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        aA[q] = __builtin_fmaf(-c.G, sB[q], -(c.gw[0] * sw[q]));
        aB[q] = __builtin_fmaf(-c.G, sA[q], -(c.gw[1] * sw[q]));
    }
    const float inv = 1.0f / __builtin_fmaf(c.wm[0], nA, c.wm[1] * nB);
    float U[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) U[q] = __builtin_fmaf(c.wm[0], jA[q], c.wm[1] * jB[q]) * inv;
    const int64_t at = idx(c, x, y, z);
    relax(f, nA, __builtin_fmaf(c.tm[0], aA[0], U[0]), __builtin_fmaf(c.tm[0], aA[1], U[1]),
          __builtin_fmaf(c.tm[0], aA[2], U[2]), c.omega[0], d, c.plane, at);
    relax(f + 19, nB, __builtin_fmaf(c.tm[1], aB[0], U[0]), __builtin_fmaf(c.tm[1], aB[1], U[1]),
          __builtin_fmaf(c.tm[1], aB[2], U[2]), c.omega[1], d + 19 * c.plane, c.plane, at);
}

// ---------------------------------------------------------------------------------------------
// Fused 3-D step.  A block of BX x BZ threads owns the columns x in [xb, xb + BX), z in
// [zb, zb + BZ) and walks rows y upward through [yb, ye).  Iteration `it` pulls one y-slice of
// the tile plus its one-node halo ring in x and z (the ring's nodes are pulled by the first
// 2 (BX + 2) + 2 BZ threads), writes the slice's densities into a 4-slot LDS ring, and after
// one barrier collides the previous slice, whose populations were kept in registers: all 18
// neighbour densities of a node come from three ring slots.  The first and last slices pulled
// are density-only halos.  A slot written at iteration it+1 was last read by the collision of
// iteration it-1, finished by every thread before the barrier of iteration it.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ bool in_x(const Chan3& c, int x) { return (unsigned)(x - c.x0) < (unsigned)(c.x1 - c.x0); }

// True if a solid node may lie among (x, y, z) and its 18 neighbours (periodic in x).
__device__ __forceinline__ bool near_solid(const Chan3& c, int x, int y, int z) {
    if (!in_x(c, wrapc(x - 1, c.nx)) && !in_x(c, x) && !in_x(c, wrapc(x + 1, c.nx))) return false;
    return (c.walls_y && (y <= 1 || y >= c.ny - 2)) || (c.walls_z && (z <= 1 || z >= c.nz - 2));
}

// Buffer-descriptor access for the fused step: one descriptor per component of the source buffer
// (19 planes, at most 4 GiB, checked by the host), unsigned 32-bit byte offsets, plane offsets in
// scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)(uint32_t)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ unsigned idx32(const Chan3& c, int x, int y, int z) {
    return ((unsigned)z * (unsigned)c.ny + (unsigned)y) * (unsigned)c.pitch + (unsigned)x;
}

// As pull, through the descriptors rA, rB of the two components (Pb = plane bytes); WALLS adds
// the bounce-back tests.
template <bool WALLS>
__device__ __forceinline__ void pull_buf(__amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rB, unsigned Pb,
                                         const Chan3& c, int x, int y, int z, float f[38]) {
    const unsigned own = idx32(c, x, y, z) * 4u;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int xs = wrapc(x - kCX[i], c.nx), ys = wrapc(y - kCY[i], c.ny), zs = wrapc(z - kCZ[i], c.nz);
        const unsigned off = idx32(c, xs, ys, zs) * 4u;
        if (WALLS && i > 0) {
            // bounce-back lanes read their own node's opposite direction: the plane goes into the
            // per-lane offset so the scalar offset stays uniform
            const unsigned o = solid(c, xs, ys, zs) ? own + (unsigned)kOpp[i] * Pb : off + (unsigned)i * Pb;
            f[i] = bload(rA, o, 0u);
            f[19 + i] = bload(rB, o, 0u);
        } else {
            f[i] = bload(rA, off, (unsigned)i * Pb);
            f[19 + i] = bload(rB, off, (unsigned)i * Pb);
        }
    }
}

__device__ __forceinline__ void pull_any(__amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rB, unsigned Pb,
                                         const Chan3& c, int x, int y, int z, float f[38]) {
    if (near_solid(c, x, y, z))
        pull_buf<true>(rA, rB, Pb, c, x, y, z, f);
    else
        pull_buf<false>(rA, rB, Pb, c, x, y, z, f);
}

template <int BX, int BZ>
__global__ void __launch_bounds__(BX * BZ)
k3_fused(const Chan3* __restrict__ cp, float* __restrict__ ws, int src, int cy) {
    constexpr int SX = BX + 2, SZ = BZ + 2;
    constexpr int NH = 2 * SX + 2 * BZ;   // halo ring of the x-z tile
    static_assert(NH <= BX * BZ, "one thread per halo node");
    __shared__ float sn[2][4][SZ][SX];
    const Chan3 c = *cp;
    const int tid = threadIdx.x;
    const int tx = tid % BX, tz = tid / BX;
    // Workgroups are dispatched to the eight XCDs in turn (block b to XCD b mod 8), each XCD with
    // its own L2.  Give XCD k the k-th contiguous eighth of the tiles (x fastest, then z, then
    // the row chunk), so that the tiles whose halos overlap share one L2.
    const int gx = (c.nx + BX - 1) / BX, gz = (c.nz + BZ - 1) / BZ;
    const int ntiles = gridDim.x;
    const int blk = blockIdx.x, xcd = blk & 7, per = ntiles >> 3, rem = ntiles & 7;
    const int t = xcd * per + min(xcd, rem) + (blk >> 3);
    const int xb = (t % gx) * BX, zb = ((t / gx) % gz) * BZ;
    const int yb = (t / gx / gz) * cy, ye = min(yb + cy, c.ny);
    // Tile columns past the edge of the box hold the periodic images of nodes (as many times over
    // as needed when the box is narrower than the tile), so the LDS neighbours of every active
    // column are the true periodic neighbours; only active threads collide and store.
    const bool act = xb + tx < c.nx && zb + tz < c.nz;
    const int x = (xb + tx) % c.nx, z = (zb + tz) % c.nz;
    // halo node of this thread (ring position h = tid), in tile coordinates (hx, hz) in [0, SX) x [0, SZ)
    int hx = 0, hz = 0;
    if (tid < SX) {
        hx = tid; hz = 0;
    } else if (tid < 2 * SX) {
        hx = tid - SX; hz = SZ - 1;
    } else if (tid < 2 * SX + BZ) {
        hx = 0; hz = 1 + tid - 2 * SX;
    } else {
        hx = SX - 1; hz = 1 + tid - 2 * SX - BZ;
    }
    const int hxg = (xb - 1 + hx + c.nx) % c.nx, hzg = (zb - 1 + hz + c.nz) % c.nz;
    const bool halo = tid < NH;
    const int64_t comp_bytes = (int64_t)19 * c.plane * 4;
    const float* gsrc = ws + c.off + (int64_t)src * 38 * c.plane;
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(gsrc, comp_bytes);
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(gsrc + 19 * c.plane, comp_bytes);
    const unsigned Pb = (unsigned)(c.plane * 4);
    float* __restrict__ d = ws + c.off + (int64_t)(src ^ 1) * 38 * c.plane;
    float q[38];
#pragma unroll
    for (int i = 0; i < 38; ++i) q[i] = 0.0f;
    float qA = 0.0f, qB = 0.0f;
    int y = wrapc(yb - 1, c.ny);
    const int niter = ye - yb + 2;
    for (int it = 0; it < niter; ++it) {
        const int slot = it & 3;
        // the halo ring first, so that its registers are free again before the slice's own pull
        if (halo) {
            float h[38];
            float hA = 0.0f, hB = 0.0f;
            if (!solid(c, hxg, y, hzg)) {
                pull_any(rA, rB, Pb, c, hxg, y, hzg, h);
                hA = sum19(h);
                hB = sum19(h + 19);
            }
            sn[0][slot][hz][hx] = hA;
            sn[1][slot][hz][hx] = hB;
        }
        float p[38];
        float nA = 0.0f, nB = 0.0f;
        const bool sol = solid(c, x, y, z);
        pull_any(rA, rB, Pb, c, x, y, z, p);
        if (!sol) {
            nA = sum19(p);
            nB = sum19(p + 19);
        }
        sn[0][slot][tz + 1][tx + 1] = nA;
        sn[1][slot][tz + 1][tx + 1] = nB;
        __syncthreads();
        const int yc = y == 0 ? c.ny - 1 : y - 1;   // the slice pulled one iteration ago
        if (it >= 2 && act && !solid(c, x, yc, z)) {
            const int sy[3] = {(it - 2) & 3, (it - 1) & 3, slot};   // slices yc - 1, yc, yc + 1
            float jA[3] = {0.0f, 0.0f, 0.0f}, jB[3] = {0.0f, 0.0f, 0.0f};
            float sA[3] = {0.0f, 0.0f, 0.0f}, sB[3] = {0.0f, 0.0f, 0.0f}, sw[3] = {0.0f, 0.0f, 0.0f};
            const bool nw = near_solid(c, x, yc, z);
#pragma unroll
            for (int i = 1; i < 19; ++i) {
                const float cx = (float)kCX[i], cyf = (float)kCY[i], cz = (float)kCZ[i];
                jA[0] += cx * q[i]; jA[1] += cyf * q[i]; jA[2] += cz * q[i];
                jB[0] += cx * q[19 + i]; jB[1] += cyf * q[19 + i]; jB[2] += cz * q[19 + i];
                const int s = sy[kCY[i] + 1];
                const float w = i < 7 ? kWA : kWE;
                const float a = w * sn[0][s][tz + 1 + kCZ[i]][tx + 1 + kCX[i]];
                const float b = w * sn[1][s][tz + 1 + kCZ[i]][tx + 1 + kCX[i]];
                sA[0] += a * cx; sA[1] += a * cyf; sA[2] += a * cz;
                sB[0] += b * cx; sB[1] += b * cyf; sB[2] += b * cz;
                if (nw) {
                    const float so = solid(c, wrapc(x + kCX[i], c.nx), wrapc(yc + kCY[i], c.ny),
                                           wrapc(z + kCZ[i], c.nz)) ? w : 0.0f;
                    sw[0] += so * cx; sw[1] += so * cyf; sw[2] += so * cz;
                }
            }
            float aA[3], aB[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                aA[k] = __builtin_fmaf(-c.G, sB[k], -(c.gw[0] * sw[k]));
                aB[k] = __builtin_fmaf(-c.G, sA[k], -(c.gw[1] * sw[k]));
            }
            const float inv = 1.0f / __builtin_fmaf(c.wm[0], qA, c.wm[1] * qB);
            float U[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) U[k] = __builtin_fmaf(c.wm[0], jA[k], c.wm[1] * jB[k]) * inv;
            const int64_t at = idx(c, x, yc, z);
            relax(q, qA, __builtin_fmaf(c.tm[0], aA[0], U[0]), __builtin_fmaf(c.tm[0], aA[1], U[1]),
                  __builtin_fmaf(c.tm[0], aA[2], U[2]), c.omega[0], d, c.plane, at);
            relax(q + 19, qB, __builtin_fmaf(c.tm[1], aB[0], U[0]), __builtin_fmaf(c.tm[1], aB[1], U[1]),
                  __builtin_fmaf(c.tm[1], aB[2], U[2]), c.omega[1], d + 19 * c.plane, c.plane, at);
        }
#pragma unroll
        for (int i = 0; i < 38; ++i) q[i] = p[i];
        qA = nA;
        qB = nB;
        y = y == c.ny - 1 ? 0 : y + 1;
    }
}

// Initial state: the resident buffer holds the populations whose pull is the rest equilibrium
// w_i n0(x): g_i(x) = w_i n0(x + c_i) if x + c_i is fluid, else w_i n0(x).  The FP64 host
// fields (nz*ny*nx each) are staged in population buffer 1.
__global__ void __launch_bounds__(kThreads)
k3_init(const Chan3* __restrict__ cp, float* __restrict__ ws) {
    const Chan3 c = *cp;
    const int x = blockIdx.x * kThreads + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= c.nx) return;
    const double* __restrict__ rho = reinterpret_cast<const double*>(ws + c.off + 38 * c.plane);
    float* __restrict__ g = ws + c.off;
    const int64_t cells = (int64_t)c.nx * c.ny * c.nz;
    const bool sol = solid(c, x, y, z);
    const int64_t at = idx(c, x, y, z);
    for (int k = 0; k < 2; ++k) {
        const double* rk = rho + k * cells;
        const double n0 = rk[((int64_t)z * c.ny + y) * c.nx + x] * (double)c.inv_m[k];
        for (int i = 0; i < 19; ++i) {
            const float w = i == 0 ? 1.0f / 3.0f : (i < 7 ? kWA : kWE);
            const int xn = wrapc(x + kCX[i], c.nx), yn = wrapc(y + kCY[i], c.ny), zn = wrapc(z + kCZ[i], c.nz);
            double nn = n0;
            if (!solid(c, xn, yn, zn)) nn = rk[((int64_t)zn * c.ny + yn) * c.nx + xn] * (double)c.inv_m[k];
            g[(k * 19 + i) * c.plane + at] = sol ? 0.0f : w * (float)nn;
        }
    }
}

// Pulled populations f(t) of every node into buffer 1 - src.
__global__ void __launch_bounds__(kThreads)
k3_pull_out(const Chan3* __restrict__ cp, float* __restrict__ ws, int src) {
    const Chan3 c = *cp;
    const int x = blockIdx.x * kThreads + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= c.nx) return;
    const float* __restrict__ g = ws + c.off + (int64_t)src * 38 * c.plane;
    float* __restrict__ o = ws + c.off + (int64_t)(src ^ 1) * 38 * c.plane;
    float f[38];
    const bool sol = solid(c, x, y, z);
    if (!sol) pull(g, c, x, y, z, f);
    const int64_t at = idx(c, x, y, z);
#pragma unroll
    for (int i = 0; i < 38; ++i) o[i * c.plane + at] = sol ? 0.0f : f[i];
}

// Observables from the density field (k3_density first): FP64 mass per (y, z) row and a health
// flag, then one block sums the rows in order and finds the centre-line front.  Block reductions
// run in a fixed order: a butterfly over each wave's 64 lanes, then the wave results through LDS.
constexpr int kWaves = kThreads / 64;

template <typename T>
__device__ __forceinline__ T bsum(T v, T* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) r += sh[w];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int bmin(int v, int* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) r = min(r, sh[w]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kThreads)
k3_obs_rows(const Chan3* __restrict__ cp, const float* __restrict__ ws, Part3* __restrict__ parts) {
    __shared__ double sd[kWaves];
    __shared__ int si[kWaves];
    const Chan3 c = *cp;
    const int y = blockIdx.x, z = blockIdx.y;
    const float* __restrict__ nAf = ws + c.off + 76 * c.plane;
    const float* __restrict__ nBf = nAf + c.plane;
    double mA = 0.0, mB = 0.0;
    int bad = 0;
    for (int x = threadIdx.x; x < c.nx; x += kThreads) {
        if (solid(c, x, y, z)) continue;
        const float a = nAf[idx(c, x, y, z)], b = nBf[idx(c, x, y, z)];
        mA += (double)a;
        mB += (double)b;
        if (!(a >= -1e-3f) || !(b >= -1e-3f) || !isfinite(a) || !isfinite(b)) bad = 1;
    }
    mA = bsum(mA, sd);
    mB = bsum(mB, sd);
    bad = bsum(bad, si);
    if (threadIdx.x == 0) {
        Part3 p;
        p.mass[0] = mA;
        p.mass[1] = mB;
        p.bad = bad;
        p.pad = 0;
        parts[(int64_t)z * c.ny + y] = p;
    }
}

__global__ void __launch_bounds__(kThreads)
k3_obs_final(const Chan3* __restrict__ cp, const float* __restrict__ ws, const Part3* __restrict__ parts,
             Obs3* __restrict__ out) {
    __shared__ double sd[kWaves];
    __shared__ int si[kWaves];
    const Chan3 c = *cp;
    const int tid = threadIdx.x;
    const float* __restrict__ nAf = ws + c.off + 76 * c.plane;
    const float* __restrict__ nBf = nAf + c.plane;
    double mA = 0.0, mB = 0.0;
    int bad = 0;
    for (int r = tid; r < c.ny * c.nz; r += kThreads) {
        mA += parts[r].mass[0];
        mB += parts[r].mass[1];
        bad |= parts[r].bad;
    }
    mA = bsum(mA, sd);
    mB = bsum(mB, sd);
    bad = bsum(bad, si);
    // centre line: the (up to) four lines nearest (y, z) = ((ny-1)/2, (nz-1)/2)
    const int ys[2] = {(c.ny - 1) / 2, c.ny / 2}, zs[2] = {(c.nz - 1) / 2, c.nz / 2};
    auto phi = [&](int x) -> double {
        double v = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                v += 0.25 * ((double)nAf[idx(c, x, ys[a], zs[b])] - (double)nBf[idx(c, x, ys[a], zs[b])]);
        return v;
    };
    const int big = 0x7fffffff;
    int xz = big;
    const int xs0 = c.x0 / 2;
    for (int x = xs0 + tid; x + 1 < c.nx; x += kThreads)
        if (xz == big && phi(x) >= 0.0 && phi(x + 1) < 0.0) xz = x;
    xz = bmin(xz, si);
    if (tid == 0) {
        Obs3 o;
        o.t = 0;
        o.mass[0] = mA;
        o.mass[1] = mB;
        if (xz == big) {
            o.z = __builtin_nan("");
        } else {
            const double a = phi(xz), b = phi(xz + 1);
            o.z = (double)xz + a / (a - b) - (double)c.x0;
        }
        o.flags = (phi(xs0) < 0.0 ? 1 : 0) | (bad ? 2 : 0);
        o.reserved = 0;
        *out = o;
    }
}

dim3 grid_of(const Chan3& c) { return dim3((c.nx + kThreads - 1) / kThreads, c.ny, c.nz); }

}  // namespace

hipError_t launch_init(const Chan3& h, const Chan3* c, float* ws, hipStream_t s) {
    hipLaunchKernelGGL(k3_init, grid_of(h), dim3(kThreads), 0, s, c, ws);
    return hipGetLastError();
}

hipError_t launch_step(const Chan3& h, const Chan3* c, float* ws, int src, hipStream_t s) {
    hipLaunchKernelGGL(k3_density, grid_of(h), dim3(kThreads), 0, s, c, ws, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_collide, grid_of(h), dim3(kThreads), 0, s, c, ws, src);
    return hipGetLastError();
}

hipError_t launch_step_fused(const Chan3& h, const Chan3* c, float* ws, int src, int cy, hipStream_t s) {
    constexpr int BX = 64, BZ = 4;
    cy = cy < 1 ? 1 : (cy > h.ny ? h.ny : cy);
    const int64_t ntiles = (int64_t)((h.nx + BX - 1) / BX) * ((h.nz + BZ - 1) / BZ) * ((h.ny + cy - 1) / cy);
    if (ntiles > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k3_fused<BX, BZ>), dim3((unsigned)ntiles), dim3(BX * BZ), 0, s, c, ws, src, cy);
    return hipGetLastError();
}

hipError_t launch_observe(const Chan3& h, const Chan3* c, float* ws, int src, Part3* parts, Obs3* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k3_density, grid_of(h), dim3(kThreads), 0, s, c, ws, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_obs_rows, dim3(h.ny, h.nz), dim3(kThreads), 0, s, c, ws, parts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_obs_final, dim3(1), dim3(kThreads), 0, s, c, ws, parts, out);
    return hipGetLastError();
}

hipError_t launch_pull_out(const Chan3& h, const Chan3* c, float* ws, int src, hipStream_t s) {
    hipLaunchKernelGGL(k3_pull_out, grid_of(h), dim3(kThreads), 0, s, c, ws, src);
    return hipGetLastError();
}

}  // namespace scf3

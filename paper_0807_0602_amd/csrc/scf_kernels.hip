// HIP kernels for gfx950 of the binary Shan-Chen capillary-filling step.
//
// Model (S. Chibbaro, "Capillary filling with pseudo-potential binary Lattice-Boltzmann
// model", Sec. 2): per component k in {A, B} a D2Q9 BGK equation (eq. lbe) whose equilibrium
// (eqs. feq1-feq3) is evaluated at a shifted velocity u_k^eq = U + tau_k F_k / rho_k, with the
// common velocity U = sum_k (rho_k u_k / tau_k) / sum_k (rho_k / tau_k), the bulk
// pseudo-potential force of eq. forcing (psi = n, cross-component coupling only) and the wall
// force of eq. forcingw.  Walls are solid rows with half-way bounce-back (Sec. 3, Fig. 1), or
// the nodes of an optional solid mask.
//
// Storage: FP32, structure of arrays per component and direction, rows padded to 64 floats.
// The resident buffer holds POST-COLLISION populations f*(t-1); a step pulls
// f_i(x, t) = f*_i(x - c_i, t-1) (or the node's own opposite population when x - c_i is solid),
// forms n_k(x, t), computes forces from the neighbours' n_k(t), collides and stores f*(t).
//
// Direction numbering of Sec. 2:
//   i :  0  1  2  3  4  5  6  7  8
//   cx:  0  1  0 -1  0  1 -1 -1  1
//   cy:  0  0  1  0 -1  1  1 -1 -1
#include "scf_internal.h"

// No implicit multiply-add contraction: every fused multiply-add below is written out, so the
// rounding of each expression is fixed by the source and every kernel instantiation (block
// width, masked or row-walled channel) computes a node bit for bit alike.
#pragma clang fp contract(off)

namespace scf {
namespace {

constexpr float W1 = 1.0f / 9.0f;    // interaction weight of axis links
constexpr float W2 = 1.0f / 36.0f;   // interaction weight of diagonal links
constexpr int kRowThreads = 256;     // block size of the per-row kernels

__device__ __forceinline__ bool solid_at(const Chan& c, int x, int y) {
    return (y == 0 || y == c.ny - 1) && (unsigned)(x - c.x0) < (unsigned)(c.x1 - c.x0);
}
__device__ __forceinline__ int dec_wrap(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int inc_wrap(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// Rows 0, 1, ny-2, ny-1 may touch a solid row node; all others never do.
__device__ __forceinline__ bool near_wall(const Chan& c, int y) {
    return c.x1 > c.x0 && (y <= 1 || y >= c.ny - 2);
}

// Solid-neighbourhood code of node (x, y): bit i is set when x + c_i is solid (bit 0: the node
// itself).  Population i streams in from x - c_i = x + c_opp(i), so it bounces back when bit
// opp(i) is set; the wall force sums the weighted directions of the set bits 1..8.
__device__ __forceinline__ uint32_t rows_code(const Chan& c, int x, int y) {
    const int xm = dec_wrap(x, c.nx), xp = inc_wrap(x, c.nx);
    const int ym = dec_wrap(y, c.ny), yp = inc_wrap(y, c.ny);
    const int nxs[9] = {x, xp, x, xm, x, xp, xm, xm, xp};   // x + c_i
    const int nys[9] = {y, y, yp, y, ym, yp, yp, ym, ym};
    uint32_t code = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) code |= (uint32_t)solid_at(c, nxs[i], nys[i]) << i;
    return code;
}

// Code of a masked channel, precomputed at init (k_codes) as one uint16 per node.
__device__ __forceinline__ uint32_t mask_code(const Chan& c, const float* ws, int x, int y) {
    return reinterpret_cast<const uint16_t*>(ws + c.moff)[y * c.pitch + x];
}

// Either kind; 0 for the rows of a row-walled channel that touch no solid node.
__device__ __forceinline__ uint32_t node_code(const Chan& c, const float* ws, int x, int y) {
    if (c.masked) return mask_code(c, ws, x, y);
    return near_wall(c, y) ? rows_code(c, x, y) : 0u;
}

// Pull the 18 populations streaming into node (x, y) from post-collision buffer g; with WALLS,
// `code` (see rows_code) selects the bounce-back directions.
template <bool WALLS>
__device__ __forceinline__ void pull18(const float* __restrict__ g, const Chan& c, int x, int y,
                                       uint32_t code, float f[18]) {
    const int xm = dec_wrap(x, c.nx), xp = inc_wrap(x, c.nx);
    const int ym = dec_wrap(y, c.ny), yp = inc_wrap(y, c.ny);
    const int64_t P = c.plane;
    const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
    const int sy[9] = {y, y, ym, y, yp, ym, ym, yp, yp};
    const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int pi = i;
        int idx = sy[i] * c.pitch + sx[i];
        if (WALLS && i > 0 && ((code >> opp[i]) & 1u)) {
            pi = opp[i];
            idx = y * c.pitch + x;
        }
        f[i] = g[pi * P + idx];
        f[9 + i] = g[(9 + pi) * P + idx];
    }
}

// Pull of node (x, y) for the per-row kernels; returns the node's solid-neighbourhood code.
__device__ __forceinline__ uint32_t pull_node(const float* __restrict__ g, const Chan& c,
                                              const float* ws, int x, int y, float f[18]) {
    const uint32_t code = node_code(c, ws, x, y);
    if (c.masked || near_wall(c, y))
        pull18<true>(g, c, x, y, code, f);
    else
        pull18<false>(g, c, x, y, 0u, f);
    return code;
}

// Buffer-descriptor access for the fused step: one descriptor per population buffer (18 planes,
// at most 4 GiB, checked by the host), 32-bit byte offsets, plane offsets in scalar registers.
constexpr int kBufferDword3 = 0x00020000;   // raw buffer, 32-bit data format (gfx9 family)

// Byte counts and offsets are unsigned 32-bit values (the builtins take them as int bit patterns).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)(uint32_t)bytes, kBufferDword3);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// As pull18, through a buffer descriptor; Pb = plane size in bytes.
template <bool WALLS>
__device__ __forceinline__ void pull18_buf(__amdgpu_buffer_rsrc_t r, uint32_t Pb, const Chan& c, int x,
                                           int y, uint32_t code, float f[18]) {
    const int xm = dec_wrap(x, c.nx), xp = inc_wrap(x, c.nx);
    const int ym = dec_wrap(y, c.ny), yp = inc_wrap(y, c.ny);
    const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
    const int sy[9] = {y, y, ym, y, yp, ym, ym, yp, yp};
    const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t off = ((uint32_t)sy[i] * (uint32_t)c.pitch + (uint32_t)sx[i]) * 4u;
        if (WALLS && i > 0) {
            // bounce-back lanes read their own node's opposite direction: fold the plane into
            // the per-lane offset so the scalar offset stays uniform
            const bool sol = (code >> opp[i]) & 1u;
            const uint32_t o = sol ? ((uint32_t)y * (uint32_t)c.pitch + (uint32_t)x) * 4u + (uint32_t)opp[i] * Pb
                                   : off + (uint32_t)i * Pb;
            f[i] = bload(r, o, 0u);
            f[9 + i] = bload(r, o, 9u * Pb);
        } else {
            f[i] = bload(r, off, (uint32_t)i * Pb);
            f[9 + i] = bload(r, off, (uint32_t)(9 + i) * Pb);
        }
    }
}

// Pull for the fused step; returns the node's solid-neighbourhood code.  MASK instantiates the
// masked-channel path (a code load per node); row-walled channels test their rows instead.
template <bool MASK>
__device__ __forceinline__ uint32_t pull_node_buf(__amdgpu_buffer_rsrc_t r, uint32_t Pb, const Chan& c,
                                                  const float* ws, int x, int y, float f[18]) {
    if (MASK && c.masked) {
        const uint32_t code = mask_code(c, ws, x, y);
        pull18_buf<true>(r, Pb, c, x, y, code, f);
        return code;
    }
    if (near_wall(c, y)) {
        const uint32_t code = rows_code(c, x, y);
        pull18_buf<true>(r, Pb, c, x, y, code, f);
        return code;
    }
    pull18_buf<false>(r, Pb, c, x, y, 0u, f);
    return 0u;
}

// Destinations of the post-collision populations: plain global stores or buffer stores.  The
// single step's stores are non-temporal (the values are not read again within the step, and each
// wave writes whole cache lines).  The two-step kernel stores through the cache: its lanes are
// offset by two columns from the output strip, so each wave covers parts of three lines, and
// non-temporal partial lines reached memory twice (85 instead of 72 written bytes per node).
struct GlobalOut {
    float* d;
    int64_t P;
    int idx;
    __device__ __forceinline__ void operator()(int q, float v) const {
        __builtin_nontemporal_store(v, &d[q * P + idx]);
    }
};
template <int AUX>   // 2: non-temporal, 0: cached
struct BufferOutT {
    __amdgpu_buffer_rsrc_t r;
    uint32_t Pb;
    uint32_t off;
    __device__ __forceinline__ void operator()(int q, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off,
                                              (int)((uint32_t)q * Pb), AUX);
    }
};
using BufferOut = BufferOutT<2>;
using BufferOutCached = BufferOutT<0>;

__device__ __forceinline__ float sum9(const float* f) {
    float s = f[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) s += f[i];
    return s;
}

// One Cartesian component of sum_i w_i v(x + c_i) c_i: the axis pair (p, m) along the axis and
// the diagonal pairs (p1, m1), (p2, m2) whose component is +1 / -1.
__device__ __forceinline__ float link_sum(float p, float m, float p1, float m1, float p2, float m2) {
    return __builtin_fmaf(W1, p - m, W2 * ((p1 - m1) + (p2 - m2)));
}

// sum_i w_i s(x + c_i) c_i over solid neighbours (eq. forcingw without -n_k G_kw), from the
// node's solid-neighbourhood code.
__device__ __forceinline__ void wall_sum(uint32_t code, float& sx, float& sy) {
    const float sE = (code >> 1) & 1u, sN = (code >> 2) & 1u;
    const float sW = (code >> 3) & 1u, sS = (code >> 4) & 1u;
    const float sNE = (code >> 5) & 1u, sNW = (code >> 6) & 1u;
    const float sSW = (code >> 7) & 1u, sSE = (code >> 8) & 1u;
    sx = link_sum(sE, sW, sNE, sSW, sSE, sNW);
    sy = link_sum(sN, sS, sNE, sSW, sNW, sSE);
}

// Equilibrium of eqs. feq1-feq3 at (n, u) and BGK relaxation of one component's 9 populations,
// f*_i = f_i + omega D_i with D_i = f_i^eq - f_i.  For i > 0 the equilibrium is the rest part
// r_i = n (1 - alpha)/5 (axis) or a quarter of it (diagonal) plus n times (or n/4 times)
//   c.u/3 + (c.u)^2/2 - u.u/6,
// and D_i is formed as (r_i - f_i) + n dev_i so that only small numbers are rounded; the rest
// direction takes D_0 = -sum_{i>0} D_i, which keeps the node's mass to the rounding of small
// terms.  The odd part c.u/3 uses a two-term 1/3: a single rounded 1/3 would scale the
// equilibrium momentum by (1 + 3e-8) at every collision, a bias that compounds over steps.
constexpr float kThirdHi = 1.0f / 3.0f;
constexpr float kThirdLo = (float)(1.0 / 3.0 - (double)kThirdHi);

__device__ __forceinline__ float third(float v) { return __builtin_fmaf(v, kThirdHi, v * kThirdLo); }

template <class Out>
__device__ __forceinline__ void relax_store(const float* f, float n, float ux, float uy, float c1,
                                            float om, const Out& out, int qbase) {
    const float usq6 = __builtin_fmaf(ux, ux, uy * uy) * (1.0f / 6.0f);
    const float up = ux + uy, um = uy - ux;
    const float ox = third(ux), oy = third(uy), op = third(up), oq = third(um);
    const float ex = __builtin_fmaf(0.5f * ux, ux, -usq6), ey = __builtin_fmaf(0.5f * uy, uy, -usq6);
    const float ep = __builtin_fmaf(0.5f * up, up, -usq6), eq = __builtin_fmaf(0.5f * um, um, -usq6);
    const float r = n * c1, r4 = 0.25f * r, n4 = 0.25f * n;
    float D[9];
    D[1] = __builtin_fmaf(n, ex + ox, r - f[1]);
    D[3] = __builtin_fmaf(n, ex - ox, r - f[3]);
    D[2] = __builtin_fmaf(n, ey + oy, r - f[2]);
    D[4] = __builtin_fmaf(n, ey - oy, r - f[4]);
    D[5] = __builtin_fmaf(n4, ep + op, r4 - f[5]);
    D[7] = __builtin_fmaf(n4, ep - op, r4 - f[7]);
    D[6] = __builtin_fmaf(n4, eq + oq, r4 - f[6]);
    D[8] = __builtin_fmaf(n4, eq - oq, r4 - f[8]);
    D[0] = -(((D[1] + D[2]) + (D[3] + D[4])) + ((D[5] + D[6]) + (D[7] + D[8])));
#pragma unroll
    for (int i = 0; i < 9; ++i) out(qbase + i, __builtin_fmaf(om, D[i], f[i]));
}

// Collide one fluid node: f holds its pulled populations (A then B), nA/nB their sums,
// sAx.. the weighted neighbour sums of n_A and n_B, swx/swy the weighted solid-neighbour sum.
template <class Out>
__device__ __forceinline__ void collide_store(const Chan& c, const float f[18], float nA, float nB,
                                              float sAx, float sAy, float sBx, float sBy, float swx,
                                              float swy, const Out& out) {
    const float jAx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const float jAy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
    const float jBx = (f[10] - f[12]) + (f[14] - f[15]) + (f[17] - f[16]);
    const float jBy = (f[11] - f[13]) + (f[14] - f[16]) + (f[15] - f[17]);
    // a_k = F_k / n_k: -G sum w n_kbar(x+c) c  -  G_kw sum w s(x+c) c
    const float aAx = __builtin_fmaf(-c.G, sBx, -(c.gw[0] * swx));
    const float aAy = __builtin_fmaf(-c.G, sBy, -(c.gw[0] * swy));
    const float aBx = __builtin_fmaf(-c.G, sAx, -(c.gw[1] * swx));
    const float aBy = __builtin_fmaf(-c.G, sAy, -(c.gw[1] * swy));
    const float den = __builtin_fmaf(c.wm[0], nA, c.wm[1] * nB);
    const float Ux = __builtin_fmaf(c.wm[0], jAx, c.wm[1] * jBx) / den;
    const float Uy = __builtin_fmaf(c.wm[0], jAy, c.wm[1] * jBy) / den;
    relax_store(f, nA, __builtin_fmaf(c.tm[0], aAx, Ux), __builtin_fmaf(c.tm[0], aAy, Uy), c.c1[0],
                c.omega[0], out, 0);
    relax_store(f + 9, nB, __builtin_fmaf(c.tm[1], aBx, Ux), __builtin_fmaf(c.tm[1], aBy, Uy),
                c.c1[1], c.omega[1], out, 9);
}

// ---------------------------------------------------------------------------------------------
// Fused step.  A block of BX threads owns a strip of BX columns and a chunk [yb, ye) of rows,
// walked row by row, upward or downward.  Iteration `it` pulls one row, writes its densities
// into a 4-slot LDS ring (plus the two halo columns, pulled by lanes 0 and 1), and after one
// barrier collides the previous row, whose populations were kept in registers.  The first and
// last rows pulled are density-only halos.  A slot written at iteration it+1 was last read by
// the collision of iteration it-1, which every thread finished before the barrier of iteration
// it, so one barrier per row suffices.
//
// Neighbouring chunks of a strip walk in opposite directions: all chunks start together, so
// the rows two chunks share are then pulled by both at about the same time and the second
// read hits in L2 instead of going back to HBM.
// ---------------------------------------------------------------------------------------------
template <int BX, bool MASK>
__global__ void __launch_bounds__(BX)
k_step_fused(const Chan* __restrict__ chans, const TileDesc* __restrict__ tiles, int ntiles,
             const int32_t* __restrict__ first, float* __restrict__ ws, int src) {
    __shared__ float sn[2][4][BX + 2];
    const int tid = threadIdx.x;
    // Tiles are taken in list order; the host orders the list for the XCD placement it wants
    // (blocks are dealt round-robin to the 8 XCDs).  Empty tiles pad such orders.  With a
    // persistent schedule block b takes the tiles [first[b], first[b+1]) instead.
    const int t_beg = first ? first[blockIdx.x] : (int)blockIdx.x;
    const int t_end = first ? first[blockIdx.x + 1] : ntiles;
    const int t_inc = first ? 1 : (int)gridDim.x;
    for (int t = t_beg; t < t_end; t += t_inc) {
        const TileDesc td = tiles[t];
        if (td.ye <= td.yb) continue;
        const Chan c = chans[td.chan];
        const bool down = td.down != 0;
        const int w = min(BX, c.nx - td.xb);
        const bool act = tid < w;
        const int x = td.xb + (act ? tid : w - 1);
        const int64_t buf_bytes = (int64_t)18 * c.plane * 4;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(ws + c.off + (int64_t)src * 18 * c.plane, buf_bytes);
        const __amdgpu_buffer_rsrc_t rd = make_rsrc(ws + c.off + (int64_t)(src ^ 1) * 18 * c.plane, buf_bytes);
        const uint32_t Pb = (uint32_t)(c.plane * 4);
        const int hx = tid == 0 ? (td.xb == 0 ? c.nx - 1 : td.xb - 1)
                                : (td.xb + w == c.nx ? 0 : td.xb + w);
        const int hslot = tid == 0 ? 0 : w + 1;
        float q[18];
#pragma unroll
        for (int i = 0; i < 18; ++i) q[i] = 0.0f;
        float qA = 0.0f, qB = 0.0f;
        uint32_t qcode = 0;
        // first row pulled: the halo below (upward walk) or above (downward walk) the chunk
        int y = down ? (td.ye == c.ny ? 0 : td.ye) : (td.yb == 0 ? c.ny - 1 : td.yb - 1);
        const int niter = td.ye - td.yb + 2;
        for (int it = 0; it < niter; ++it) {
            const int slot = it & 3;
            float p[18];
            const uint32_t code = pull_node_buf<MASK>(rs, Pb, c, ws, x, y, p);
            float nA = 0.0f, nB = 0.0f;
            if (!(code & 1u)) {
                nA = sum9(p);
                nB = sum9(p + 9);
            }
            if (act) {
                sn[0][slot][tid + 1] = nA;
                sn[1][slot][tid + 1] = nB;
            }
            if (tid < 2) {
                float h[18];
                const uint32_t hcode = pull_node_buf<MASK>(rs, Pb, c, ws, hx, y, h);
                float hA = 0.0f, hB = 0.0f;
                if (!(hcode & 1u)) {
                    hA = sum9(h);
                    hB = sum9(h + 9);
                }
                sn[0][slot][hslot] = hA;
                sn[1][slot][hslot] = hB;
            }
            __syncthreads();
            if (it >= 2 && act) {
                // the row collided now was pulled one iteration ago
                const int yc = down ? (y == c.ny - 1 ? 0 : y + 1) : (y == 0 ? c.ny - 1 : y - 1);
                if (!(qcode & 1u)) {
                    const int s0 = (it - 1) & 3;
                    const int sm = down ? slot : (it - 2) & 3;   // row yc - 1
                    const int sp = down ? (it - 2) & 3 : slot;   // row yc + 1
                    const int l = tid + 1;
                    const float AE = sn[0][s0][l + 1], AW = sn[0][s0][l - 1];
                    const float AN = sn[0][sp][l], AS = sn[0][sm][l];
                    const float ANE = sn[0][sp][l + 1], ANW = sn[0][sp][l - 1];
                    const float ASW = sn[0][sm][l - 1], ASE = sn[0][sm][l + 1];
                    const float BE = sn[1][s0][l + 1], BW = sn[1][s0][l - 1];
                    const float BN = sn[1][sp][l], BS = sn[1][sm][l];
                    const float BNE = sn[1][sp][l + 1], BNW = sn[1][sp][l - 1];
                    const float BSW = sn[1][sm][l - 1], BSE = sn[1][sm][l + 1];
                    const float sAx = link_sum(AE, AW, ANE, ASW, ASE, ANW);
                    const float sAy = link_sum(AN, AS, ANE, ASW, ANW, ASE);
                    const float sBx = link_sum(BE, BW, BNE, BSW, BSE, BNW);
                    const float sBy = link_sum(BN, BS, BNE, BSW, BNW, BSE);
                    float swx = 0.0f, swy = 0.0f;
                    if (qcode) wall_sum(qcode, swx, swy);
                    collide_store(c, q, qA, qB, sAx, sAy, sBx, sBy, swx, swy,
                                  BufferOut{rd, Pb, ((uint32_t)yc * (uint32_t)c.pitch + (uint32_t)x) * 4u});
                }
            }
#pragma unroll
            for (int i = 0; i < 18; ++i) q[i] = p[i];
            qA = nA;
            qB = nB;
            qcode = code;
            y = down ? (y == 0 ? c.ny - 1 : y - 1) : (y == c.ny - 1 ? 0 : y + 1);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Two time steps per pass (temporal blocking).  A block of BX lanes owns the output columns
// [xb, xb + w), w = the tile's width <= BX - 6, and rows [yb, ye); lane l holds column
// xb - 3 + l.  Stage 1 is the single step above, pulled on all w + 6 columns and collided on the
// w + 4 inner ones; its post-collision values f*(t) never leave the chip.  Stage 2 streams them:
// the x part by whole-wave lane shifts (DPP; the lanes at a wave's edge take their neighbour's
// values through LDS), the y part by keeping the shifted rows in registers; bounce-back uses the
// node's own unshifted f*(t).  Stage 2 then forms n(t+1) on the w + 2 columns around the output
// into a second density ring and collides the w output columns, storing f*(t+1).  Rows lag:
// iteration k pulls row yb-3+k, stage 1 collides row yb-4+k, stage 2 pulls row yb-5+k and
// collides and stores row yb-6+k.  Three barriers per row: after the stage-1 densities, after
// the edge values, after the stage-2 densities.  The pulled rows that wait one iteration for
// their collision (one per stage) wait in per-lane LDS slots rather than in registers (copying
// them between registers cost about a sixth of the loop's vector instructions), and the next
// row's loads are issued as soon as the current row is in its slot, a whole iteration ahead.
// Each node is computed with exactly the arithmetic of the single step, so two stages equal two
// single steps bit for bit.  LDS (12 KB per wave) holds the kernel to three waves per SIMD.
// ---------------------------------------------------------------------------------------------
struct RegOut {
    float* r;
    __device__ __forceinline__ void operator()(int q, float v) const { r[q] = v; }
};

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Whole-wave lane shifts: lane l receives the value of lane l - 1 (from_left) or l + 1
// (from_right); the lane without a source keeps its own value.  Every lane must be active.
__device__ __forceinline__ float lane_from_left(float v) {
    const int i = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(i, i, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_from_right(float v) {
    const int i = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(i, i, 0x130, 0xf, 0xf, false));
}

// Neighbour sums sum_i w_i n_k(x + c_i) c_i of both components at slot l of three density
// rows (m: y - 1, o: y, p: y + 1).
__device__ __forceinline__ void ring_sums(const float* Am, const float* Ao, const float* Ap,
                                          const float* Bm, const float* Bo, const float* Bp, int l,
                                          float& sAx, float& sAy, float& sBx, float& sBy) {
    sAx = link_sum(Ao[l + 1], Ao[l - 1], Ap[l + 1], Am[l - 1], Am[l + 1], Ap[l - 1]);
    sAy = link_sum(Ap[l], Am[l], Ap[l + 1], Am[l - 1], Ap[l - 1], Am[l + 1]);
    sBx = link_sum(Bo[l + 1], Bo[l - 1], Bp[l + 1], Bm[l - 1], Bm[l + 1], Bp[l - 1]);
    sBy = link_sum(Bp[l], Bm[l], Bp[l + 1], Bm[l - 1], Bp[l - 1], Bm[l + 1]);
}

template <int BX, bool MASK>
__global__ void __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_step_fused2(const Chan* __restrict__ chans, const TileDesc* __restrict__ tiles, int ntiles,
              const int32_t* __restrict__ first, float* __restrict__ ws, int src) {
    constexpr int NW = BX / 64;
    __shared__ float r1[2][3][BX];       // n(t)
    __shared__ float r2[2][3][BX];       // n(t + 1)
    __shared__ float eR[NW][6];          // lane 63 of each wave: f*_1, f*_5, f*_8 (A, B)
    __shared__ float eL[NW][6];          // lane 0 of each wave:  f*_3, f*_6, f*_7 (A, B)
    // rows awaiting collision, one slot per lane (each lane reads and writes only its own)
    __shared__ float sq[18][BX];         // stage 1: pulled populations of the previous row
    __shared__ float sq2[18][BX];        // stage 2: pulled populations of the previous row
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    // grid-stride over the list, or block b's own range [first[b], first[b+1]) (persistent)
    const int t_beg = first ? first[blockIdx.x] : (int)blockIdx.x;
    const int t_end = first ? first[blockIdx.x + 1] : ntiles;
    const int t_inc = first ? 1 : (int)gridDim.x;
    for (int t = t_beg; t < t_end; t += t_inc) {
        const TileDesc td = tiles[t];
        if (td.ye <= td.yb) continue;
        const Chan c = chans[td.chan];
        const int w = min(td.w, c.nx - td.xb);
        const bool in1 = tid < w + 6;                  // pulled columns xb - 3 .. xb + w + 2
        const bool c1 = tid >= 1 && tid < w + 5;       // stage-1 collisions
        const bool in2 = tid >= 3 && tid < w + 3;      // stage-2 collisions: the output columns
        const int x = wrap_mod(td.xb - 3 + min(tid, w + 5), c.nx);
        const int64_t buf_bytes = (int64_t)18 * c.plane * 4;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(ws + c.off + (int64_t)src * 18 * c.plane, buf_bytes);
        const __amdgpu_buffer_rsrc_t rd = make_rsrc(ws + c.off + (int64_t)(src ^ 1) * 18 * c.plane, buf_bytes);
        const uint32_t Pb = (uint32_t)(c.plane * 4);
        // stage 1: densities and code of the pulled row awaiting collision (its populations wait
        // in sq)
        float qA = 0.0f, qB = 0.0f;
        uint32_t qcode = 0;
        // stage 2: shifted f*(t) of the last two stage-1 rows (dirs 0,1,3,2,5,6 and 2,5,6 per
        // component), own unshifted f*(t) of the last row; the pulled row awaiting collision
        // waits in sq2
        float gm1[12], gm2[6], uf[14];   // uf: directions 1,3,4,5,6,7,8 per component
        float q2A = 0.0f, q2B = 0.0f;
        uint32_t q2code = 0;
#pragma unroll
        for (int i = 0; i < 14; ++i) uf[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 12; ++i) gm1[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) gm2[i] = 0.0f;
        const int niter = td.ye - td.yb + 6;
        // the stage-1 pull of row a + 1 is issued during iteration k as soon as row a is in its
        // slot, so that its latency overlaps the rest of the iteration
        float pn[18];
        uint32_t pcode = pull_node_buf<MASK>(rs, Pb, c, ws, x, wrap_mod(td.yb - 3, c.ny), pn);
        for (int k = 0; k < niter; ++k) {
            const int s0 = k % 3, s1 = (k + 2) % 3, s2 = (k + 1) % 3;   // iterations k, k-1, k-2
            // A: stage-1 pull of row a (issued one iteration ago), densities n(t) into r1
            const int a = wrap_mod(td.yb - 3 + k, c.ny);
            const uint32_t code = pcode;
            float nA = 0.0f, nB = 0.0f;
            if (!(code & 1u)) {
                nA = sum9(pn);
                nB = sum9(pn + 9);
            }
            // the previous row's populations out of the lane's slot, this row's in
            float q[18];
#pragma unroll
            for (int i = 0; i < 18; ++i) {
                q[i] = sq[i][tid];
                sq[i][tid] = pn[i];
            }
            if (in1) {
                r1[0][s0][tid] = nA;
                r1[1][s0][tid] = nB;
            }
            // the next row's stage-1 loads overlap the rest of the iteration
            if (k + 1 < niter) {
                const int an = a == c.ny - 1 ? 0 : a + 1;
                pcode = pull_node_buf<MASK>(rs, Pb, c, ws, x, an, pn);
            }
            __syncthreads();
            // B: stage-1 collision of row a - 1 into registers, then the x part of streaming
            float fs[18];
#pragma unroll
            for (int i = 0; i < 18; ++i) fs[i] = 0.0f;
            if (k >= 2 && c1 && !(qcode & 1u)) {
                float sAx, sAy, sBx, sBy;
                ring_sums(r1[0][s2], r1[0][s1], r1[0][s0], r1[1][s2], r1[1][s1], r1[1][s0], tid,
                          sAx, sAy, sBx, sBy);
                float swx = 0.0f, swy = 0.0f;
                if (qcode) wall_sum(qcode, swx, swy);
                collide_store(c, q, qA, qB, sAx, sAy, sBx, sBy, swx, swy, RegOut{fs});
            }
            float g[18];
#pragma unroll
            for (int o = 0; o < 18; o += 9) {
                g[o + 0] = fs[o + 0];
                g[o + 2] = fs[o + 2];
                g[o + 4] = fs[o + 4];
                g[o + 1] = lane_from_left(fs[o + 1]);
                g[o + 5] = lane_from_left(fs[o + 5]);
                g[o + 8] = lane_from_left(fs[o + 8]);
                g[o + 3] = lane_from_right(fs[o + 3]);
                g[o + 6] = lane_from_right(fs[o + 6]);
                g[o + 7] = lane_from_right(fs[o + 7]);
            }
            if (lane == 63) {
                eR[wv][0] = fs[1]; eR[wv][1] = fs[5]; eR[wv][2] = fs[8];
                eR[wv][3] = fs[10]; eR[wv][4] = fs[14]; eR[wv][5] = fs[17];
            }
            if (lane == 0) {
                eL[wv][0] = fs[3]; eL[wv][1] = fs[6]; eL[wv][2] = fs[7];
                eL[wv][3] = fs[12]; eL[wv][4] = fs[15]; eL[wv][5] = fs[16];
            }
            __syncthreads();
            if (lane == 0 && wv > 0) {
                g[1] = eR[wv - 1][0]; g[5] = eR[wv - 1][1]; g[8] = eR[wv - 1][2];
                g[10] = eR[wv - 1][3]; g[14] = eR[wv - 1][4]; g[17] = eR[wv - 1][5];
            }
            if (lane == 63 && wv < NW - 1) {
                g[3] = eL[wv + 1][0]; g[6] = eL[wv + 1][1]; g[7] = eL[wv + 1][2];
                g[12] = eL[wv + 1][3]; g[15] = eL[wv + 1][4]; g[16] = eL[wv + 1][5];
            }
            // C: stage-2 pull of row b = a - 2: directions 0,1,3 from row b, 2,5,6 from row
            // b - 1, 4,7,8 from row b + 1 (this iteration's shifted values)
            float f2[18];
            float n2A = 0.0f, n2B = 0.0f;
            uint32_t code2 = 0;
#pragma unroll
            for (int i = 0; i < 18; ++i) f2[i] = 0.0f;
            if (k >= 4) {
                const int b = wrap_mod(td.yb - 5 + k, c.ny);
                if (MASK && c.masked)
                    code2 = mask_code(c, ws, x, b);
                else if (near_wall(c, b))
                    code2 = rows_code(c, x, b);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int o = 9 * m;
                    f2[o + 0] = gm1[6 * m + 0];
                    f2[o + 1] = gm1[6 * m + 1];
                    f2[o + 3] = gm1[6 * m + 2];
                    f2[o + 2] = gm2[3 * m + 0];
                    f2[o + 5] = gm2[3 * m + 1];
                    f2[o + 6] = gm2[3 * m + 2];
                    f2[o + 4] = g[o + 4];
                    f2[o + 7] = g[o + 7];
                    f2[o + 8] = g[o + 8];
                }
                if (code2) {
                    // own unshifted f*(t) of row b: direction 2 is the unshifted gm1 entry, the
                    // others are kept in uf (slot of direction d: ufs[d])
                    const int ufs[9] = {-1, 0, -1, 1, 2, 3, 4, 5, 6};
#pragma unroll
                    for (int i = 1; i < 9; ++i)
                        if ((code2 >> opp[i]) & 1u) {
                            const int d = opp[i];
                            f2[i] = d == 2 ? gm1[3] : uf[ufs[d]];
                            f2[9 + i] = d == 2 ? gm1[9] : uf[7 + ufs[d]];
                        }
                }
                if (!(code2 & 1u)) {
                    n2A = sum9(f2);
                    n2B = sum9(f2 + 9);
                }
            }
            r2[0][s0][tid] = n2A;
            r2[1][s0][tid] = n2B;
            float q2[18];
#pragma unroll
            for (int i = 0; i < 18; ++i) {
                q2[i] = sq2[i][tid];
                sq2[i][tid] = f2[i];
            }
            __syncthreads();
            // D: stage-2 collision of row b - 1 (pulled one iteration ago), store f*(t + 1)
            if (k >= 6 && in2 && !(q2code & 1u)) {
                const int yc = wrap_mod(td.yb - 6 + k, c.ny);
                float sAx, sAy, sBx, sBy;
                ring_sums(r2[0][s2], r2[0][s1], r2[0][s0], r2[1][s2], r2[1][s1], r2[1][s0], tid,
                          sAx, sAy, sBx, sBy);
                float swx = 0.0f, swy = 0.0f;
                if (q2code) wall_sum(q2code, swx, swy);
                collide_store(c, q2, q2A, q2B, sAx, sAy, sBx, sBy, swx, swy,
                              BufferOutCached{rd, Pb, ((uint32_t)yc * (uint32_t)c.pitch + (uint32_t)x) * 4u});
            }
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                uf[7 * m + 0] = fs[9 * m + 1];
                uf[7 * m + 1] = fs[9 * m + 3];
                uf[7 * m + 2] = fs[9 * m + 4];
                uf[7 * m + 3] = fs[9 * m + 5];
                uf[7 * m + 4] = fs[9 * m + 6];
                uf[7 * m + 5] = fs[9 * m + 7];
                uf[7 * m + 6] = fs[9 * m + 8];
            }
            qA = nA;
            qB = nB;
            qcode = code;
            q2A = n2A;
            q2B = n2B;
            q2code = code2;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int o = 9 * m;
                gm2[3 * m + 0] = gm1[6 * m + 3];
                gm2[3 * m + 1] = gm1[6 * m + 4];
                gm2[3 * m + 2] = gm1[6 * m + 5];
                gm1[6 * m + 0] = g[o + 0];
                gm1[6 * m + 1] = g[o + 1];
                gm1[6 * m + 2] = g[o + 3];
                gm1[6 * m + 3] = g[o + 2];
                gm1[6 * m + 4] = g[o + 5];
                gm1[6 * m + 5] = g[o + 6];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Two-kernel step: (1) densities of every node into the density field, (2) pull, neighbour
// densities read back from the field, collision.  Same per-node arithmetic as the fused step.
// One block per row; threads stride along x.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kRowThreads)
k_density(const Chan* __restrict__ chans, const RowRef* __restrict__ rows, float* __restrict__ ws,
          int src) {
    const RowRef r = rows[blockIdx.x];
    const Chan c = chans[r.chan];
    const float* __restrict__ g = ws + c.off + (int64_t)src * 18 * c.plane;
    float* __restrict__ dn = ws + c.off + 36 * c.plane;
    for (int x = threadIdx.x; x < c.nx; x += kRowThreads) {
        float p[18];
        const uint32_t code = pull_node(g, c, ws, x, r.y, p);
        float nA = 0.0f, nB = 0.0f;
        if (!(code & 1u)) {
            nA = sum9(p);
            nB = sum9(p + 9);
        }
        dn[r.y * c.pitch + x] = nA;
        dn[c.plane + r.y * c.pitch + x] = nB;
    }
}

__global__ void __launch_bounds__(kRowThreads)
k_collide(const Chan* __restrict__ chans, const RowRef* __restrict__ rows, float* __restrict__ ws,
          int src) {
    const RowRef r = rows[blockIdx.x];
    const Chan c = chans[r.chan];
    const float* __restrict__ g = ws + c.off + (int64_t)src * 18 * c.plane;
    float* __restrict__ d = ws + c.off + (int64_t)(src ^ 1) * 18 * c.plane;
    const float* __restrict__ nA_f = ws + c.off + 36 * c.plane;
    const float* __restrict__ nB_f = nA_f + c.plane;
    const int y = r.y;
    if (!c.masked && c.x1 > c.x0 && (y == 0 || y == c.ny - 1) && c.x0 == 0 && c.x1 == c.nx) return;
    const int ym = dec_wrap(y, c.ny), yp = inc_wrap(y, c.ny);
    for (int x = threadIdx.x; x < c.nx; x += kRowThreads) {
        if (node_code(c, ws, x, y) & 1u) continue;
        float p[18];
        const uint32_t code = pull_node(g, c, ws, x, y, p);
        const float nA = sum9(p), nB = sum9(p + 9);
        const int xm = dec_wrap(x, c.nx), xp = inc_wrap(x, c.nx);
        const int r0 = y * c.pitch, rm = ym * c.pitch, rp = yp * c.pitch;
        const float AE = nA_f[r0 + xp], AW = nA_f[r0 + xm], AN = nA_f[rp + x], AS = nA_f[rm + x];
        const float ANE = nA_f[rp + xp], ANW = nA_f[rp + xm], ASW = nA_f[rm + xm], ASE = nA_f[rm + xp];
        const float BE = nB_f[r0 + xp], BW = nB_f[r0 + xm], BN = nB_f[rp + x], BS = nB_f[rm + x];
        const float BNE = nB_f[rp + xp], BNW = nB_f[rp + xm], BSW = nB_f[rm + xm], BSE = nB_f[rm + xp];
        const float sAx = link_sum(AE, AW, ANE, ASW, ASE, ANW);
        const float sAy = link_sum(AN, AS, ANE, ASW, ANW, ASE);
        const float sBx = link_sum(BE, BW, BNE, BSW, BSE, BNW);
        const float sBy = link_sum(BN, BS, BNE, BSW, BNW, BSE);
        float swx = 0.0f, swy = 0.0f;
        if (code) wall_sum(code, swx, swy);
        collide_store(c, p, nA, nB, sAx, sAy, sBx, sBy, swx, swy, GlobalOut{d, c.plane, r0 + x});
    }
}

// ---------------------------------------------------------------------------------------------
// Initial state.  The resident buffer holds post-collision values, so it is set to the
// populations that one pull turns into the rest equilibrium f_i = e_i n0(x) (e_0 = alpha,
// e_axis = (1-alpha)/5, e_diag = (1-alpha)/20): g_i(x) = e_i n0(x + c_i) if x + c_i is fluid,
// else e_i n0(x).  The FP64 host fields (rho_k, ny*nx) are staged in population buffer 1.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kRowThreads)
k_init(const Chan* __restrict__ chans, const RowRef* __restrict__ rows, float* __restrict__ ws) {
    const RowRef r = rows[blockIdx.x];
    const Chan c = chans[r.chan];
    const double* __restrict__ rho = reinterpret_cast<const double*>(ws + c.off + 18 * c.plane);
    float* __restrict__ g = ws + c.off;
    const int64_t P = c.plane;
    const int64_t cells = (int64_t)c.nx * c.ny;
    const int y = r.y;
    const int ym = dec_wrap(y, c.ny), yp = inc_wrap(y, c.ny);
    for (int x = threadIdx.x; x < c.nx; x += kRowThreads) {
        const int xm = dec_wrap(x, c.nx), xp = inc_wrap(x, c.nx);
        const int nxs[9] = {x, xp, x, xm, x, xp, xm, xm, xp};   // x + c_i
        const int nys[9] = {y, y, yp, y, ym, yp, yp, ym, ym};
        const uint32_t code = node_code(c, ws, x, y);
        const bool solid = code & 1u;
        const int idx = y * c.pitch + x;
        for (int k = 0; k < 2; ++k) {
            const double* rk = rho + k * cells;
            const double n0 = rk[(int64_t)y * c.nx + x] * (double)c.inv_m[k];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const float e = i == 0 ? c.c0[k] : (i < 5 ? c.c1[k] : 0.25f * c.c1[k]);
                double nn = n0;
                if (!((code >> i) & 1u))
                    nn = rk[(int64_t)nys[i] * c.nx + nxs[i]] * (double)c.inv_m[k];
                g[(k * 9 + i) * P + idx] = solid ? 0.0f : e * (float)nn;
            }
        }
    }
}

// Pulled populations f(t) of every node into buffer `1 - src`, layout [k][i][y][pitch].
__global__ void __launch_bounds__(kRowThreads)
k_pull_out(const Chan* __restrict__ chans, const RowRef* __restrict__ rows, float* __restrict__ ws,
           int src) {
    const RowRef r = rows[blockIdx.x];
    const Chan c = chans[r.chan];
    const float* __restrict__ g = ws + c.off + (int64_t)src * 18 * c.plane;
    float* __restrict__ o = ws + c.off + (int64_t)(src ^ 1) * 18 * c.plane;
    for (int x = threadIdx.x; x < c.nx; x += kRowThreads) {
        float p[18];
        const bool solid = pull_node(g, c, ws, x, r.y, p) & 1u;
#pragma unroll
        for (int i = 0; i < 18; ++i) o[i * c.plane + r.y * c.pitch + x] = solid ? 0.0f : p[i];
    }
}

// ---------------------------------------------------------------------------------------------
// Observables.  Pass 1 (one block per row): densities of the row into the density field,
// FP64 row sums of n_A and n_B over fluid nodes and a health flag.  Pass 2 (one block per
// channel): the row sums in fixed order, then the centre-line front and the wall-row film
// fronts by a parallel first-crossing search.  Both passes are deterministic.
// ---------------------------------------------------------------------------------------------
// Block reductions in a fixed order (results are bit-reproducible): a butterfly over the 64 lanes
// of each wave by cross-lane swaps, then the kRowThreads / 64 wave results through LDS, summed by
// every thread in wave order.  Two barriers per reduction.
constexpr int kRowWaves = kRowThreads / 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = scratch[0];
#pragma unroll
    for (int w = 1; w < kRowWaves; ++w) r += scratch[w];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int block_min(int v, int* scratch) {
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = scratch[0];
#pragma unroll
    for (int w = 1; w < kRowWaves; ++w) r = min(r, scratch[w]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kRowThreads)
k_obs_rows(const Chan* __restrict__ chans, const RowRef* __restrict__ rows, float* __restrict__ ws,
           int src, RowPartial* __restrict__ part) {
    __shared__ double sd[kRowWaves];
    __shared__ int si[kRowWaves];
    const RowRef r = rows[blockIdx.x];
    const Chan c = chans[r.chan];
    const float* __restrict__ g = ws + c.off + (int64_t)src * 18 * c.plane;
    float* __restrict__ dn = ws + c.off + 36 * c.plane;
    double mA = 0.0, mB = 0.0;
    int bad = 0;
    for (int x = threadIdx.x; x < c.nx; x += kRowThreads) {
        float p[18];
        const uint32_t code = pull_node(g, c, ws, x, r.y, p);
        float nA = 0.0f, nB = 0.0f;
        if (!(code & 1u)) {
            nA = sum9(p);
            nB = sum9(p + 9);
            mA += (double)nA;
            mB += (double)nB;
            if (!(nA >= -1e-3f) || !(nB >= -1e-3f) || !isfinite(nA) || !isfinite(nB)) bad = 1;
        }
        dn[r.y * c.pitch + x] = nA;
        dn[c.plane + r.y * c.pitch + x] = nB;
    }
    mA = block_sum(mA, sd);
    mB = block_sum(mB, sd);
    bad = block_sum(bad, si);
    if (threadIdx.x == 0) {
        RowPartial o;
        o.mass[0] = mA;
        o.mass[1] = mB;
        o.bad = bad;
        o.pad[0] = o.pad[1] = o.pad[2] = 0;
        part[c.row_base + r.y] = o;
    }
}

// Linear refinement of a first downward crossing at x (v(x) >= level > v(x+1)), minus x0.
__device__ __forceinline__ double refine(double vx, double vx1, int x, double level, int x0) {
    return (double)x + (vx - level) / (vx - vx1) - (double)x0;
}

__global__ void __launch_bounds__(kRowThreads)
k_obs_final(const Chan* __restrict__ chans, const float* __restrict__ ws,
            const RowPartial* __restrict__ part, ObsRec* __restrict__ now, ObsRec* __restrict__ ring,
            const int32_t* __restrict__ counter, int max_samples, int record) {
    __shared__ double sd[kRowWaves];
    __shared__ int si[kRowWaves];
    const int ch = blockIdx.x;
    const Chan c = chans[ch];
    const int tid = threadIdx.x;
    const float* __restrict__ nA = ws + c.off + 36 * c.plane;
    const float* __restrict__ nB = nA + c.plane;
    double mA = 0.0, mB = 0.0;
    int bad = 0;
    for (int y = tid; y < c.ny; y += kRowThreads) {
        const RowPartial p = part[c.row_base + y];
        mA += p.mass[0];
        mB += p.mass[1];
        bad |= p.bad;
    }
    mA = block_sum(mA, sd);
    mB = block_sum(mB, sd);
    bad = block_sum(bad, si);
    // centre line: rows ny/2-1 and ny/2 averaged (ny even) or row (ny-1)/2
    const bool even = (c.ny & 1) == 0;
    const int ra = even ? c.ny / 2 - 1 : (c.ny - 1) / 2;
    const int rb = even ? c.ny / 2 : ra;
    auto centre = [&](const float* f, int x) -> double {
        return even ? 0.5 * ((double)f[ra * c.pitch + x] + (double)f[rb * c.pitch + x])
                    : (double)f[ra * c.pitch + x];
    };
    auto phi = [&](int x) -> double { return centre(nA, x) - centre(nB, x); };
    const int big = 0x7fffffff;
    int xz = big;
    for (int x = c.xs + tid; x + 1 < c.nx; x += kRowThreads)
        if (xz == big && phi(x) >= 0.0 && phi(x + 1) < 0.0) xz = x;
    xz = block_min(xz, si);
    const double level = centre(nA, c.xs) / 3.0;
    const float* rowlo = nA + 1 * c.pitch;
    const float* rowhi = nA + (c.ny - 2) * c.pitch;
    int xlo = big, xhi = big;
    for (int x = c.xs + tid; x + 1 < c.nx; x += kRowThreads) {
        if (xlo == big && (double)rowlo[x] >= level && (double)rowlo[x + 1] < level) xlo = x;
        if (xhi == big && (double)rowhi[x] >= level && (double)rowhi[x + 1] < level) xhi = x;
    }
    xlo = block_min(xlo, si);
    xhi = block_min(xhi, si);
    if (tid == 0) {
        ObsRec o;
        o.t = 0;
        o.mass[0] = mA;
        o.mass[1] = mB;
        o.z = xz == big ? __builtin_nan("") : refine(phi(xz), phi(xz + 1), xz, 0.0, c.x0);
        o.precursor_lo = xlo == big ? __builtin_nan("")
                                    : refine(rowlo[xlo], rowlo[xlo + 1], xlo, level, c.x0);
        o.precursor_hi = xhi == big ? __builtin_nan("")
                                    : refine(rowhi[xhi], rowhi[xhi + 1], xhi, level, c.x0);
        o.precursor = 0.5 * (o.precursor_lo + o.precursor_hi);
        o.flags = (phi(c.xs) < 0.0 ? 1 : 0) | (bad ? 2 : 0);
        o.reserved = 0;
        now[ch] = o;
        if (record) {
            const int s = *counter;
            if (s < max_samples) ring[(int64_t)ch * max_samples + s] = o;
        }
    }
}

__global__ void k_bump(int32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = *counter + 1;
}

// grid: blocks of the launch; with `first` (persistent schedules) exactly `grid` blocks, each
// with its own tile range, otherwise min(grid, ntiles) blocks (all tiles when grid <= 0).
inline int grid_of(int grid, int ntiles, const int32_t* first) {
    if (first) return grid;
    return grid > 0 ? min(grid, ntiles) : ntiles;
}

template <int BX>
hipError_t launch_fused_bx(bool masked, const Chan* chans, const TileDesc* tiles, int ntiles,
                           const int32_t* first, int grid, float* ws, int src, hipStream_t s) {
    const int g = grid_of(grid, ntiles, first);
    if (g <= 0) return hipSuccess;
    if (masked)
        hipLaunchKernelGGL((k_step_fused<BX, true>), dim3(g), dim3(BX), 0, s, chans, tiles, ntiles, first, ws, src);
    else
        hipLaunchKernelGGL((k_step_fused<BX, false>), dim3(g), dim3(BX), 0, s, chans, tiles, ntiles, first, ws, src);
    return hipGetLastError();
}

template <int BX>
hipError_t launch_fused2_bx(bool masked, const Chan* chans, const TileDesc* tiles, int ntiles,
                            const int32_t* first, int grid, float* ws, int src, hipStream_t s) {
    const int g = grid_of(grid, ntiles, first);
    if (g <= 0) return hipSuccess;
    if (masked)
        hipLaunchKernelGGL((k_step_fused2<BX, true>), dim3(g), dim3(BX), 0, s, chans, tiles, ntiles, first, ws, src);
    else
        hipLaunchKernelGGL((k_step_fused2<BX, false>), dim3(g), dim3(BX), 0, s, chans, tiles, ntiles, first, ws, src);
    return hipGetLastError();
}

template <int BX>
int resident_bx(bool masked, int fuse) {
    int n = 0;
    hipError_t e;
    if (fuse == 2)
        e = masked ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_fused2<BX, true>, BX, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_fused2<BX, false>, BX, 0);
    else
        e = masked ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_fused<BX, true>, BX, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_fused<BX, false>, BX, 0);
    return e == hipSuccess ? n : 0;
}

// Solid-neighbourhood codes of masked channels from the staged uint8 mask (ny*nx bytes after
// the two FP64 fields in population buffer 1).  Row-walled channels are skipped.
__global__ void __launch_bounds__(kRowThreads)
k_codes(const Chan* __restrict__ chans, const RowRef* __restrict__ rows, float* __restrict__ ws) {
    const RowRef r = rows[blockIdx.x];
    const Chan c = chans[r.chan];
    if (!c.masked) return;
    const int64_t cells = (int64_t)c.nx * c.ny;
    const uint8_t* __restrict__ m =
        reinterpret_cast<const uint8_t*>(ws + c.off + 18 * c.plane) + 16 * cells;
    uint16_t* __restrict__ codes = reinterpret_cast<uint16_t*>(ws + c.moff);
    const int y = r.y;
    const int ym = dec_wrap(y, c.ny), yp = inc_wrap(y, c.ny);
    for (int x = threadIdx.x; x < c.nx; x += kRowThreads) {
        const int xm = dec_wrap(x, c.nx), xp = inc_wrap(x, c.nx);
        const int nxs[9] = {x, xp, x, xm, x, xp, xm, xm, xp};   // x + c_i
        const int nys[9] = {y, y, yp, y, ym, yp, yp, ym, ym};
        uint32_t code = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) code |= (uint32_t)(m[(int64_t)nys[i] * c.nx + nxs[i]] != 0) << i;
        codes[y * c.pitch + x] = (uint16_t)code;
    }
}

}  // namespace

hipError_t launch_init(const Chan* chans, const RowRef* rows, int nrows, float* ws, hipStream_t s) {
    hipLaunchKernelGGL(k_codes, dim3(nrows), dim3(kRowThreads), 0, s, chans, rows, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_init, dim3(nrows), dim3(kRowThreads), 0, s, chans, rows, ws);
    return hipGetLastError();
}

hipError_t launch_step_fused(int bx, bool masked, const Chan* chans, const TileDesc* tiles,
                             int ntiles, const int32_t* first, int grid, float* ws, int src,
                             hipStream_t s) {
    switch (bx) {
        case 64: return launch_fused_bx<64>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        case 128: return launch_fused_bx<128>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        case 256: return launch_fused_bx<256>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        case 512: return launch_fused_bx<512>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_fused2(int bx, bool masked, const Chan* chans, const TileDesc* tiles,
                              int ntiles, const int32_t* first, int grid, float* ws, int src,
                              hipStream_t s) {
    switch (bx) {
        case 64: return launch_fused2_bx<64>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        case 128: return launch_fused2_bx<128>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        case 256: return launch_fused2_bx<256>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        case 512: return launch_fused2_bx<512>(masked, chans, tiles, ntiles, first, grid, ws, src, s);
        default: return hipErrorInvalidValue;
    }
}

int resident_blocks_per_cu(int bx, bool masked, int fuse) {
    switch (bx) {
        case 64: return resident_bx<64>(masked, fuse);
        case 128: return resident_bx<128>(masked, fuse);
        case 256: return resident_bx<256>(masked, fuse);
        case 512: return resident_bx<512>(masked, fuse);
        default: return 0;
    }
}

hipError_t launch_step_two_kernel(const Chan* chans, const RowRef* rows, int nrows, float* ws,
                                  int src, hipStream_t s) {
    hipLaunchKernelGGL(k_density, dim3(nrows), dim3(kRowThreads), 0, s, chans, rows, ws, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_collide, dim3(nrows), dim3(kRowThreads), 0, s, chans, rows, ws, src);
    return hipGetLastError();
}

hipError_t launch_observe(const Chan* chans, const RowRef* rows, int nrows, int nchan, float* ws,
                          int src, RowPartial* partials, ObsRec* now, ObsRec* ring,
                          int32_t* counter, int max_samples, int record, hipStream_t s) {
    hipLaunchKernelGGL(k_obs_rows, dim3(nrows), dim3(kRowThreads), 0, s, chans, rows, ws, src,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_final, dim3(nchan), dim3(kRowThreads), 0, s, chans, ws, partials, now,
                       ring, counter, max_samples, record);
    e = hipGetLastError();
    if (e != hipSuccess || !record) return e;
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_pull_out(const Chan* chans, const RowRef* rows, int nrows, float* ws, int src,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_pull_out, dim3(nrows), dim3(kRowThreads), 0, s, chans, rows, ws, src);
    return hipGetLastError();
}

}  // namespace scf

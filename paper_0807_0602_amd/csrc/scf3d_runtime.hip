// Host runtime of the 3-D (D3Q19) capillary: the scf3_* entry points of include/scf.h.  Like
// the 2-D library it allocates no device memory: it carves the caller's workspace.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "scf.h"
#include "scf3d_internal.h"

namespace {

int fail(int code, const std::string& msg) { return scf::set_error(code, msg); }

#define HIP_TRY3(expr)                                                                 \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(SCF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan3 {
    size_t chan = 0, parts = 0, obs = 0, pop = 0, total = 0;
};

bool geom_ok(const scf3_geometry* g, std::string* why) {
    if (!g) { *why = "geometry is NULL"; return false; }
    // ny and nz index the launch grid's y and z dimensions (at most 65535 blocks)
    if (g->nx < 3 || g->ny < 3 || g->nz < 3 || g->nx >= (1 << 20) || g->ny > 65535 || g->nz > 65535) {
        *why = "need 3 <= nx < 2^20 and 3 <= ny, nz <= 65535";
        return false;
    }
    if (g->x0 < 0 || g->x1 < g->x0 || g->x1 > g->nx) { *why = "need 0 <= x0 <= x1 <= nx"; return false; }
    return true;
}

int pitch_of(int nx) { return (nx + 63) / 64 * 64; }

// The fused kernel addresses one component's 19 planes with unsigned 32-bit buffer offsets.
bool fused_fits(int64_t plane) { return (int64_t)19 * plane * (int64_t)sizeof(float) <= (int64_t)UINT32_MAX; }

Plan3 plan(const scf3_geometry& g) {
    Plan3 p;
    size_t off = 0;
    p.chan = off; off = align_up(off + sizeof(scf3::Chan3), 256);
    p.parts = off; off = align_up(off + sizeof(scf3::Part3) * (size_t)g.ny * g.nz, 256);
    p.obs = off; off = align_up(off + sizeof(scf3::Obs3), 256);
    p.pop = off;
    const size_t plane = (size_t)g.nz * g.ny * pitch_of(g.nx);
    off = align_up(off + sizeof(float) * 78 * plane, 256);   // 2 x 38 population planes + 2 density
    p.total = off;
    return p;
}

}  // namespace

struct scf3_ctx {
    scf3_geometry geom;
    scf_params prm;
    scf3::Chan3 chan;
    Plan3 lay;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;
    int64_t t = 0;
    int fused = 1, cy = 16;
    int32_t seen_flags = 0;   // flags of the last scf3_observe (see scf3_step)
    float* base() const { return reinterpret_cast<float*>(ws); }
    scf3::Chan3* d_chan() const { return reinterpret_cast<scf3::Chan3*>(ws + lay.chan); }
};

extern "C" {

size_t scf3_workspace_bytes(const scf3_geometry* geom) {
    std::string why;
    if (!geom_ok(geom, &why)) return 0;
    return plan(*geom).total;
}

int scf3_init(scf3_ctx** out, const scf3_geometry* geom, const scf_params* p, const double* rhoA,
              const double* rhoB, void* dev_ws, size_t ws_bytes, void* hip_stream) {
    if (!out) return fail(SCF_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!geom_ok(geom, &why)) return fail(SCF_EINVAL, why);
    if (!p) return fail(SCF_EINVAL, "params is NULL");
    for (int k = 0; k < 2; ++k) {
        if (!(p->tau[k] > 0.5) || !std::isfinite(p->tau[k])) return fail(SCF_EINVAL, "tau must be > 1/2");
        if (!(p->mass[k] > 0.0) || !std::isfinite(p->mass[k])) return fail(SCF_EINVAL, "mass must be > 0");
        if (std::fabs(p->alpha[k] - 4.0 / 9.0) > 1e-12)
            return fail(SCF_EINVAL, "the D3Q19 equilibrium has a fixed rest weight: alpha must be 4/9");
        if (!std::isfinite(p->gw[k])) return fail(SCF_EINVAL, "gw must be finite");
    }
    if (!std::isfinite(p->G)) return fail(SCF_EINVAL, "G must be finite");
    if (!rhoA || !rhoB) return fail(SCF_EINVAL, "density field is NULL");
    if (!dev_ws) return fail(SCF_EINVAL, "device workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ws) % 256) return fail(SCF_EINVAL, "workspace must be 256-byte aligned");
    const Plan3 lay = plan(*geom);
    if (ws_bytes < lay.total) return fail(SCF_EINVAL, "workspace too small: need " + std::to_string(lay.total) + " bytes");
    scf3_ctx* c = new (std::nothrow) scf3_ctx();
    if (!c) return fail(SCF_ENOMEM, "out of host memory");
    c->geom = *geom;
    c->prm = *p;
    c->lay = lay;
    c->ws = static_cast<char*>(dev_ws);
    c->stream = static_cast<hipStream_t>(hip_stream);
    scf3::Chan3& h = c->chan;
    std::memset(&h, 0, sizeof h);
    h.nx = geom->nx; h.ny = geom->ny; h.nz = geom->nz; h.pitch = pitch_of(geom->nx);
    h.x0 = geom->x0; h.x1 = geom->x1; h.walls_y = geom->walls_y ? 1 : 0; h.walls_z = geom->walls_z ? 1 : 0;
    h.off = (int64_t)(lay.pop / sizeof(float));
    h.plane = (int64_t)geom->nz * geom->ny * h.pitch;
    c->fused = fused_fits(h.plane) ? 1 : 0;
    h.G = (float)p->G;
    for (int k = 0; k < 2; ++k) {
        h.gw[k] = (float)p->gw[k];
        h.omega[k] = (float)(1.0 / p->tau[k]);
        h.tm[k] = (float)(p->tau[k] / p->mass[k]);
        h.wm[k] = (float)(p->mass[k] / p->tau[k]);
        h.inv_m[k] = (float)(1.0 / p->mass[k]);
    }
    auto cleanup = [&](int rc) { delete c; return rc; };
    const size_t cells = (size_t)geom->nx * geom->ny * geom->nz;
    char* stage = c->ws + lay.pop + sizeof(float) * 38 * (size_t)h.plane;
    hipError_t e = hipMemcpyAsync(c->d_chan(), &h, sizeof h, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(stage, rhoA, sizeof(double) * cells, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(stage + sizeof(double) * cells, rhoB, sizeof(double) * cells,
                                            hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = scf3::launch_init(h, c->d_chan(), c->base(), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return cleanup(fail(SCF_EDEVICE, std::string("scf3_init: ") + hipGetErrorString(e)));
    *out = c;
    return SCF_OK;
}

int scf3_step(scf3_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return fail(SCF_EINVAL, "bad context or negative step count");
    for (int64_t i = 0; i < nsteps; ++i) {
        if (c->fused)
            HIP_TRY3(scf3::launch_step_fused(c->chan, c->d_chan(), c->base(), c->cur, c->cy, c->stream));
        else
            HIP_TRY3(scf3::launch_step(c->chan, c->d_chan(), c->base(), c->cur, c->stream));
        c->cur ^= 1;
        c->t += 1;
    }
    if (c->seen_flags & 2)
        return fail(SCF_EUNSTABLE, "the last observation found a non-finite or negative density "
                                   "(the steps were still enqueued)");
    return SCF_OK;
}

int scf3_set_schedule(scf3_ctx* c, int32_t fused, int32_t cy) {
    if (!c) return fail(SCF_EINVAL, "context is NULL");
    if (fused != 0 && fused != 1) return fail(SCF_EINVAL, "fused must be 0 or 1");
    if (fused && cy < 1) return fail(SCF_EINVAL, "cy must be >= 1");
    if (fused && !fused_fits(c->chan.plane))
        return fail(SCF_EINVAL, "box too large for the fused kernel (19 planes above 4 GiB)");
    c->fused = fused;
    if (fused) c->cy = cy;
    return SCF_OK;
}

int scf3_get_schedule(const scf3_ctx* c, int32_t* fused, int32_t* cy) {
    if (!c || !fused || !cy) return fail(SCF_EINVAL, "NULL argument");
    *fused = c->fused;
    *cy = c->cy;
    return SCF_OK;
}

int scf3_observe(scf3_ctx* c, scf3_obs* out) {
    if (!c || !out) return fail(SCF_EINVAL, "NULL argument");
    auto* parts = reinterpret_cast<scf3::Part3*>(c->ws + c->lay.parts);
    auto* obs = reinterpret_cast<scf3::Obs3*>(c->ws + c->lay.obs);
    HIP_TRY3(scf3::launch_observe(c->chan, c->d_chan(), c->base(), c->cur, parts, obs, c->stream));
    scf3::Obs3 r;
    HIP_TRY3(hipMemcpyAsync(&r, obs, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY3(hipStreamSynchronize(c->stream));
    static_assert(sizeof(scf3::Obs3) == sizeof(scf3_obs), "record layout");
    std::memcpy(out, &r, sizeof r);
    out->t = c->t;
    c->seen_flags = out->flags;
    if (out->flags & 2) return fail(SCF_EUNSTABLE, "non-finite or negative density in the state");
    return SCF_OK;
}

int scf3_get_density(scf3_ctx* c, double* nA, double* nB) {
    if (!c || !nA || !nB) return fail(SCF_EINVAL, "NULL argument");
    scf3_obs o;
    int rc = scf3_observe(c, &o);   // also refreshes the density field
    if (rc && rc != SCF_EUNSTABLE) return rc;
    const scf3::Chan3& h = c->chan;
    std::vector<float> buf((size_t)2 * h.plane);
    HIP_TRY3(hipMemcpyAsync(buf.data(), c->base() + h.off + 76 * h.plane, sizeof(float) * buf.size(),
                            hipMemcpyDeviceToHost, c->stream));
    HIP_TRY3(hipStreamSynchronize(c->stream));
    for (int z = 0; z < h.nz; ++z)
        for (int y = 0; y < h.ny; ++y)
            for (int x = 0; x < h.nx; ++x) {
                const size_t src = ((size_t)z * h.ny + y) * h.pitch + x;
                const size_t dst = ((size_t)z * h.ny + y) * h.nx + x;
                nA[dst] = buf[src];
                nB[dst] = buf[h.plane + src];
            }
    return SCF_OK;
}

int scf3_get_populations(scf3_ctx* c, double* f) {
    if (!c || !f) return fail(SCF_EINVAL, "NULL argument");
    const scf3::Chan3& h = c->chan;
    HIP_TRY3(scf3::launch_pull_out(h, c->d_chan(), c->base(), c->cur, c->stream));
    std::vector<float> buf((size_t)38 * h.plane);
    HIP_TRY3(hipMemcpyAsync(buf.data(), c->base() + h.off + (size_t)(c->cur ^ 1) * 38 * h.plane,
                            sizeof(float) * buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY3(hipStreamSynchronize(c->stream));
    for (int q = 0; q < 38; ++q)
        for (int z = 0; z < h.nz; ++z)
            for (int y = 0; y < h.ny; ++y)
                for (int x = 0; x < h.nx; ++x)
                    f[(((size_t)q * h.nz + z) * h.ny + y) * h.nx + x] =
                        buf[(size_t)q * h.plane + ((size_t)z * h.ny + y) * h.pitch + x];
    return SCF_OK;
}

int64_t scf3_time(const scf3_ctx* c) { return c ? c->t : -1; }

void scf3_destroy(scf3_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"

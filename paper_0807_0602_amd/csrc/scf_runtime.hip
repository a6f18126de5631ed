// Host runtime of libscf: the C ABI of include/scf.h.
//
// One Engine serves both the single-channel context and the batch: a set of channels packed
// into the caller's device workspace, a tile list for the fused step, a row list for the
// per-row kernels, HIP graphs of captured step loops and the observation ring.  The library
// never allocates device memory; it only carves the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "scf.h"
#include "scf_internal.h"

namespace {

thread_local std::string g_err = "";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(SCF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int pitch_of(int nx) { return (nx + 63) / 64 * 64; }

constexpr int kMaxRowsPerGeom = 1 << 20;
// Persistent schedules: at most this many blocks per launch, and bands of at least kMinRange
// rows where a channel is taller (each band pays the pipeline's start-up rows once).
constexpr int kMaxPersistBlocks = 8192;
constexpr int kMinRange = 16;
// Version of the schedule space and kernels in the autotuner cache key (a cached schedule from
// another version is timed again).
constexpr int kTuneVersion = 5;
constexpr int kPlanesPerChannel = 38;   // 2 x 18 population planes + 2 density planes

// Float planes of one channel: populations and densities, plus one for the uint16 codes of a
// solid mask.
int planes_of(const scf_geometry& g) { return kPlanesPerChannel + (g.solid ? 1 : 0); }

// FNV-1a of the 0/1 solid mask (0 when the channel has none); identifies the geometry in
// checkpoints.
uint64_t mask_hash(const scf_geometry& g) {
    if (!g.solid) return 0;
    uint64_t h = 1469598103934665603ull;
    const size_t n = (size_t)g.nx * g.ny;
    for (size_t i = 0; i < n; ++i) {
        h ^= (uint64_t)(g.solid[i] != 0);
        h *= 1099511628211ull;
    }
    return h | 1;
}

bool geom_ok(const scf_geometry* g, std::string* why) {
    if (!g) { *why = "geometry is NULL"; return false; }
    if (g->nx < 3 || g->ny < 3 || g->nx >= kMaxRowsPerGeom || g->ny >= kMaxRowsPerGeom) {
        *why = "nx and ny must be in [3, 2^20)";
        return false;
    }
    if (g->x0 < 0 || g->x1 < g->x0 || g->x1 > g->nx) {
        *why = "need 0 <= x0 <= x1 <= nx";
        return false;
    }
    // one population buffer (18 planes of FP32) is addressed with unsigned 32-bit byte offsets
    if ((int64_t)18 * 4 * g->ny * pitch_of(g->nx) > (int64_t)std::numeric_limits<uint32_t>::max()) {
        *why = "ny * nx too large for one channel (18 planes must stay below 4 GiB)";
        return false;
    }
    return true;
}

bool params_ok(const scf_params* p, std::string* why) {
    if (!p) { *why = "params is NULL"; return false; }
    for (int k = 0; k < 2; ++k) {
        if (!(p->tau[k] > 0.5) || !std::isfinite(p->tau[k])) { *why = "tau must be > 1/2"; return false; }
        if (!(p->alpha[k] >= 0.0 && p->alpha[k] < 1.0)) { *why = "alpha must be in [0, 1)"; return false; }
        if (!(p->mass[k] > 0.0) || !std::isfinite(p->mass[k])) { *why = "mass must be > 0"; return false; }
        if (!std::isfinite(p->gw[k])) { *why = "gw must be finite"; return false; }
    }
    if (!std::isfinite(p->G)) { *why = "G must be finite"; return false; }
    return true;
}

struct Layout {
    size_t chans = 0, rows = 0, tiles = 0, first = 0, parts = 0, now = 0, ring = 0, counter = 0;
    std::vector<size_t> chan_off;   // byte offset of each channel's region
    size_t total = 0;
    int nrows = 0, max_tiles = 0;
};

// Most tiles one list can hold: 58-column strips (bx = 64 with two steps per pass), cy = 1.
int max_tiles_of(const scf_geometry& g) { return ((g.nx + 57) / 58) * g.ny; }

Layout plan(int nchan, const scf_geometry* g, int max_samples) {
    Layout L;
    size_t off = 0;
    L.chans = off; off = align_up(off + sizeof(scf::Chan) * nchan, 256);
    for (int c = 0; c < nchan; ++c) { L.nrows += g[c].ny; L.max_tiles += max_tiles_of(g[c]); }
    L.rows = off; off = align_up(off + sizeof(scf::RowRef) * L.nrows, 256);
    // padding of the XCD-contiguous order; a persistent schedule splits at most one range per
    // block at strip ends beyond the strips themselves
    L.max_tiles += 8 + kMaxPersistBlocks;
    // two lists: single-step tiles, then the two-step tiles; then each list's per-block offsets
    L.tiles = off; off = align_up(off + sizeof(scf::TileDesc) * 2 * (size_t)L.max_tiles, 256);
    L.first = off; off = align_up(off + sizeof(int32_t) * 2 * (size_t)(kMaxPersistBlocks + 1), 256);
    L.parts = off; off = align_up(off + sizeof(scf::RowPartial) * L.nrows, 256);
    L.now = off; off = align_up(off + sizeof(scf::ObsRec) * nchan, 256);
    L.ring = off; off = align_up(off + sizeof(scf::ObsRec) * (size_t)nchan * max_samples, 256);
    L.counter = off; off = align_up(off + 256, 256);
    for (int c = 0; c < nchan; ++c) {
        L.chan_off.push_back(off);
        off = align_up(off + sizeof(float) * planes_of(g[c]) * (size_t)g[c].ny * pitch_of(g[c].nx), 256);
    }
    L.total = off;
    return L;
}

scf::Chan make_chan(const scf_geometry& g, const scf_params& p, size_t byte_off, int row_base) {
    scf::Chan c;
    std::memset(&c, 0, sizeof c);
    c.nx = g.nx; c.ny = g.ny; c.pitch = pitch_of(g.nx); c.x0 = g.x0; c.x1 = g.x1; c.xs = g.x0 / 2;
    c.row_base = row_base;
    c.off = (int64_t)(byte_off / sizeof(float));
    c.plane = (int64_t)g.ny * c.pitch;
    c.masked = g.solid ? 1 : 0;
    c.moff = c.off + (int64_t)kPlanesPerChannel * c.plane;
    c.G = (float)p.G;
    for (int k = 0; k < 2; ++k) {
        c.gw[k] = (float)p.gw[k];
        c.omega[k] = (float)(1.0 / p.tau[k]);
        c.tm[k] = (float)(p.tau[k] / p.mass[k]);
        c.wm[k] = (float)(p.mass[k] / p.tau[k]);
        c.c1[k] = (float)((1.0 - p.alpha[k]) / 5.0);
        c.c0[k] = (float)p.alpha[k];
        c.inv_m[k] = (float)(1.0 / p.mass[k]);
    }
    return c;
}

}  // namespace

namespace scf {
// Error reporting shared with the surrogate runtime.
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace scf

struct Engine {
    int nchan = 0;
    std::vector<scf_geometry> geom;   // copies with the mask pointer cleared (masks are not kept)
    std::vector<uint64_t> mhash;      // mask_hash per channel
    bool any_masked = false;
    std::vector<scf_params> prm;
    std::vector<scf::Chan> chans;
    Layout lay;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;   // capture-only stream (nothing executes on it)
    int cur = 0;
    int64_t t = 0;
    int variant = SCF_VARIANT_FUSED;
    // default schedule: the one the autotuner picks for the 16384 x 1024 capillary (two steps
    // per launch, 256-wide blocks on 224-column strips, persistent strip-aligned bands dealt to
    // the XCDs in eighths)
    int bx = 256, cy = 16, order = SCF_ORDER_PERSIST | SCF_ORDER_XCD, graph_steps = 64, fuse = 2;
    int ntiles = 0, ntiles2 = 0;
    // blocks of the single-step and two-step launches under a persistent schedule (0: one
    // block per tile), and the device's compute units
    int grid1 = 0, grid2 = 0;
    int cus = 0;
    int bpc = 0;   // requested blocks per CU of persistent schedules (0: occupancy)
    float tuned_ms = 0.0f;   // time per step of the last autotuned schedule
    hipGraphExec_t g_steps[2] = {nullptr, nullptr};
    hipGraphExec_t g_sample[2] = {nullptr, nullptr};
    int sample_every = 0, max_samples = 1;
    int64_t recorded = 0;
    bool batch = false;
    // flags of the last observation copied to the host (scf_observe, scf_batch_observe); a
    // later step reports bit 1 as SCF_EUNSTABLE without synchronising
    int32_t seen_flags = 0;

    scf::Chan* d_chans() const { return reinterpret_cast<scf::Chan*>(ws + lay.chans); }
    scf::RowRef* d_rows() const { return reinterpret_cast<scf::RowRef*>(ws + lay.rows); }
    scf::TileDesc* d_tiles() const { return reinterpret_cast<scf::TileDesc*>(ws + lay.tiles); }
    scf::TileDesc* d_tiles2() const { return d_tiles() + lay.max_tiles; }
    int32_t* d_first() const { return reinterpret_cast<int32_t*>(ws + lay.first); }
    int32_t* d_first2() const { return d_first() + kMaxPersistBlocks + 1; }
    bool persistent() const { return (order & SCF_ORDER_PERSIST) != 0; }
    scf::RowPartial* d_parts() const { return reinterpret_cast<scf::RowPartial*>(ws + lay.parts); }
    scf::ObsRec* d_now() const { return reinterpret_cast<scf::ObsRec*>(ws + lay.now); }
    scf::ObsRec* d_ring() const { return reinterpret_cast<scf::ObsRec*>(ws + lay.ring); }
    int32_t* d_counter() const { return reinterpret_cast<int32_t*>(ws + lay.counter); }
    float* base() const { return reinterpret_cast<float*>(ws); }

    ~Engine() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
    }

    void drop_graphs() {
        for (int p = 0; p < 2; ++p) {
            if (g_steps[p]) (void)hipGraphExecDestroy(g_steps[p]);
            if (g_sample[p]) (void)hipGraphExecDestroy(g_sample[p]);
            g_steps[p] = g_sample[p] = nullptr;
        }
    }

    // Tiles of every channel in the requested order.  Within a strip, consecutive row chunks
    // alternate direction (see k_step_fused).  Blocks take tiles in list order and are dealt
    // round-robin to the 8 XCDs; with SCF_ORDER_XCD the list is permuted so that each XCD gets
    // a contiguous eighth of the base order (empty tiles pad the last round).
    std::vector<scf::TileDesc> make_tiles(int bxv, int cyv, int ord) const {
        // bxv is the strip width: bx for single steps, strip2(bx) for two steps per pass
        const bool bands = (ord & SCF_ORDER_BANDS) != 0;
        std::vector<scf::TileDesc> tl;
        for (int c = 0; c < nchan; ++c) {
            const scf_geometry& g = geom[c];
            const int chunk = std::min(cyv, g.ny);
            const int nstrip = (g.nx + bxv - 1) / bxv;
            const int nchunk = (g.ny + chunk - 1) / chunk;
            for (int a = 0; a < (bands ? nchunk : nstrip); ++a)
                for (int b = 0; b < (bands ? nstrip : nchunk); ++b) {
                    const int s_ = bands ? b : a;
                    const int k = bands ? a : b;
                    scf::TileDesc td;
                    std::memset(&td, 0, sizeof td);
                    td.chan = c;
                    td.xb = s_ * bxv;
                    td.yb = k * chunk;
                    td.ye = std::min(td.yb + chunk, g.ny);
                    td.down = k & 1;
                    td.w = bxv;
                    tl.push_back(td);
                }
        }
        if (!(ord & SCF_ORDER_XCD)) return tl;
        const int n = (int)tl.size();
        const int per = (n + 7) / 8;
        std::vector<scf::TileDesc> out((size_t)per * 8);
        for (int v = 0; v < per * 8; ++v) {
            const int t = (v & 7) * per + (v >> 3);
            if (t < n) {
                out[v] = tl[t];
            } else {
                std::memset(&out[v], 0, sizeof out[v]);   // empty tile (ye == yb)
            }
        }
        return out;
    }

    // (channel, band, strip) tiles over strips `stripw` wide, k_c = max(1, round(ny_c / target))
    // near-equal bands per channel, aligned across the channel's strips; odd bands walk downward.
    void band_tiles(int stripw, double target, std::vector<scf::TileDesc>& tl) const {
        tl.clear();
        for (int c = 0; c < nchan; ++c) {
            const int ny = geom[c].ny, ns = (geom[c].nx + stripw - 1) / stripw;
            const int k = std::max(1, (int)std::lround(ny / target));
            for (int j = 0; j < k; ++j)
                for (int s_ = 0; s_ < ns; ++s_) {
                    scf::TileDesc td;
                    std::memset(&td, 0, sizeof td);
                    td.chan = c;
                    td.xb = s_ * stripw;
                    td.yb = (int)((int64_t)j * ny / k);
                    td.ye = (int)((int64_t)(j + 1) * ny / k);
                    td.down = j & 1;
                    td.w = stripw;
                    tl.push_back(td);
                }
        }
    }

    // Cost of a tile in quarter rows: 4 per row it outputs plus `warm` for the pipeline's start-up
    // rows (2 for one step per pass, 6 for two; a start-up row does about a quarter of a row's
    // work).  Greedy packing of the list, in order and whole tiles only, into blocks of capacity
    // `cap`; returns the blocks used and, with `starts`, each block's first tile.
    static int64_t tile_cost(const scf::TileDesc& t, int warm) { return 4 * (int64_t)(t.ye - t.yb) + warm; }
    static int pack_tiles(const std::vector<scf::TileDesc>& tl, int64_t cap, int warm,
                          std::vector<int32_t>* starts) {
        int nb = 0;
        int64_t cur = cap + 1;
        for (size_t t = 0; t < tl.size(); ++t) {
            const int64_t w = tile_cost(tl[t], warm);
            if (cur + w > cap) {
                ++nb;
                cur = 0;
                if (starts) starts->push_back((int32_t)t);
            }
            cur += w;
        }
        return nb;
    }

    // Persistent schedule over strips `stripw` wide for `nblocks` blocks (one round: every block
    // resident at once).  Each block runs a contiguous run of the (channel, band, strip) list, so
    // horizontally adjacent tiles run at the same time and share the cache lines at their edges.
    // The runs are balanced by work, not by tile count: for a band height `target` (a geometric
    // grid from kMinRange to the tallest channel) every channel gets k_c = round(ny_c / target)
    // bands, the smallest block capacity that packs the list into nblocks runs is found by
    // bisection, and the target with the smallest capacity wins (ties: the taller bands).  A
    // single channel thus gets the tallest bands that give one tile per block; channels of
    // unequal height and length share the blocks by their rows.  With SCF_ORDER_XCD (nblocks a
    // multiple of 8) XCD x takes the x-th contiguous eighth of the runs, spread evenly over its
    // slots b = x, x + 8, ...  first[b] .. first[b+1] index block b's tiles.
    void make_tiles_persist(int stripw, int warm, int nblocks, int ord, std::vector<scf::TileDesc>& tl,
                            std::vector<int32_t>& first) const {
        int maxny = 1;
        for (int c = 0; c < nchan; ++c) maxny = std::max(maxny, geom[c].ny);
        auto min_cap = [&](const std::vector<scf::TileDesc>& t) {
            int64_t lo = 0, hi = 0;
            for (const scf::TileDesc& d : t) {
                lo = std::max(lo, tile_cost(d, warm));
                hi += tile_cost(d, warm);
            }
            hi = std::max(hi, lo);
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (pack_tiles(t, mid, warm, nullptr) <= nblocks) hi = mid; else lo = mid + 1;
            }
            return lo;
        };
        std::vector<scf::TileDesc> t0;
        int64_t best = -1;
        double best_target = maxny;
        for (double target = std::min(kMinRange, maxny);; target *= 1.04) {
            const double tg = std::min(target, (double)maxny);
            band_tiles(stripw, tg, t0);
            const int64_t c = min_cap(t0);
            if (best < 0 || c <= best) {
                best = c;
                best_target = tg;
            }
            if (tg >= maxny) break;
        }
        band_tiles(stripw, best_target, t0);
        std::vector<int32_t> starts;
        const int nb = pack_tiles(t0, best, warm, &starts);
        starts.push_back((int32_t)t0.size());
        // run j of the nb runs goes to block b; with the XCD order, XCD x's runs
        // [nb x / 8, nb (x + 1) / 8) are spread evenly over its nblocks / 8 slots
        const bool xcd = (ord & SCF_ORDER_XCD) && nblocks % 8 == 0;
        tl.clear();
        first.assign((size_t)nblocks + 1, 0);
        for (int b = 0; b < nblocks; ++b) {
            first[b] = (int32_t)tl.size();
            int64_t j0, j1;
            if (xcd) {
                const int x = b % 8, i = b / 8, per = nblocks / 8;
                const int64_t e0 = (int64_t)nb * x / 8, e1 = (int64_t)nb * (x + 1) / 8;
                j0 = e0 + (e1 - e0) * i / per;
                j1 = e0 + (e1 - e0) * (i + 1) / per;
            } else {
                j0 = (int64_t)nb * b / nblocks;
                j1 = (int64_t)nb * (b + 1) / nblocks;
            }
            for (int64_t j = j0; j < j1; ++j)
                for (int32_t t = starts[(size_t)j]; t < starts[(size_t)j + 1]; ++t) tl.push_back(t0[(size_t)t]);
        }
        first[nblocks] = (int32_t)tl.size();
    }

    // Blocks of a persistent launch: every CU filled to the kernel's occupancy (a multiple of 8
    // for the XCD order); 0 if the occupancy query fails.
    int persist_blocks(int bxv, int fz, int ord) const {
        const int occ = bpc > 0 ? bpc : scf::resident_blocks_per_cu(bxv, any_masked, fz);
        if (occ < 1 || cus < 1) return 0;
        int n = std::min(cus * occ, kMaxPersistBlocks);
        if ((ord & SCF_ORDER_XCD) && n >= 8) n -= n % 8;
        return n;
    }

    // Output columns per block of the two-step kernel: at most bx - 6 (its lanes pull three
    // extra columns each side); 480 for 512-wide and 224 for 256-wide blocks, so that strip edges
    // fall on 128-byte lines (measured faster although 26-32 lanes idle: a misaligned edge line
    // is read and written by two strips at different times); bx - 6 for narrower blocks.
    static int strip2(int bxv) { return bxv == 512 ? 480 : bxv == 256 ? 224 : bxv - 6; }

    int upload_tiles(int bxv, int cyv, int ord) {
        std::vector<scf::TileDesc> tl, tl2;
        std::vector<int32_t> f1, f2;
        int g1 = 0, g2 = 0;
        if (ord & SCF_ORDER_PERSIST) {
            g1 = persist_blocks(bxv, 1, ord);
            g2 = persist_blocks(bxv, 2, ord);
            if (!g1 || !g2) return fail(SCF_EDEVICE, "occupancy query for the persistent schedule failed");
            make_tiles_persist(bxv, 2, g1, ord, tl, f1);
            make_tiles_persist(strip2(bxv), 6, g2, ord, tl2, f2);
        } else {
            tl = make_tiles(bxv, cyv, ord);
            tl2 = make_tiles(strip2(bxv), cyv, ord);
        }
        if ((int)tl.size() > lay.max_tiles || (int)tl2.size() > lay.max_tiles)
            return fail(SCF_EINVAL, "tile list exceeds its reserved space");
        HIP_TRY(hipMemcpyAsync(d_tiles(), tl.data(), sizeof(scf::TileDesc) * tl.size(),
                               hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(d_tiles2(), tl2.data(), sizeof(scf::TileDesc) * tl2.size(),
                               hipMemcpyHostToDevice, stream));
        if (ord & SCF_ORDER_PERSIST) {
            HIP_TRY(hipMemcpyAsync(d_first(), f1.data(), sizeof(int32_t) * f1.size(), hipMemcpyHostToDevice, stream));
            HIP_TRY(hipMemcpyAsync(d_first2(), f2.data(), sizeof(int32_t) * f2.size(), hipMemcpyHostToDevice, stream));
        }
        HIP_TRY(hipStreamSynchronize(stream));
        ntiles = (int)tl.size();
        ntiles2 = (int)tl2.size();
        grid1 = g1;
        grid2 = g2;
        bx = bxv;
        cy = cyv;
        order = ord;
        return SCF_OK;
    }

    // Steps one launch advances from parity src (two with fuse = 2 when n >= 2 are left).
    int steps_of_launch(int64_t n) const {
        return (variant == SCF_VARIANT_FUSED && fuse == 2 && n >= 2) ? 2 : 1;
    }

    // One launch of `k` (1 or 2) steps reading buffer src and writing src ^ 1.
    hipError_t launch_steps(hipStream_t s, int src, int k) const {
        const bool p = persistent();
        if (k == 2)
            return scf::launch_step_fused2(bx, any_masked, d_chans(), d_tiles2(), ntiles2,
                                           p ? d_first2() : nullptr, grid2, base(), src, s);
        if (variant == SCF_VARIANT_TWO_KERNEL)
            return scf::launch_step_two_kernel(d_chans(), d_rows(), lay.nrows, base(), src, s);
        return scf::launch_step_fused(bx, any_masked, d_chans(), d_tiles(), ntiles, p ? d_first() : nullptr,
                                      grid1, base(), src, s);
    }

    // Launches that advance n steps (each flips the resident buffer once).
    int64_t launches_for(int64_t n) const {
        return (variant == SCF_VARIANT_FUSED && fuse == 2) ? n / 2 + (n & 1) : n;
    }

    hipError_t launch_obs(hipStream_t s, int record) const {
        return scf::launch_observe(d_chans(), d_rows(), lay.nrows, nchan, base(), cur,
                                   d_parts(), d_now(), d_ring(), d_counter(), max_samples, record, s);
    }

    // Capture `n` steps starting from parity p, optionally followed by a recorded observation.
    int capture(int p, int n, bool observe, hipGraphExec_t* out) {
        if (!cap) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
        hipError_t err = hipSuccess;
        int src = p;
        for (int64_t left = n; left > 0 && err == hipSuccess;) {
            const int k = steps_of_launch(left);
            err = launch_steps(cap, src, k);
            src ^= 1;
            left -= k;
        }
        if (err == hipSuccess && observe)
            err = scf::launch_observe(d_chans(), d_rows(), lay.nrows, nchan, base(), src, d_parts(),
                                      d_now(), d_ring(), d_counter(), max_samples, 1, cap);
        hipError_t end = hipStreamEndCapture(cap, &graph);
        if (err != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(SCF_EDEVICE, std::string("launch during capture: ") + hipGetErrorString(err));
        }
        if (end != hipSuccess) return fail(SCF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(end));
        hipError_t inst = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (inst != hipSuccess) return fail(SCF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(inst));
        return SCF_OK;
    }

    // Advance n steps with no observation.
    int advance(int64_t n) {
        while (n > 0) {
            if (graph_steps > 0 && n >= graph_steps) {
                if (!g_steps[cur]) {
                    int rc = capture(cur, graph_steps, false, &g_steps[cur]);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(g_steps[cur], stream));
                cur ^= (int)(launches_for(graph_steps) & 1);
                t += graph_steps;
                n -= graph_steps;
            } else {
                const int k = steps_of_launch(n);
                HIP_TRY(launch_steps(stream, cur, k));
                cur ^= 1;
                t += k;
                n -= k;
            }
        }
        return SCF_OK;
    }

    int observe_record() {
        HIP_TRY(scf::launch_observe(d_chans(), d_rows(), lay.nrows, nchan, base(), cur, d_parts(),
                                    d_now(), d_ring(), d_counter(), max_samples, 1, stream));
        recorded += 1;
        return SCF_OK;
    }

    // Advance n steps, recording every sample_every steps (batch mode).
    int advance_sampled(int64_t n) {
        const int S = sample_every;
        while (n > 0) {
            const int64_t phase = t % S;
            if (phase == 0 && n >= S && graph_steps > 0 && S <= 4096) {
                if (!g_sample[cur]) {
                    int rc = capture(cur, S, true, &g_sample[cur]);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(g_sample[cur], stream));
                cur ^= (int)(launches_for(S) & 1);
                t += S;
                n -= S;
                recorded += 1;
                continue;
            }
            const int64_t m = std::min<int64_t>(n, S - phase);
            int rc = advance(m);
            if (rc) return rc;
            n -= m;
            if (t % S == 0) {
                rc = observe_record();
                if (rc) return rc;
            }
        }
        return SCF_OK;
    }

    int setup(int nch, const scf_geometry* g, const scf_params* p, const double* const* rhoA,
              const double* const* rhoB, int samp_every, int max_samp, void* dev_ws, size_t bytes,
              void* s) {
        std::string why;
        if (nch < 1) return fail(SCF_EINVAL, "nchan must be >= 1");
        if (!dev_ws) return fail(SCF_EINVAL, "device workspace is NULL");
        if (reinterpret_cast<uintptr_t>(dev_ws) % 256) return fail(SCF_EINVAL, "workspace must be 256-byte aligned");
        for (int c = 0; c < nch; ++c) {
            if (!geom_ok(&g[c], &why)) return fail(SCF_EINVAL, "channel " + std::to_string(c) + ": " + why);
            if (!params_ok(&p[c], &why)) return fail(SCF_EINVAL, "channel " + std::to_string(c) + ": " + why);
            if (!rhoA || !rhoB || !rhoA[c] || !rhoB[c]) return fail(SCF_EINVAL, "density field is NULL");
        }
        if (max_samp < 1) return fail(SCF_EINVAL, "max_samples must be >= 1");
        {
            int dev = 0;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        }
        nchan = nch;
        geom.assign(g, g + nch);
        mhash.clear();
        any_masked = false;
        for (int c = 0; c < nch; ++c) {
            mhash.push_back(mask_hash(g[c]));
            any_masked = any_masked || g[c].solid != nullptr;
            geom[c].solid = nullptr;
        }
        prm.assign(p, p + nch);
        lay = plan(nch, g, max_samp);
        if (bytes < lay.total)
            return fail(SCF_EINVAL, "workspace too small: need " + std::to_string(lay.total) + " bytes");
        ws = static_cast<char*>(dev_ws);
        ws_bytes = bytes;
        stream = static_cast<hipStream_t>(s);
        sample_every = samp_every;
        max_samples = max_samp;
        std::vector<scf::RowRef> rows;
        int row_base = 0;
        for (int c = 0; c < nch; ++c) {
            chans.push_back(make_chan(g[c], p[c], lay.chan_off[c], row_base));
            for (int y = 0; y < g[c].ny; ++y) rows.push_back({c, y});
            row_base += g[c].ny;
        }
        HIP_TRY(hipMemcpyAsync(d_chans(), chans.data(), sizeof(scf::Chan) * nch, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(d_rows(), rows.data(), sizeof(scf::RowRef) * rows.size(), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemsetAsync(d_counter(), 0, 256, stream));
        // stage the FP64 fields (and the mask bytes) in population buffer 1 of each channel,
        // then build the mask codes and buffer 0
        for (int c = 0; c < nch; ++c) {
            const size_t cells = (size_t)g[c].nx * g[c].ny;
            char* stage = ws + lay.chan_off[c] + sizeof(float) * 18 * chans[c].plane;
            HIP_TRY(hipMemcpyAsync(stage, rhoA[c], sizeof(double) * cells, hipMemcpyHostToDevice, stream));
            HIP_TRY(hipMemcpyAsync(stage + sizeof(double) * cells, rhoB[c], sizeof(double) * cells,
                                   hipMemcpyHostToDevice, stream));
            if (g[c].solid)
                HIP_TRY(hipMemcpyAsync(stage + 2 * sizeof(double) * cells, g[c].solid, cells,
                                       hipMemcpyHostToDevice, stream));
        }
        HIP_TRY(scf::launch_init(d_chans(), d_rows(), lay.nrows, base(), stream));
        cur = 0;
        t = 0;
        int rc = upload_tiles(bx, cy, order);
        if (rc) return rc;
        if (sample_every > 0) {
            rc = observe_record();   // the t = 0 record
            if (rc) return rc;
        }
        HIP_TRY(hipStreamSynchronize(stream));
        return SCF_OK;
    }

    int set_tile(const scf_tile* tl) {
        if (!tl) return fail(SCF_EINVAL, "tile is NULL");
        if (tl->bx != 64 && tl->bx != 128 && tl->bx != 256 && tl->bx != 512)
            return fail(SCF_EINVAL, "bx must be 64, 128, 256 or 512");
        if (tl->cy < 1) return fail(SCF_EINVAL, "cy must be >= 1");
        if (tl->order < 0 || tl->order > (SCF_ORDER_BANDS | SCF_ORDER_XCD | SCF_ORDER_PERSIST))
            return fail(SCF_EINVAL, "unknown order");
        if (tl->graph_steps < 0) return fail(SCF_EINVAL, "graph_steps must be >= 0");
        if (tl->fuse != 1 && tl->fuse != 2) return fail(SCF_EINVAL, "fuse must be 1 or 2");
        if (tl->blocks_per_cu < 0 || tl->blocks_per_cu > 32) return fail(SCF_EINVAL, "blocks_per_cu must be in [0, 32]");
        HIP_TRY(hipStreamSynchronize(stream));
        drop_graphs();
        graph_steps = tl->graph_steps;
        fuse = tl->fuse;
        bpc = tl->blocks_per_cu;
        return upload_tiles(tl->bx, tl->cy, tl->order);
    }

    void get_tile(scf_tile* tl) const {
        tl->bx = bx;
        tl->cy = cy;
        tl->order = order;
        tl->graph_steps = graph_steps;
        tl->fuse = fuse;
        const int g = fuse == 2 ? grid2 : grid1;
        tl->blocks_per_cu = (persistent() && cus > 0) ? g / cus : 0;
    }

    // Time each candidate by repeated steps that all read the resident buffer and write the
    // idle one, so the state is never modified.
    int autotune(int trial, scf_tile* chosen) {
        if (trial < 1) return fail(SCF_EINVAL, "trial_steps must be >= 1");
        HIP_TRY(hipStreamSynchronize(stream));
        int maxny = 0;
        for (auto& g : geom) maxny = std::max(maxny, g.ny);
        const int bxs[4] = {64, 128, 256, 512};
        const int cys[10] = {4, 8, 16, 24, 32, 40, 48, 64, 128, 1 << 30};
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const int saved_variant = variant;
        variant = SCF_VARIANT_FUSED;
        bpc = 0;   // persistent candidates fill the CUs to the kernel's occupancy
        struct Cand { int bx, cy, ord, fuse; float ms; };   // ms per time step
        std::vector<Cand> cands;
        for (int ord = 0; ord < 4; ++ord)
            for (int bxv : bxs)
                for (int cyv : cys) {
                    if (cyv != (1 << 30) && cyv >= maxny) continue;
                    for (int k = 1; k <= 2; ++k) cands.push_back({bxv, cyv, ord, k, 0.0f});
                }
        // persistent schedules (range lengths follow from the occupancy, cy is not used)
        for (int ord : {(int)SCF_ORDER_PERSIST, (int)(SCF_ORDER_PERSIST | SCF_ORDER_XCD)})
            for (int bxv : bxs)
                for (int k = 1; k <= 2; ++k) cands.push_back({bxv, cy, ord, k, 0.0f});
        // time every candidate with `trial` launches, then the best eight again with four
        // times as many, and keep the fastest of the second round
        auto time_cand = [&](Cand& cd, int launches) -> int {
            int rc = upload_tiles(cd.bx, cd.cy, cd.ord);
            if (rc) return rc;
            for (int i = 0; i < 2; ++i) (void)launch_steps(stream, cur, cd.fuse);
            (void)hipEventRecord(e0, stream);
            for (int i = 0; i < launches; ++i) (void)launch_steps(stream, cur, cd.fuse);
            (void)hipEventRecord(e1, stream);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(SCF_EDEVICE, "autotune timing failed");
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            cd.ms = ms / (float)(launches * cd.fuse);
            return SCF_OK;
        };
        int rc = SCF_OK;
        for (Cand& cd : cands)
            if ((rc = time_cand(cd, trial))) break;
        if (!rc) {
            std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
            cands.resize(std::min<size_t>(cands.size(), 8));
            for (Cand& cd : cands)
                if ((rc = time_cand(cd, 4 * trial))) break;
            std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        variant = saved_variant;
        if (rc) return rc;
        drop_graphs();
        fuse = cands[0].fuse;
        tuned_ms = cands[0].ms;
        rc = upload_tiles(cands[0].bx, cands[0].cy, cands[0].ord);
        if (rc) return rc;
        if (chosen) get_tile(chosen);
        return SCF_OK;
    }

    // Key of the autotuner cache: the device (architecture name and compute units) and the
    // geometry class of the channels (sizes, wall extents, masks) in channel order, FNV-1a over
    // their values.  Schedules change only the order of work, so nothing else enters.
    uint64_t tune_key() const {
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](uint64_t v) {
            for (int i = 0; i < 8; ++i) {
                h ^= (v >> (8 * i)) & 0xffu;
                h *= 1099511628211ull;
            }
        };
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            for (const char* p = prop.gcnArchName; *p; ++p) mix((uint64_t)(unsigned char)*p);
        mix((uint64_t)kTuneVersion);
        mix((uint64_t)cus);
        mix((uint64_t)nchan);
        for (int c = 0; c < nchan; ++c) {
            mix((uint64_t)geom[c].nx);
            mix((uint64_t)geom[c].ny);
            mix((uint64_t)geom[c].x0);
            mix((uint64_t)geom[c].x1);
            mix(mhash[c]);
        }
        return h;
    }

    // autotune() with a cache file of lines "key bx cy order fuse blocks_per_cu ms_per_step":
    // a line with this context's key applies that schedule without timing; otherwise the
    // schedules are timed and the choice is appended.  The graph length is kept either way.
    int autotune_cached(int trial, const char* path, scf_tile* chosen) {
        if (!path) return autotune(trial, chosen);
        const uint64_t key = tune_key();
        if (FILE* f = std::fopen(path, "r")) {
            char line[256];
            bool found = false;
            scf_tile tl;
            while (std::fgets(line, sizeof line, f)) {
                unsigned long long k = 0;
                int v[5];
                float ms = 0.0f;
                if (std::sscanf(line, "%llx %d %d %d %d %d %f", &k, &v[0], &v[1], &v[2], &v[3], &v[4], &ms) == 7 &&
                    k == key) {
                    tl.bx = v[0]; tl.cy = v[1]; tl.order = v[2]; tl.fuse = v[3]; tl.blocks_per_cu = v[4];
                    found = true;   // the last matching line wins
                }
            }
            std::fclose(f);
            if (found) {
                tl.graph_steps = graph_steps;
                int rc = set_tile(&tl);
                if (rc) return rc;
                if (chosen) get_tile(chosen);
                return SCF_OK;
            }
        }
        int rc = autotune(trial, chosen);
        if (rc) return rc;
        FILE* f = std::fopen(path, "a");
        if (!f) return fail(SCF_EINVAL, std::string("autotuner cache not writable (schedule applied): ") + path);
        const bool ok = std::fprintf(f, "%016llx %d %d %d %d %d %.6f\n", (unsigned long long)key, bx, cy, order, fuse,
                                     bpc, tuned_ms) > 0;
        if (std::fclose(f) != 0 || !ok)
            return fail(SCF_EINVAL, std::string("autotuner cache write failed (schedule applied): ") + path);
        return SCF_OK;
    }

    int get_density(int c, double* nA, double* nB) {
        if (c < 0 || c >= nchan || !nA || !nB) return fail(SCF_EINVAL, "bad channel or NULL output");
        HIP_TRY(launch_obs(stream, 0));
        const scf_geometry& g = geom[c];
        const int pitch = chans[c].pitch;
        std::vector<float> h((size_t)2 * g.ny * pitch);
        HIP_TRY(hipMemcpyAsync(h.data(), ws + lay.chan_off[c] + sizeof(float) * 36 * chans[c].plane,
                               sizeof(float) * h.size(), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                nA[(size_t)y * g.nx + x] = h[(size_t)y * pitch + x];
                nB[(size_t)y * g.nx + x] = h[(size_t)(g.ny + y) * pitch + x];
            }
        return SCF_OK;
    }
};

struct scf_ctx { Engine e; };
struct scf_batch { Engine e; };

extern "C" {

const char* scf_last_error(void) { return g_err.c_str(); }

size_t scf_workspace_bytes(const scf_geometry* geom) {
    std::string why;
    if (!geom_ok(geom, &why)) return 0;
    return plan(1, geom, 1).total;
}

int scf_init(scf_ctx** out, const scf_geometry* geom, const scf_params* params, const double* rhoA,
             const double* rhoB, void* dev_ws, size_t ws_bytes, void* hip_stream) {
    if (!out) return fail(SCF_EINVAL, "out is NULL");
    *out = nullptr;
    scf_ctx* c = new (std::nothrow) scf_ctx();
    if (!c) return fail(SCF_ENOMEM, "out of host memory");
    const double* a[1] = {rhoA};
    const double* b[1] = {rhoB};
    int rc = c->e.setup(1, geom, params, a, b, 0, 1, dev_ws, ws_bytes, hip_stream);
    if (rc) { delete c; return rc; }
    *out = c;
    return SCF_OK;
}

// Instability found by the last observation, reported after the steps were enqueued.
static int lazy_unstable(const Engine& e) {
    if (e.seen_flags & 2)
        return fail(SCF_EUNSTABLE, "the last observation found a non-finite or negative density "
                                   "(the steps were still enqueued)");
    return SCF_OK;
}

int scf_step(scf_ctx* ctx, int64_t nsteps) {
    if (!ctx || nsteps < 0) return fail(SCF_EINVAL, "bad context or negative step count");
    int rc = ctx->e.advance(nsteps);
    return rc ? rc : lazy_unstable(ctx->e);
}

int scf_observe(scf_ctx* ctx, scf_obs* out) {
    if (!ctx || !out) return fail(SCF_EINVAL, "NULL argument");
    Engine& e = ctx->e;
    HIP_TRY(e.launch_obs(e.stream, 0));
    scf::ObsRec r;
    HIP_TRY(hipMemcpyAsync(&r, e.d_now(), sizeof r, hipMemcpyDeviceToHost, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    static_assert(sizeof(scf::ObsRec) == sizeof(scf_obs), "record layout");
    std::memcpy(out, &r, sizeof r);
    out->t = e.t;
    e.seen_flags = out->flags;
    if (out->flags & 2) return fail(SCF_EUNSTABLE, "non-finite or negative density in the state");
    return SCF_OK;
}

int scf_get_density(scf_ctx* ctx, double* nA, double* nB) {
    if (!ctx) return fail(SCF_EINVAL, "NULL context");
    return ctx->e.get_density(0, nA, nB);
}

int scf_get_populations(scf_ctx* ctx, double* f) {
    if (!ctx || !f) return fail(SCF_EINVAL, "NULL argument");
    Engine& e = ctx->e;
    HIP_TRY(scf::launch_pull_out(e.d_chans(), e.d_rows(), e.lay.nrows, e.base(), e.cur, e.stream));
    const scf_geometry& g = e.geom[0];
    const int pitch = e.chans[0].pitch;
    const int64_t P = e.chans[0].plane;
    std::vector<float> h((size_t)18 * P);
    HIP_TRY(hipMemcpyAsync(h.data(), e.ws + e.lay.chan_off[0] + sizeof(float) * (size_t)(e.cur ^ 1) * 18 * P,
                           sizeof(float) * h.size(), hipMemcpyDeviceToHost, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    for (int q = 0; q < 18; ++q)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x)
                f[((size_t)q * g.ny + y) * g.nx + x] = h[(size_t)q * P + (size_t)y * pitch + x];
    return SCF_OK;
}

int scf_set_variant(scf_ctx* ctx, int32_t variant) {
    if (!ctx) return fail(SCF_EINVAL, "NULL context");
    if (variant != SCF_VARIANT_FUSED && variant != SCF_VARIANT_TWO_KERNEL)
        return fail(SCF_EINVAL, "unknown variant");
    HIP_TRY(hipStreamSynchronize(ctx->e.stream));
    ctx->e.drop_graphs();
    ctx->e.variant = variant;
    return SCF_OK;
}

int scf_set_tile(scf_ctx* ctx, const scf_tile* tile) {
    if (!ctx) return fail(SCF_EINVAL, "NULL context");
    return ctx->e.set_tile(tile);
}

int scf_get_tile(const scf_ctx* ctx, scf_tile* tile) {
    if (!ctx || !tile) return fail(SCF_EINVAL, "NULL argument");
    ctx->e.get_tile(tile);
    return SCF_OK;
}

int scf_autotune(scf_ctx* ctx, int32_t trial_steps, scf_tile* chosen) {
    if (!ctx) return fail(SCF_EINVAL, "NULL context");
    return ctx->e.autotune(trial_steps, chosen);
}

int scf_autotune_cached(scf_ctx* ctx, int32_t trial_steps, const char* cache_path, scf_tile* chosen) {
    if (!ctx) return fail(SCF_EINVAL, "NULL context");
    return ctx->e.autotune_cached(trial_steps, cache_path, chosen);
}

int64_t scf_time(const scf_ctx* ctx) { return ctx ? ctx->e.t : -1; }

namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, nchan;
    int32_t nx, ny, x0, x1;
    uint64_t mask;   // mask_hash of the geometry
    scf_params params;
    int64_t t;
    int64_t floats;
};

bool same_geometry(const CkptHeader& h, const scf_geometry& g, uint64_t mhash) {
    return h.nx == g.nx && h.ny == g.ny && h.x0 == g.x0 && h.x1 == g.x1 && h.mask == mhash;
}
}  // namespace

int scf_save(scf_ctx* ctx, const char* path) {
    if (!ctx || !path) return fail(SCF_EINVAL, "NULL argument");
    Engine& e = ctx->e;
    CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "SCFCKPT2", 8);
    h.version = 2;
    h.nchan = 1;
    h.nx = e.geom[0].nx;
    h.ny = e.geom[0].ny;
    h.x0 = e.geom[0].x0;
    h.x1 = e.geom[0].x1;
    h.mask = e.mhash[0];
    h.params = e.prm[0];
    h.t = e.t;
    h.floats = 18 * e.chans[0].plane;
    std::vector<float> buf((size_t)h.floats);
    HIP_TRY(hipMemcpyAsync(buf.data(), e.ws + e.lay.chan_off[0] + sizeof(float) * (size_t)e.cur * 18 * e.chans[0].plane,
                           sizeof(float) * buf.size(), hipMemcpyDeviceToHost, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SCF_EINVAL, std::string("cannot open ") + path);
    bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SCF_OK : fail(SCF_ESTATE, std::string("write failed: ") + path);
}

int scf_load(scf_ctx* ctx, const char* path) {
    if (!ctx || !path) return fail(SCF_EINVAL, "NULL argument");
    Engine& e = ctx->e;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SCF_EINVAL, std::string("cannot open ") + path);
    CkptHeader h;
    bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, "SCFCKPT2", 8) == 0 &&
              h.version == 2 && h.nchan == 1 && same_geometry(h, e.geom[0], e.mhash[0]) &&
              std::memcmp(&h.params, &e.prm[0], sizeof h.params) == 0 &&
              h.floats == 18 * e.chans[0].plane;
    std::vector<float> buf;
    if (ok) {
        buf.resize((size_t)h.floats);
        ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    }
    std::fclose(f);
    if (!ok) return fail(SCF_ESTATE, std::string("checkpoint does not match this context: ") + path);
    HIP_TRY(hipStreamSynchronize(e.stream));
    HIP_TRY(hipMemcpyAsync(e.ws + e.lay.chan_off[0] + sizeof(float) * (size_t)e.cur * 18 * e.chans[0].plane,
                           buf.data(), sizeof(float) * buf.size(), hipMemcpyHostToDevice, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    e.t = h.t;
    return SCF_OK;
}

void scf_destroy(scf_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->e.stream);
    delete ctx;
}

size_t scf_batch_workspace_bytes(int32_t nchan, const scf_geometry* geoms, int32_t max_samples) {
    if (nchan < 1 || !geoms || max_samples < 1) return 0;
    std::string why;
    for (int c = 0; c < nchan; ++c)
        if (!geom_ok(&geoms[c], &why)) return 0;
    return plan(nchan, geoms, max_samples).total;
}

int scf_batch_init(scf_batch** out, int32_t nchan, const scf_geometry* geoms, const scf_params* params,
                   const double* const* rhoA, const double* const* rhoB, int32_t sample_every,
                   int32_t max_samples, void* dev_ws, size_t ws_bytes, void* hip_stream) {
    if (!out) return fail(SCF_EINVAL, "out is NULL");
    *out = nullptr;
    if (sample_every < 1) return fail(SCF_EINVAL, "sample_every must be >= 1");
    if (!geoms || !params) return fail(SCF_EINVAL, "NULL geometry or params");
    scf_batch* b = new (std::nothrow) scf_batch();
    if (!b) return fail(SCF_ENOMEM, "out of host memory");
    b->e.batch = true;
    int rc = b->e.setup(nchan, geoms, params, rhoA, rhoB, sample_every, max_samples, dev_ws, ws_bytes,
                        hip_stream);
    if (rc) { delete b; return rc; }
    *out = b;
    return SCF_OK;
}

int scf_batch_step(scf_batch* b, int64_t nsteps) {
    if (!b || nsteps < 0) return fail(SCF_EINVAL, "bad batch or negative step count");
    int rc = b->e.advance_sampled(nsteps);
    return rc ? rc : lazy_unstable(b->e);
}

int scf_batch_observe(scf_batch* b, scf_obs* out, int64_t* nsamples) {
    if (!b || !out || !nsamples) return fail(SCF_EINVAL, "NULL argument");
    Engine& e = b->e;
    const size_t n = (size_t)e.nchan * e.max_samples;
    std::vector<scf::ObsRec> h(n);
    HIP_TRY(hipMemcpyAsync(h.data(), e.d_ring(), sizeof(scf::ObsRec) * n, hipMemcpyDeviceToHost, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    const int64_t have = std::min<int64_t>(e.recorded, e.max_samples);
    bool unstable = false;
    for (int c = 0; c < e.nchan; ++c)
        for (int64_t s = 0; s < e.max_samples; ++s) {
            scf_obs& o = out[(size_t)c * e.max_samples + s];
            std::memcpy(&o, &h[(size_t)c * e.max_samples + s], sizeof o);
            if (s < have) {
                o.t = s * (int64_t)e.sample_every;
                if (o.flags & 2) unstable = true;
            } else {
                std::memset(&o, 0, sizeof o);
                o.t = -1;
            }
        }
    *nsamples = have;
    e.seen_flags = unstable ? 2 : 0;
    if (unstable) return fail(SCF_EUNSTABLE, "a recorded sample holds a non-finite or negative density");
    return SCF_OK;
}

int scf_batch_get_density(scf_batch* b, int32_t c, double* nA, double* nB) {
    if (!b) return fail(SCF_EINVAL, "NULL batch");
    return b->e.get_density(c, nA, nB);
}

int scf_batch_set_tile(scf_batch* b, const scf_tile* tile) {
    if (!b) return fail(SCF_EINVAL, "NULL batch");
    return b->e.set_tile(tile);
}

int scf_batch_get_tile(const scf_batch* b, scf_tile* tile) {
    if (!b || !tile) return fail(SCF_EINVAL, "NULL argument");
    b->e.get_tile(tile);
    return SCF_OK;
}

int scf_batch_autotune(scf_batch* b, int32_t trial_steps, scf_tile* chosen) {
    if (!b) return fail(SCF_EINVAL, "NULL batch");
    return b->e.autotune(trial_steps, chosen);
}

int scf_batch_autotune_cached(scf_batch* b, int32_t trial_steps, const char* cache_path, scf_tile* chosen) {
    if (!b) return fail(SCF_EINVAL, "NULL batch");
    return b->e.autotune_cached(trial_steps, cache_path, chosen);
}

void scf_batch_destroy(scf_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->e.stream);
    delete b;
}

}  // extern "C"

// tt_api.hip -- C ABI of libtt (declared in include/tt.h): host-side argument
// checks, workspace layout, and the iteration loop that polls convergence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tt_internal.h"

namespace {
thread_local std::string g_err;
}  // namespace

namespace tt {
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace tt

namespace {
using tt::fail;

// Device scratch of tt_forward_noalloc: the workspace of a forward solve for
// callers that cannot allocate.  Each device holds its own copy from the
// moment the library's code is loaded on it until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): its device address comes from
// hipGetSymbolAddress, once per device (scratch_ptr below).
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

#define TT_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(TT_EHIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// default tile k-extents (the forward update is long, so shorter tiles with
// more parallel tiles per plane win; the adjoint step is short, so longer
// tiles amortise the staging better); measured on the 101^3 spherical batch
constexpr int kDefaultTileK = 32;
constexpr int kDefaultTileKFwd = 16;
constexpr int kDefaultTileKAdj = 28;

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

int check_grid(const tt_grid* g) {
    if (!g) return fail(TT_EINVAL, "grid is NULL");
    if (g->coord != 0 && g->coord != 1) return fail(TT_EINVAL, "grid.coord must be 0 or 1");
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 4) return fail(TT_EINVAL, "grid.n[%d] = %d < 4", a, g->n[a]);
        if (g->n[a] > 8192) return fail(TT_EINVAL, "grid.n[%d] = %d > 8192", a, g->n[a]);
        if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a])) return fail(TT_EINVAL, "grid.h[%d] must be > 0", a);
        if (!std::isfinite(g->o[a])) return fail(TT_EINVAL, "grid.o[%d] not finite", a);
    }
    // per-node records are addressed with 32-bit indices within one layout of
    // n0 (n1 + n2 - 1) n1p records, n1p the row pitch (n1 + 7 rounded up to 8)
    const double n1p = (double)((g->n[1] + 14) / 8 * 8);
    if ((double)g->n[0] * (g->n[1] + g->n[2] - 1) * n1p >= 2147483647.0)
        return fail(TT_EINVAL, "grid too large: n0 * (n1 + n2 - 1) * n1p must stay below 2^31");
    if (g->coord == 1) {
        double rmin = g->o[0];
        if (!(rmin > 0.0)) return fail(TT_EINVAL, "spherical grid needs r > 0");
        double lat0 = g->o[1], lat1 = g->o[1] + (g->n[1] - 1) * g->h[1];
        const double lim = 1.5533;  // 89 degrees
        if (std::fabs(lat0) > lim || std::fabs(lat1) > lim)
            return fail(TT_EINVAL, "spherical grid latitude must stay within +-89 degrees");
    }
    return TT_OK;
}

int check_opts(const tt_opts* o) {
    if (!o) return fail(TT_EINVAL, "opts is NULL");
    if (!(o->tol > 0.0)) return fail(TT_EINVAL, "opts.tol must be > 0");
    if (o->max_iter < 1) return fail(TT_EINVAL, "opts.max_iter must be >= 1");
    if (!(o->kappa > 0.0) || !std::isfinite(o->kappa)) return fail(TT_EINVAL, "opts.kappa must be > 0");
    if (o->tile_k < 0 || o->tile_k > tt::kMaxTileK)
        return fail(TT_EINVAL, "opts.tile_k must be in [0, %d]", tt::kMaxTileK);
    if (o->groups < 0 || o->groups > TT_MAX_GROUPS)
        return fail(TT_EINVAL, "opts.groups must be in [0, %d]", TT_MAX_GROUPS);
    return TT_OK;
}

// number of concurrently iterated source groups of a solve
int groups_of(const tt_opts* o, int nsrc) {
    int g;
    if (o && (o->flags & TT_FLAG_TIME_SWEEPS))
        g = 1;
    else if (o && o->groups > 0)
        g = o->groups;
    else
        g = nsrc / 32 < 1 ? 1 : (nsrc / 32 > 4 ? 4 : nsrc / 32);
    return g > nsrc ? nsrc : g;
}

// first source of group q of G
int group_begin(int nsrc, int G, int q) { return (int)(((long long)nsrc * q) / G); }

tt::Geo make_geo(const tt_grid* g, int tk) {
    tt::Geo G;
    std::memset(&G, 0, sizeof G);
    for (int a = 0; a < 3; ++a) {
        G.n[a] = g->n[a];
        G.m[a] = g->n[a] - 2;
        G.o[a] = g->o[a];
        G.h[a] = g->h[a];
        G.inv2h[a] = 1.0 / (2.0 * g->h[a]);
        G.invh[a] = 1.0 / g->h[a];
    }
    G.coord = g->coord;
    G.tk = tk;
    G.nt[0] = (G.m[0] + tt::kBI - 1) / tt::kBI;
    G.nt[1] = (G.m[1] + tt::kBJ - 1) / tt::kBJ;
    G.nt[2] = 0;
    for (int sd = 0; sd <= G.nt[0] + G.nt[1] - 2; ++sd) {
        const int c = tt::col_tile_hi(G, sd) - tt::col_tile_lo(G, sd) + 1;
        G.nt[2] = c > G.nt[2] ? c : G.nt[2];
    }
    G.ntiles = G.nt[0] * G.nt[1] * G.nt[2];
    G.N = (long long)G.n[0] * G.n[1] * G.n[2];
    G.si = (long long)G.n[1] * G.n[2];
    G.sj = G.n[2];
    G.NB = G.N - (long long)G.m[0] * G.m[1] * G.m[2];
    G.W = G.n[1] + G.n[2] - 1;
    // adjoint layouts: a tile row's 8 records start on a multiple of 8 records
    // (three 128-byte lines of 48-byte records) for either sign of the j sweep
    G.n1p = (G.n[1] + 7 + 7) / 8 * 8;
    G.joff[0] = 7;
    G.joff[1] = ((9 - G.n[1]) % 8 + 8) % 8;
    G.Sa = (long long)G.n[0] * G.W * G.n1p;
    return G;
}

// Workspace layout (each region 256-byte aligned):
//   Src[nsrc] | tab0[n0] | tab1[n1] | tab2[n2] | active[nsrc] | iter[nsrc] | counter |
//   part[nsrc*nslots] | model[4*Sa*4] (forward) | part2[nsrc*nslots] (adjoint) |
//   coef[nsrc*4*Sa*6] (or [nsrc*N*6] compact) | diag[nsrc*N] | rhs[nsrc*N] | box[nsrc*6] | bnd_in, bnd_rhs[nsrc*NB] (adjoint)
struct Layout {
    size_t off_src, off_t0, off_t1, off_t2, off_active, off_iter, off_counter, off_part, off_part2, off_coef,
        off_diag, off_rhs, off_box, off_bnd, off_model, total;
};

Layout layout(const tt::Geo& G, int nsrc, int nslots, int which, bool compact = false) {
    Layout L;
    size_t o = 0;
    L.off_src = o; o = align_up(o + sizeof(tt::Src) * (size_t)nsrc);
    L.off_t0 = o; o = align_up(o + sizeof(double) * (size_t)G.n[0]);
    L.off_t1 = o; o = align_up(o + sizeof(double2) * (size_t)G.n[1]);
    L.off_t2 = o; o = align_up(o + sizeof(double2) * (size_t)G.n[2]);
    L.off_active = o; o = align_up(o + sizeof(int) * (size_t)nsrc);
    L.off_iter = o; o = align_up(o + sizeof(int) * (size_t)nsrc);
    L.off_counter = o; o = align_up(o + sizeof(int));
    L.off_part = o;
    L.off_part2 = o;
    L.off_coef = o;
    L.off_diag = o;
    L.off_rhs = o;
    L.off_box = o;
    L.off_bnd = o;
    L.off_model = o;
    if (which == 0 || which == 1) {
        L.off_part = o; o = align_up(o + sizeof(double) * (size_t)nsrc * nslots);
    }
    if (which == 0) {
        L.off_model = o; o = align_up(o + sizeof(double) * 4 * 4 * (size_t)G.Sa);
    }
    if (which == 1) {
        L.off_part2 = o; o = align_up(o + sizeof(double) * (size_t)nsrc * nslots);
        L.off_coef = o;
        o = align_up(o + sizeof(double) * 6 * (size_t)nsrc * (compact ? (size_t)G.N : 4 * (size_t)G.Sa));
        L.off_diag = o; o = align_up(o + sizeof(double) * (size_t)nsrc * (size_t)G.N);
        L.off_rhs = o; o = align_up(o + sizeof(double) * (size_t)nsrc * (size_t)G.N);
        L.off_box = o; o = align_up(o + sizeof(int) * 6 * (size_t)nsrc);
        L.off_bnd = o; o = align_up(o + sizeof(double) * 2 * (size_t)nsrc * (size_t)G.NB);  // bnd_in, bnd_rhs
    }
    L.total = o;
    return L;
}

void fill_plan(tt::Plan& P, const tt::Geo& G, int nsrc) {
    P.G = G;
    P.nsrc = nsrc;
    // tile-plane p holds the tiles (TI, TJ, p - s) of the tile columns with
    // s = TI + TJ and lo(s) <= p - s <= hi(s); s + lo(s) and s + hi(s) grow with
    // s, so those s form one run
    const int smax = G.nt[0] + G.nt[1] - 2;
    const int pmax = smax + tt::col_tile_hi(G, smax);
    P.plane_count.clear();
    P.plane_id.clear();
    P.plane_s0.clear();
    for (int p = 0; p <= pmax; ++p) {
        int cnt = 0, s0 = -1;
        for (int sd = 0; sd <= smax; ++sd) {
            if (sd + tt::col_tile_lo(G, sd) > p || sd + tt::col_tile_hi(G, sd) < p) continue;
            if (s0 < 0) s0 = sd;
            cnt += tt::diag_count(G, sd);
        }
        if (cnt == 0) continue;
        P.plane_count.push_back(cnt);
        P.plane_id.push_back(p);
        P.plane_s0.push_back(s0);
    }
    P.nplanes = (int)P.plane_count.size();
    P.max_plane_tiles = 0;
    for (int c : P.plane_count) P.max_plane_tiles = c > P.max_plane_tiles ? c : P.max_plane_tiles;
    P.nbblocks = (int)((G.NB + tt::kBndThreads - 1) / tt::kBndThreads);
    P.nslots = 8 * G.ntiles + 8 * P.nbblocks;
}

// Host check of the tile-plane enumeration before any sweep is launched:
// every tile the kernels decode lies in the grid's tile columns and in its
// column's slab range, its plane number is TI + TJ + TK, and the planes cover
// each tile exactly once.
int check_tiling(const tt::Plan& P) {
    const tt::Geo& G = P.G;
    std::vector<unsigned char> seen((size_t)G.ntiles, 0);
    long long total = 0;
    for (int q = 0; q < P.nplanes; ++q) {
        for (int b = 0; b < P.plane_count[q]; ++b) {
            int TI, TJ, TK;
            tt::tile_decode(G, P.plane_id[q], P.plane_s0[q], b, TI, TJ, TK);
            const int sd = TI + TJ;
            const int rel = TK - tt::col_tile_lo(G, sd);
            if (TI < 0 || TI >= G.nt[0] || TJ < 0 || TJ >= G.nt[1] || rel < 0 || TK > tt::col_tile_hi(G, sd) ||
                rel >= G.nt[2] || TI + TJ + TK != P.plane_id[q])
                return fail(TT_EINVAL, "internal: tile %d of tile-plane %d decodes outside the grid", b, P.plane_id[q]);
            unsigned char& f = seen[((size_t)TI * G.nt[1] + TJ) * G.nt[2] + rel];
            if (f) return fail(TT_EINVAL, "internal: tile-plane %d repeats a tile", P.plane_id[q]);
            f = 1;
            ++total;
        }
    }
    long long want = 0;
    for (int sd = 0; sd <= G.nt[0] + G.nt[1] - 2; ++sd)
        want += (long long)tt::diag_count(G, sd) * (tt::col_tile_hi(G, sd) - tt::col_tile_lo(G, sd) + 1);
    if (total != want) return fail(TT_EINVAL, "internal: tile-planes cover %lld of %lld tiles", total, want);
    return TT_OK;
}

void bind_workspace(tt::Plan& P, void* ws, const Layout& L) {
    char* b = static_cast<char*>(ws);
    P.src = reinterpret_cast<tt::Src*>(b + L.off_src);
    P.tab0 = reinterpret_cast<double*>(b + L.off_t0);
    P.tab1 = reinterpret_cast<double2*>(b + L.off_t1);
    P.tab2 = reinterpret_cast<double2*>(b + L.off_t2);
    P.active = reinterpret_cast<int*>(b + L.off_active);
    P.iter = reinterpret_cast<int*>(b + L.off_iter);
    P.counter = reinterpret_cast<int*>(b + L.off_counter);
    P.part = reinterpret_cast<double*>(b + L.off_part);
    P.part2 = reinterpret_cast<double*>(b + L.off_part2);
    P.coef = reinterpret_cast<double*>(b + L.off_coef);
    P.diag = reinterpret_cast<double*>(b + L.off_diag);
    P.rhs = reinterpret_cast<double*>(b + L.off_rhs);
    P.box = reinterpret_cast<int*>(b + L.off_box);
    P.bnd_in = reinterpret_cast<double*>(b + L.off_bnd);
    P.bnd_rhs = P.bnd_in + (size_t)P.nsrc * (size_t)P.G.NB;
    P.model = reinterpret_cast<double*>(b + L.off_model);
    P.T.t0 = P.tab0;
    P.T.t1 = P.tab1;
    P.T.t2 = P.tab2;
}

int tile_k_of(const tt_opts* o, int which) {
    int tk = (o && o->tile_k > 0) ? o->tile_k
                                  : (which == 0 ? kDefaultTileKFwd : (which == 1 ? kDefaultTileKAdj : kDefaultTileK));
    return tk > tt::kMaxTileK ? tt::kMaxTileK : tk;
}

// pinned host words that receive the active-source count of each iteration
// (allocated once per thread and kept until the process ends: freeing them
// from a thread-exit destructor could run after the HIP runtime is gone)
thread_local int* g_pinned = nullptr;

int pinned_counter(int** out) {
    if (!g_pinned)
        TT_HIP(hipHostMalloc(reinterpret_cast<void**>(&g_pinned), 2 * TT_MAX_GROUPS * sizeof(int),
                             hipHostMallocDefault));
    *out = g_pinned;
    return TT_OK;
}

// per-thread, per-device streams of groups 1.. (group 0 runs on the caller's
// stream); created on first use with default priority and kept
constexpr int kMaxDevices = 64;
thread_local hipStream_t g_group_streams[kMaxDevices][TT_MAX_GROUPS] = {};

int group_stream(int q, hipStream_t caller, hipStream_t* out) {
    if (q == 0) {
        *out = caller;
        return TT_OK;
    }
    int dev = 0;
    TT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TT_EINVAL, "device index %d out of range", dev);
    hipStream_t& s = g_group_streams[dev][q];
    if (!s) TT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    *out = s;
    return TT_OK;
}

// stream used only to capture graphs (capture is not allowed on the legacy
// default stream); nothing runs on it
thread_local hipStream_t g_capture_stream = nullptr;

// Capture `iters` iterations into an executable graph.
template <typename Launch>
int capture_iterations(Launch launch_one, int iters, hipGraphExec_t* exec) {
    if (!g_capture_stream) TT_HIP(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    TT_HIP(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    for (int q = 0; q < iters; ++q) launch_one(g_capture_stream);
    hipError_t e = hipStreamEndCapture(g_capture_stream, &graph);
    if (e != hipSuccess) return fail(TT_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(TT_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    return TT_OK;
}

// Per-thread, per-device events that fork the source groups off the caller's
// stream and join them back (created on first use with timing disabled, and
// kept: a call made while the caller's stream is being captured records and
// waits on them like any stream work).
thread_local hipEvent_t g_fork_ev[kMaxDevices] = {};
thread_local hipEvent_t g_join_ev[kMaxDevices][TT_MAX_GROUPS] = {};

int cached_event(hipEvent_t& ev, hipEvent_t* out) {
    if (!ev) TT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    *out = ev;
    return TT_OK;
}

int device_index(int* dev) {
    TT_HIP(hipGetDevice(dev));
    if (*dev < 0 || *dev >= kMaxDevices) return fail(TT_EINVAL, "device index %d out of range", *dev);
    return TT_OK;
}

// Graphs replayed by asynchronous calls: each is destroyed by a later call of
// the same thread once the event recorded after its last replay has completed.
thread_local std::vector<std::pair<hipGraphExec_t, hipEvent_t>> g_retired;

void reclaim_graphs() {
    size_t keep = 0;
    for (size_t q = 0; q < g_retired.size(); ++q) {
        if (hipEventQuery(g_retired[q].second) == hipSuccess) {
            (void)hipGraphExecDestroy(g_retired[q].first);
            (void)hipEventDestroy(g_retired[q].second);
        } else {
            g_retired[keep++] = g_retired[q];
        }
    }
    g_retired.resize(keep);
}

// One group of a batched solve: its plan, kernel arguments and stream.
struct Group {
    tt::Plan P;
    tt::SweepArgs a;
    hipStream_t st = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int issued = 0;
    bool done = false;
};

// Host-polled iterations (TT_FLAG_POLL): enqueue iterations of every group on
// its own stream until no source of any group is active.  Each group's count
// of active sources after iteration k is copied to pinned host memory; the
// host waits for it while iteration k+1 of every group is already queued, so
// no stream idles on the poll.  Returns with every group's work complete.
template <typename Launch>
int run_polled(std::vector<Group>& gs, bool use_graph, Launch launch_one) {
    int* host = nullptr;
    int rc = pinned_counter(&host);
    if (rc) return rc;
    int result = TT_OK;
    for (auto& g : gs) {
        if (use_graph && (rc = capture_iterations([&](hipStream_t s_) { launch_one(g, s_); }, 1, &g.exec))) {
            result = rc;
            break;
        }
        if (hipEventCreateWithFlags(&g.ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&g.ev[1], hipEventDisableTiming) != hipSuccess) {
            result = fail(TT_EHIP, "event create failed");
            break;
        }
    }
    while (result == TT_OK) {
        for (size_t q = 0; q < gs.size() && result == TT_OK; ++q) {
            Group& g = gs[q];
            if (g.done || g.issued >= g.P.max_iter) continue;
            if (g.exec) {
                hipError_t e = hipGraphLaunch(g.exec, g.st);
                if (e != hipSuccess) result = fail(TT_EHIP, "graph launch: %s", hipGetErrorString(e));
            } else {
                launch_one(g, g.st);
            }
            int* slot = &host[2 * q + (g.issued & 1)];
            hipError_t e = hipMemcpyAsync(slot, g.P.counter, sizeof(int), hipMemcpyDeviceToHost, g.st);
            if (e == hipSuccess) e = hipEventRecord(g.ev[g.issued & 1], g.st);
            if (e != hipSuccess && result == TT_OK) result = fail(TT_EHIP, "iteration enqueue: %s", hipGetErrorString(e));
            ++g.issued;
        }
        bool pending = false;
        for (size_t q = 0; q < gs.size() && result == TT_OK; ++q) {
            Group& g = gs[q];
            if (g.done) continue;
            // wait for the previous iteration's count (or the last one when no more can be issued)
            const int wait_for = (g.issued < g.P.max_iter) ? g.issued - 2 : g.issued - 1;
            if (wait_for < 0) {
                pending = true;
                continue;
            }
            hipError_t e = hipEventSynchronize(g.ev[wait_for & 1]);
            if (e != hipSuccess) {
                result = fail(TT_EHIP, "iteration wait: %s", hipGetErrorString(e));
                break;
            }
            if (host[2 * q + (wait_for & 1)] == 0 || wait_for == g.P.max_iter - 1)
                g.done = true;
            else
                pending = true;
        }
        if (!pending) break;
    }
    for (auto& g : gs) {
        hipError_t e = hipStreamSynchronize(g.st);
        if (e != hipSuccess && result == TT_OK) result = fail(TT_EHIP, "stream sync: %s", hipGetErrorString(e));
        if (g.ev[0]) (void)hipEventDestroy(g.ev[0]);
        if (g.ev[1]) (void)hipEventDestroy(g.ev[1]);
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && result == TT_OK) result = fail(TT_EHIP, "kernel launch: %s", hipGetErrorString(e));
    return result;
}

// Asynchronous iterations (the default): every group gets exactly max_iter
// iterations enqueued on its stream and nothing waits on the host.  A source
// that converges is marked inactive on the device and its workgroups exit at
// once in later launches, so the iterations past the last source's
// convergence cost launch overhead only.  With use_graph, kGraphChunk
// iterations are captured once per group and replayed (not while the caller's
// stream is itself being captured: the launches then go into the caller's
// graph).
constexpr int kGraphChunk = 4;

template <typename Launch>
int run_async(std::vector<Group>& gs, bool use_graph, Launch launch_one) {
    if (use_graph) reclaim_graphs();  // (never while the caller's stream is captured: it queries events)
    int rc = TT_OK;
    const int chunk = use_graph ? kGraphChunk : 1;
    for (auto& g : gs)
        if (use_graph && g.P.max_iter >= kGraphChunk &&
            (rc = capture_iterations([&](hipStream_t s_) { launch_one(g, s_); }, kGraphChunk, &g.exec)))
            return rc;
    // Enqueue round-robin over the groups, one iteration (or one replayed
    // chunk) at a time: a launch blocks the host while its stream's queue is
    // full, and enqueuing one group's whole budget first would hold the other
    // groups back until that group had nearly finished.
    int maxit = 0;
    for (auto& g : gs) maxit = g.P.max_iter > maxit ? g.P.max_iter : maxit;
    for (int q = 0; q < maxit; q += chunk) {
        for (auto& g : gs) {
            const int it = g.P.max_iter;
            if (q >= it) continue;
            if (g.exec && q + kGraphChunk <= it) {
                TT_HIP(hipGraphLaunch(g.exec, g.st));
            } else {
                for (int r = q; r < it && r < q + chunk; ++r) launch_one(g, g.st);
            }
        }
    }
    for (auto& g : gs) {
        if (!g.exec) continue;
        hipEvent_t done = nullptr;
        TT_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        TT_HIP(hipEventRecord(done, g.st));
        g_retired.push_back({g.exec, done});
        g.exec = nullptr;
    }
    TT_HIP(hipGetLastError());
    return TT_OK;
}

// After the iterations (and any per-group kernels after them): join the
// groups' streams back into the caller's stream (asynchronous) or wait for
// them (polled; run_polled has already waited for the iterations).
int finish_groups(std::vector<Group>& gs, hipStream_t caller, bool polled) {
    if (polled) {
        for (auto& g : gs) TT_HIP(hipStreamSynchronize(g.st));
        return TT_OK;
    }
    int dev = 0, rc = device_index(&dev);
    if (rc) return rc;
    for (size_t q = 1; q < gs.size(); ++q) {
        hipEvent_t ev = nullptr;
        if ((rc = cached_event(g_join_ev[dev][q], &ev))) return rc;
        TT_HIP(hipEventRecord(ev, gs[q].st));
        TT_HIP(hipStreamWaitEvent(caller, ev, 0));
    }
    return TT_OK;
}

// Whether work enqueued on `st` is being captured into a graph.
bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

// Host-polled solve: asked for, or implied by per-launch sweep timing (whose
// events are read back when the call returns).
bool polled_mode(const tt_opts* o) { return (o->flags & (TT_FLAG_POLL | TT_FLAG_TIME_SWEEPS)) != 0; }

// Workspace bytes of a solve split into `groups` groups (one region per group).
size_t grouped_total(const tt::Geo& G, int nsrc, int groups, int which, bool compact = false) {
    size_t total = 0;
    for (int q = 0; q < groups; ++q) {
        const int n = group_begin(nsrc, groups, q + 1) - group_begin(nsrc, groups, q);
        tt::Plan P;
        fill_plan(P, G, n);
        total += layout(G, n, P.nslots, which, compact).total;
    }
    return total;
}

bool compact_of(const tt_opts* o) { return o && (o->flags & TT_FLAG_COMPACT_ADJOINT); }

// Plans of the groups of a solve, bound to consecutive workspace regions, with
// their streams made to wait for the work already queued on the caller's stream.
int make_groups(const tt::Geo& G, int nsrc, int groups, int which, void* ws, size_t ws_bytes, const tt_opts* opts,
                hipStream_t caller, std::vector<Group>& gs) {
    const bool compact = which == 1 && compact_of(opts);
    const size_t need = grouped_total(G, nsrc, groups, which, compact);
    if (ws_bytes < need) return fail(TT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    if (opts->budgets)
        for (int q = 0; q < nsrc; ++q)
            if (opts->budgets[q] < 1 || opts->budgets[q] > opts->max_iter)
                return fail(TT_EINVAL, "opts.budgets[%d] = %d is outside [1, max_iter = %d]", q, opts->budgets[q],
                            opts->max_iter);
    hipEvent_t fork = nullptr;
    if (groups > 1) {
        int dev = 0, rc0 = device_index(&dev);
        if (rc0 || (rc0 = cached_event(g_fork_ev[dev], &fork))) return rc0;
        TT_HIP(hipEventRecord(fork, caller));
    }
    gs.resize(groups);
    char* base = static_cast<char*>(ws);
    int rc = TT_OK;
    for (int q = 0; q < groups && rc == TT_OK; ++q) {
        Group& g = gs[q];
        const int n = group_begin(nsrc, groups, q + 1) - group_begin(nsrc, groups, q);
        fill_plan(g.P, G, n);
        Layout L = layout(G, n, g.P.nslots, which, compact);
        bind_workspace(g.P, base, L);
        g.P.compact = compact;
        base += L.total;
        g.P.kappa = opts->kappa;
        g.P.tol = opts->tol;
        g.P.max_iter = opts->max_iter;
        if (opts->budgets) {  // the group iterates its largest per-source budget
            g.P.max_iter = 1;
            for (int k = group_begin(nsrc, groups, q); k < group_begin(nsrc, groups, q + 1); ++k)
                g.P.max_iter = opts->budgets[k] > g.P.max_iter ? opts->budgets[k] : g.P.max_iter;
        }
        g.P.hist_stride = opts->max_iter;
        rc = group_stream(q, caller, &g.st);
        if (rc == TT_OK && q > 0) {
            hipError_t e = hipStreamWaitEvent(g.st, fork, 0);
            if (e != hipSuccess) rc = fail(TT_EHIP, "stream wait: %s", hipGetErrorString(e));
        }
    }
    return rc;
}

// sweep-kernel timing totals of this thread: [0] forward, [1] adjoint
thread_local double g_sweep_ms[2] = {0.0, 0.0};
thread_local int64_t g_sweep_launches[2] = {0, 0};

// sum and release the event pairs recorded during a solve (stream already synchronised)
void collect_timing(std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>>& ev, int which) {
    for (auto& pr : ev) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.first.first, pr.first.second) == hipSuccess) {
            g_sweep_ms[which] += ms;
            g_sweep_launches[which] += pr.second;
        }
        (void)hipEventDestroy(pr.first.first);
        (void)hipEventDestroy(pr.first.second);
    }
    ev.clear();
}

int check_ptrs(std::initializer_list<const void*> ps) {
    int q = 0;
    for (const void* p : ps) {
        if (!p) return fail(TT_EINVAL, "required pointer argument %d is NULL", q);
        ++q;
    }
    return TT_OK;
}

// Forward solve on a workspace that the caller checked (tt_forward) or the
// scratch array provides (tt_forward_noalloc, one source group); the plan
// checks are done by the callers.
int forward_run(const tt::Geo& G, const double* s, const double* xi, const double* eta, int32_t nsrc,
                const double* src_pos, const double* src_par, const double* tau_init, const tt_opts* opts, double* tau,
                int32_t* status, void* ws, size_t ws_bytes, int groups, hipStream_t caller) {
    int rc = TT_OK;
    std::vector<Group> gs;
    if ((rc = make_groups(G, nsrc, groups, 0, ws, ws_bytes, opts, caller, gs))) return rc;
    std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> ev;
    for (int q = 0; q < groups; ++q) {
        Group& g = gs[q];
        const int q0 = group_begin(nsrc, groups, q);
        g.P.eps_hist = opts->eps_hist ? opts->eps_hist + (long long)q0 * opts->max_iter : nullptr;
        if (opts->flags & TT_FLAG_TIME_SWEEPS) g.P.timing = &ev;
        tt::launch_tables(g.P, g.st);
        tt::launch_src_setup(g.P, src_pos + 3LL * q0, src_par + 3LL * q0, g.st);
        g.a = tt::make_args(g.P, s, xi, eta, tau + (long long)q0 * G.N, status + q0);
        tt::launch_fwd_init(g.P, g.a, tau_init ? tau_init + (long long)q0 * G.N : nullptr, s, xi, eta, g.st);
    }
    TT_HIP(hipGetLastError());
    const bool polled = polled_mode(opts);
    const bool graph = (opts->flags & TT_FLAG_GRAPH) && !(opts->flags & TT_FLAG_TIME_SWEEPS) && !capturing(caller);
    auto one = [&](Group& g, hipStream_t s_) { tt::launch_fwd_iteration(g.P, g.a, s_); };
    rc = polled ? run_polled(gs, graph, one) : run_async(gs, graph, one);
    collect_timing(ev, 0);
    if (rc == TT_OK) rc = finish_groups(gs, caller, polled);
    return rc;
}

// Argument and tiling checks shared by the forward entry points.
int forward_checks(const tt_grid* grid, int32_t nsrc, const tt_opts* opts, std::initializer_list<const void*> ptrs,
                   tt::Geo* G) {
    int rc = check_grid(grid);
    if (rc || (rc = check_opts(opts))) return rc;
    if (nsrc < 0) return fail(TT_EINVAL, "nsrc < 0");
    if (nsrc > 65535) return fail(TT_EINVAL, "nsrc > 65535");
    if (nsrc > 0 && (rc = check_ptrs(ptrs))) return rc;
    *G = make_geo(grid, tile_k_of(opts, 0));
    tt::Plan P;
    fill_plan(P, *G, 1);
    if (P.max_plane_tiles > 65535) return fail(TT_EINVAL, "too many tiles per tile-plane; raise opts.tile_k");
    return check_tiling(P);
}

// Device address of this device's scratch array (hipGetSymbolAddress once per
// device, with that device current; kept for the life of the process).
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(void** out) {
    int dev = 0, rc = device_index(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TT_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TT_OK;
}

}  // namespace

extern "C" {

const char* tt_last_error(void) { return g_err.c_str(); }

int32_t tt_default_tile_k(int32_t which) {
    return which == 0 ? kDefaultTileKFwd : (which == 1 ? kDefaultTileKAdj : 0);
}

int tt_sweep_timing(int32_t which, double* total_ms, int64_t* launches, int32_t reset) {
    if (which < 0 || which > 1) return fail(TT_EINVAL, "which must be 0 or 1");
    if (total_ms) *total_ms = g_sweep_ms[which];
    if (launches) *launches = g_sweep_launches[which];
    if (reset) {
        g_sweep_ms[which] = 0.0;
        g_sweep_launches[which] = 0;
    }
    return TT_OK;
}

size_t tt_workspace_size(const tt_grid* grid, int32_t nsrc, const tt_opts* opts, int32_t which) {
    if (check_grid(grid) || nsrc < 1 || which < 0 || which > 3) return 0;
    if (opts && (opts->groups < 0 || opts->groups > TT_MAX_GROUPS)) return 0;
    if (opts && (opts->tile_k < 0 || opts->tile_k > tt::kMaxTileK)) return 0;
    tt::Geo G = make_geo(grid, tile_k_of(opts, which));
    return grouped_total(G, nsrc, which <= 1 ? groups_of(opts, nsrc) : 1, which, which == 1 && compact_of(opts));
}

int tt_source_params(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
                     const double* src_pos, double* src_par, void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc) return rc;
    if (nsrc < 0) return fail(TT_EINVAL, "nsrc < 0");
    if (nsrc == 0) return TT_OK;
    if ((rc = check_ptrs({s, xi, eta, src_pos, src_par}))) return rc;
    tt::Geo G = make_geo(grid, kDefaultTileK);
    tt::launch_source_params(G, s, xi, eta, src_pos, src_par, nsrc, (hipStream_t)stream);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_forward(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
               const double* src_pos, const double* src_par, const double* tau_init, const tt_opts* opts, double* tau,
               int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    tt::Geo G;
    int rc = forward_checks(grid, nsrc, opts, {s, xi, eta, src_pos, src_par, tau, status, ws}, &G);
    if (rc || nsrc == 0) return rc;
    return forward_run(G, s, xi, eta, nsrc, src_pos, src_par, tau_init, opts, tau, status, ws, ws_bytes,
                       groups_of(opts, nsrc), (hipStream_t)stream);
}

int tt_forward_noalloc(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
                       const double* src_pos, const double* src_par, const double* tau_init, const tt_opts* opts,
                       double* tau, int32_t* status, void* stream) {
    g_err.clear();
    tt::Geo G;
    int rc = forward_checks(grid, nsrc, opts, {s, xi, eta, src_pos, src_par, tau, status}, &G);
    if (rc || nsrc == 0) return rc;
    if (opts->flags & (TT_FLAG_POLL | TT_FLAG_TIME_SWEEPS | TT_FLAG_GRAPH))
        return fail(TT_EINVAL, "tt_forward_noalloc: TT_FLAG_POLL, TT_FLAG_TIME_SWEEPS and TT_FLAG_GRAPH need "
                               "allocations (pinned memory, events, graphs) and are not available here");
    const size_t need = grouped_total(G, nsrc, 1, 0);
    if (need > kScratchBytes)
        return fail(TT_EINVAL, "tt_forward_noalloc: this grid and batch need %zu bytes of workspace, more than the "
                               "%zu-byte scratch; use tt_forward with a caller workspace", need, kScratchBytes);
    void* ws = nullptr;
    if ((rc = scratch_ptr(&ws))) return rc;
    return forward_run(G, s, xi, eta, nsrc, src_pos, src_par, tau_init, opts, tau, status, ws, kScratchBytes, 1,
                       (hipStream_t)stream);
}

size_t tt_forward_noalloc_limit(void) { return kScratchBytes; }

int tt_sample(const tt_grid* grid, int32_t nsrc, const double* src_pos, const double* src_par, const double* tau,
              int32_t nrec, const double* rec_pos, double* T_rec, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc) return rc;
    if (nsrc < 0 || nrec < 0) return fail(TT_EINVAL, "negative count");
    if (nsrc == 0 || nrec == 0) return TT_OK;
    if ((rc = check_ptrs({src_pos, src_par, tau, rec_pos, T_rec, ws}))) return rc;
    tt::Geo G = make_geo(grid, kDefaultTileK);
    tt::Plan P;
    fill_plan(P, G, nsrc);
    Layout L = layout(G, nsrc, P.nslots, 2);
    if (ws_bytes < L.total) return fail(TT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    bind_workspace(P, ws, L);
    hipStream_t st = (hipStream_t)stream;
    tt::launch_tables(P, st);
    tt::launch_src_setup(P, src_pos, src_par, st);
    tt::launch_sample(P, tau, nrec, rec_pos, T_rec, st);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

// shared set-up of the relocation entry points: the receiver-side fields as
// sources of a sampling plan
static int reloc_plan(const tt_grid* grid, int32_t nfield, const double* field_pos, const double* field_par,
                      const double* tau, int32_t nev, const double* ev_pos, void* ws, size_t ws_bytes,
                      hipStream_t st, tt::Plan& P) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (nfield < 0 || nev < 0) return fail(TT_EINVAL, "negative count");
    if (nfield > 65535) return fail(TT_EINVAL, "nfield > 65535");
    if (nev > 0x7fffffff / 4) return fail(TT_EINVAL, "nev too large");
    if ((rc = check_ptrs({field_pos, field_par, tau, ev_pos, ws}))) return rc;
    tt::Geo G = make_geo(grid, kDefaultTileK);
    fill_plan(P, G, nfield);
    Layout L = layout(G, nfield, P.nslots, 2);
    if (ws_bytes < L.total) return fail(TT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    bind_workspace(P, ws, L);
    tt::launch_tables(P, st);
    tt::launch_src_setup(P, field_pos, field_par, st);
    return TT_OK;
}

int tt_reloc_times(const tt_grid* grid, int32_t nfield, const double* field_pos, const double* field_par,
                   const double* tau, int32_t nev, const double* ev_pos, const double* ev_t0, double* T, void* ws,
                   size_t ws_bytes, void* stream) {
    g_err.clear();
    if (nfield == 0 || nev == 0) return (nfield < 0 || nev < 0) ? fail(TT_EINVAL, "negative count") : TT_OK;
    if (!T) return fail(TT_EINVAL, "T is NULL");
    tt::Plan P;
    hipStream_t st = (hipStream_t)stream;
    int rc = reloc_plan(grid, nfield, field_pos, field_par, tau, nev, ev_pos, ws, ws_bytes, st, P);
    if (rc) return rc;
    tt::launch_reloc_times(P, tau, nev, ev_pos, ev_t0, T, st);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_reloc_kernel(const tt_grid* grid, int32_t nfield, const double* field_pos, const double* field_par,
                    const double* tau, int32_t nev, const double* ev_pos, const double* R, double* K, void* ws,
                    size_t ws_bytes, void* stream) {
    g_err.clear();
    if (nfield < 0 || nev < 0) return fail(TT_EINVAL, "negative count");
    if (nev == 0) return TT_OK;
    if (!K) return fail(TT_EINVAL, "K is NULL");
    if (nfield == 0) {
        tt::launch_fill(K, 4LL * nev, 0.0, (hipStream_t)stream);
        TT_HIP(hipGetLastError());
        return TT_OK;
    }
    if (!R) return fail(TT_EINVAL, "R is NULL");
    tt::Plan P;
    hipStream_t st = (hipStream_t)stream;
    int rc = reloc_plan(grid, nfield, field_pos, field_par, tau, nev, ev_pos, ws, ws_bytes, st, P);
    if (rc) return rc;
    tt::launch_reloc_kernel(P, tau, nev, ev_pos, R, K, st);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_misfit(int32_t nsrc, int32_t nrec, const double* T_rec, const double* T_obs, const double* w, int32_t npair,
              const int32_t* pairs, const double* wpair, double alpha, double beta, double* R, double* chi,
              void* stream) {
    g_err.clear();
    if (nsrc < 0 || nrec < 0 || npair < 0) return fail(TT_EINVAL, "negative count");
    // chi is written even for an empty batch (as 0); the [nsrc][nrec] arrays
    // are required only when they hold values
    int rc = check_ptrs({chi});
    if (rc || (nsrc > 0 && nrec > 0 && (rc = check_ptrs({T_rec, T_obs, R})))) return rc;
    if (npair > 0 && !pairs) return fail(TT_EINVAL, "pairs is NULL with npair > 0");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(TT_EINVAL, "alpha/beta not finite");
    tt::launch_misfit(nsrc, nrec, T_rec, T_obs, w, npair, pairs, wpair, alpha, beta, R, chi, (hipStream_t)stream);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_misfit_cr(int32_t nsrc, int32_t nrec, const double* T_rec, const double* T_obs, const int32_t* cr_off,
                 const int32_t* cr_pair, const double* wcr, double gamma, double* R, double* chi, void* stream) {
    g_err.clear();
    if (nsrc < 0 || nrec < 0) return fail(TT_EINVAL, "negative count");
    int rc = check_ptrs({cr_off, chi});
    if (rc || (nsrc > 0 && nrec > 0 && (rc = check_ptrs({T_rec, T_obs, R})))) return rc;
    if (!std::isfinite(gamma)) return fail(TT_EINVAL, "gamma not finite");
    if (nrec == 0) return TT_OK;
    tt::launch_misfit_cr(nsrc, nrec, T_rec, T_obs, cr_off, cr_pair, wcr, gamma, R, chi, (hipStream_t)stream);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_adjoint(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
               const double* src_pos, const double* src_par, const double* tau, int32_t nrec, const double* rec_pos,
               const double* R, const tt_opts* opts, double* lam, int32_t* status, void* ws, size_t ws_bytes,
               void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc || (rc = check_opts(opts))) return rc;
    if (nsrc < 0 || nrec < 0) return fail(TT_EINVAL, "negative count");
    if (nsrc == 0) return TT_OK;
    if (nsrc > 65535) return fail(TT_EINVAL, "nsrc > 65535");
    if ((rc = check_ptrs({s, xi, eta, src_pos, src_par, tau, lam, status, ws}))) return rc;
    if (nrec > 0 && (!rec_pos || !R)) return fail(TT_EINVAL, "rec_pos/R NULL with nrec > 0");
    tt::Geo G = make_geo(grid, tile_k_of(opts, 1));
    {
        tt::Plan P;
        fill_plan(P, G, 1);
        if (P.max_plane_tiles > 65535) return fail(TT_EINVAL, "too many tiles per tile-plane; raise opts.tile_k");
        if ((rc = check_tiling(P))) return rc;
    }
    const int groups = groups_of(opts, nsrc);
    hipStream_t caller = (hipStream_t)stream;
    std::vector<Group> gs;
    if ((rc = make_groups(G, nsrc, groups, 1, ws, ws_bytes, opts, caller, gs))) return rc;
    std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> ev;
    for (int q = 0; q < groups; ++q) {
        Group& g = gs[q];
        const int q0 = group_begin(nsrc, groups, q);
        g.P.eps_hist = opts->eps_hist ? opts->eps_hist + (long long)q0 * opts->max_iter : nullptr;
        g.P.continuous = (opts->flags & TT_FLAG_CONTINUOUS_ADJOINT) != 0;
        if (opts->flags & TT_FLAG_TIME_SWEEPS) g.P.timing = &ev;
        tt::launch_tables(g.P, g.st);
        tt::launch_src_setup(g.P, src_pos + 3LL * q0, src_par + 3LL * q0, g.st);
        g.a = tt::make_args(g.P, s, xi, eta, lam + (long long)q0 * G.N, status + q0);
        tt::launch_adj_init(g.P, g.a, tau + (long long)q0 * G.N, nrec, rec_pos, R ? R + (long long)q0 * nrec : nullptr,
                            (opts->flags & TT_FLAG_ADJOINT_INIT) ? lam + (long long)q0 * G.N : nullptr, g.st);
    }
    TT_HIP(hipGetLastError());
    const bool polled = polled_mode(opts);
    const bool graph = (opts->flags & TT_FLAG_GRAPH) && !(opts->flags & TT_FLAG_TIME_SWEEPS) && !capturing(caller);
    auto one = [&](Group& g, hipStream_t s_) { tt::launch_adj_iteration(g.P, g.a, s_); };
    rc = polled ? run_polled(gs, graph, one) : run_async(gs, graph, one);
    collect_timing(ev, 1);
    if (rc == TT_OK && (opts->flags & TT_FLAG_CONTINUOUS_ADJOINT)) {
        for (int q = 0; q < groups; ++q)
            tt::launch_cadj_scale(gs[q].P, s, lam + (long long)group_begin(nsrc, groups, q) * G.N, gs[q].st);
        TT_HIP(hipGetLastError());
    }
    if (rc == TT_OK) rc = finish_groups(gs, caller, polled);
    return rc;
}

int tt_kernel(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
              const double* src_pos, const double* src_par, const double* tau, const double* lam, double* grad,
              int32_t accumulate, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc) return rc;
    if (nsrc < 0) return fail(TT_EINVAL, "nsrc < 0");
    if ((rc = check_ptrs({s, xi, eta, grad}))) return rc;
    if (nsrc > 0 && (rc = check_ptrs({src_pos, src_par, tau, lam, ws}))) return rc;
    tt::Geo G = make_geo(grid, kDefaultTileK);
    tt::Plan P;
    fill_plan(P, G, nsrc > 0 ? nsrc : 1);
    P.nsrc = nsrc;
    Layout L = layout(G, nsrc > 0 ? nsrc : 1, P.nslots, 3);
    if (nsrc > 0 && ws_bytes < L.total) return fail(TT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t st = (hipStream_t)stream;
    if (nsrc > 0) {
        bind_workspace(P, ws, L);
        tt::launch_tables(P, st);
        tt::launch_src_setup(P, src_pos, src_par, st);
    }
    tt::launch_kernel_accum(P, xi, eta, tau, lam, grad, accumulate, st);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_kernel_density(const tt_grid* grid, const double* s, const double* dens, const double* grad, double eps,
                      double zeta, double* K, double* Kd, void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc) return rc;
    if ((rc = check_ptrs({s, dens, grad, K}))) return rc;
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(TT_EINVAL, "eps must be finite and >= 0");
    if (!std::isfinite(zeta)) return fail(TT_EINVAL, "zeta must be finite");
    tt::Geo G = make_geo(grid, kDefaultTileK);
    tt::launch_kernel_density(G, s, dens, grad, eps, zeta, K, Kd, (hipStream_t)stream);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

static int check_mg(int H, const int32_t* m, const double* coords) {
    if (H < 1 || H > TT_MG_MAX_GRIDS) return fail(TT_EINVAL, "H = %d outside [1, %d]", H, TT_MG_MAX_GRIDS);
    if (!m || !coords) return fail(TT_EINVAL, "m and coords must not be NULL");
    for (int q = 0; q < 3 * H; ++q)
        if (m[q] < 1 || m[q] > 1 << 20) return fail(TT_EINVAL, "inversion grid size m[%d] = %d out of range", q, m[q]);
    long long s12 = 0;
    for (int q = 0; q < H; ++q) {
        if ((long long)m[3 * q] * m[3 * q + 1] * m[3 * q + 2] > 0x7fffffffLL)
            return fail(TT_EINVAL, "inversion grid %d too large", q);
        s12 += (long long)m[3 * q + 1] * m[3 * q + 2];
    }
    if (s12 > 0x7fffffffLL) return fail(TT_EINVAL, "inversion grids too large");
    return TT_OK;
}

size_t tt_mg_workspace_size(const tt_grid* grid, int32_t H, const int32_t* m) {
    g_err.clear();
    const double dummy = 0.0;
    if (check_grid(grid) || check_mg(H, m, &dummy)) return 0;
    const tt::Geo G = make_geo(grid, kDefaultTileK);
    return tt::plan_mg_project(G, tt::make_mg(H, m)).ws_bytes;
}

int tt_mg_project(const tt_grid* grid, int32_t H, const int32_t* m, const double* coords, const double* K,
                  double* out, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc || (rc = check_mg(H, m, coords))) return rc;
    if ((rc = check_ptrs({K, out}))) return rc;
    tt::Geo G = make_geo(grid, kDefaultTileK);
    const size_t need = tt::plan_mg_project(G, tt::make_mg(H, m)).ws_bytes;
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(TT_EINVAL, "workspace of %zu bytes too small (need %zu)", ws_bytes, need);
    tt::launch_mg_project(G, H, m, coords, K, out, (double*)ws, (hipStream_t)stream);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

int tt_mg_expand(const tt_grid* grid, int32_t H, const int32_t* m, const double* coords, const double* C,
                 double* field, void* stream) {
    g_err.clear();
    int rc = check_grid(grid);
    if (rc || (rc = check_mg(H, m, coords))) return rc;
    if ((rc = check_ptrs({C, field}))) return rc;
    tt::Geo G = make_geo(grid, kDefaultTileK);
    tt::launch_mg_expand(G, H, m, coords, C, field, (hipStream_t)stream);
    TT_HIP(hipGetLastError());
    return TT_OK;
}

}  // extern "C"

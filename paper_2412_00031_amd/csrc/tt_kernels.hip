// tt_kernels.hip -- CDNA4 (gfx950) kernels of libtt.
//
// Sweep schedule.  One directional sweep must visit the interior nodes in an
// order where x - sigma_a e_a precedes x on every axis a (the Gauss-Seidel
// order of fast sweeping, Sec. 3.1).  The stencil touches only axis neighbours
// and boundary nodes are not written during a sweep, so every such order yields
// the same numbers as the lexicographic one; the hyperplane-stepping idea of
// Sec. 3.4 (nodes with i'+j'+k' = L are independent) is used in this form:
//   - the interior is cut into 8 x 8 (i', j') tile columns (sweep-relative
//     coordinates, ragged last ones), and each tile column into slabs of tk
//     consecutive hyperplanes u = i' + j' + k' (sheared tiles: the 14-step ramp
//     of a skewed 8 x 8 walk is paid once per column, not once per tile);
//   - tiles with the same TI'+TJ'+TK' form a tile-plane; one launch processes
//     one tile-plane of every active source.  grid.x is the source, so
//     consecutive workgroups are one tile of consecutive sources: workgroups
//     are dealt to the 8 XCDs round-robin, hence every tile of a source runs
//     on the same XCD (its field stays in that XCD's L2) and the sources that
//     share an XCD read the same model lines;
//   - inside a tile one 64-lane wave owns the 8 x 8 columns; the tile and its
//     one-node halo are staged in LDS with contiguous column loads, then at
//     step t lane (li, lj) updates the node of its column on hyperplane
//     u = TK' tk + t, reading and writing LDS only, and the tile is written
//     back with contiguous column stores;
//   - per-node records (model, adjoint coefficients) are read from
//     row-coalesced layouts in which the 8 lanes of a tile row find their
//     records side by side on every step.
// Each sweep is followed by a boundary pass (one thread per boundary node), and
// each iteration by a finalize kernel that forms the convergence measure from
// per-tile partial sums in a fixed order (bitwise reproducible run to run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

// ---------------------------------------------------------------- helpers
// boundary node number b in [0, NB) -> (i, j, k); slabs i = 0 and n0-1 are full,
// slabs in between contribute the ring j in {0, n1-1} or k in {0, n2-1}.
__device__ __forceinline__ void bnd_decode(const Geo& G, long long b, int& i, int& j, int& k) {
    const long long plane = (long long)G.n[1] * G.n[2];
    const long long ring = 2LL * G.n[2] + 2LL * (G.n[1] - 2);
    if (b < plane) {
        i = 0; j = (int)(b / G.n[2]); k = (int)(b % G.n[2]);
        return;
    }
    b -= plane;
    if (b >= (long long)(G.n[0] - 2) * ring) {
        b -= (long long)(G.n[0] - 2) * ring;
        i = G.n[0] - 1; j = (int)(b / G.n[2]); k = (int)(b % G.n[2]);
        return;
    }
    i = 1 + (int)(b / ring);
    long long r = b % ring;
    if (r < G.n[2]) { j = 0; k = (int)r; return; }
    if (r < 2LL * G.n[2]) { j = G.n[1] - 1; k = (int)(r - G.n[2]); return; }
    r -= 2LL * G.n[2];
    j = 1 + (int)(r >> 1);
    k = (r & 1) ? G.n[2] - 1 : 0;
}

// inverse of bnd_decode
__device__ __forceinline__ long long bnd_encode(const Geo& G, int i, int j, int k) {
    const long long plane = (long long)G.n[1] * G.n[2];
    const long long ring = 2LL * G.n[2] + 2LL * (G.n[1] - 2);
    if (i == 0) return (long long)j * G.n[2] + k;
    if (i == G.n[0] - 1) return plane + (long long)(G.n[0] - 2) * ring + (long long)j * G.n[2] + k;
    long long base = plane + (long long)(i - 1) * ring;
    if (j == 0) return base + k;
    if (j == G.n[1] - 1) return base + G.n[2] + k;
    return base + 2LL * G.n[2] + 2LL * (j - 1) + (k == 0 ? 0 : 1);
}

__device__ __forceinline__ bool on_bnd(const Geo& G, int a, int idx) { return idx == 0 || idx == G.n[a] - 1; }
// boundary node (i, j, k) on a k face only: its column is interior
__device__ __forceinline__ bool kface_only(const Geo& G, int i, int j) { return !on_bnd(G, 0, i) && !on_bnd(G, 1, j); }

// Row-coalesced record layouts.  On a sweep hyperplane the 8 lanes of one
// tile row (fixed i, consecutive j) satisfy j + rho k = const with
// rho = sigma_1 sigma_2, so records stored by rows [i][w = j + rho k][j] put
// those 8 lanes' records next to each other (family fam 0: rho = +1, fam 1:
// rho = -1).  Four layouts, lay = 2 fam + (s1 < 0), give each row a pitch of
// n1p records and place j at j + joff[s1 < 0], so that the 8 records a tile
// row reads on one step start on a multiple of 8 records (an aligned run of
// whole 128-byte lines for 32- and 48-byte records) for either sign of the j
// sweep.  Used for the model records and the adjoint coefficients.
__device__ __forceinline__ long long arec_idx(const Geo& G, int lay, int i, int j, int k) {
    const int w = (lay >> 1) == 0 ? j + k : j - k + (G.n[2] - 1);
    return ((long long)i * G.W + w) * G.n1p + j + G.joff[lay & 1];
}

__device__ __forceinline__ int astar_of(const Geo& G, const int p[3]) {
    int as = -1;
    for (int a = 0; a < 3; ++a)
        if (on_bnd(G, a, p[a])) as = a;
    return as;
}

// ---------------------------------------------------------------- set-up
__global__ void k_tables(Geo G, double* __restrict__ t0, double2* __restrict__ t1, double2* __restrict__ t2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < G.n[0]) t0[q] = G.o[0] + (double)q * G.h[0];
    if (q < G.n[1]) {
        double v = G.o[1] + (double)q * G.h[1];
        t1[q] = G.coord == 1 ? make_double2(cos(v), sin(v)) : make_double2(v, 0.0);
    }
    if (q < G.n[2]) {
        double v = G.o[2] + (double)q * G.h[2];
        t2[q] = G.coord == 1 ? make_double2(cos(v), sin(v)) : make_double2(v, 0.0);
    }
}

__global__ void k_src_setup(Geo G, const double* __restrict__ pos, const double* __restrict__ par,
                            Src* __restrict__ out, int nsrc) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nsrc) return;
    Src S;
    const double p0 = pos[3 * q], p1 = pos[3 * q + 1], p2 = pos[3 * q + 2];
    if (G.coord == 1) {
        const double ct = cos(p1), st = sin(p1), cp = cos(p2), sp = sin(p2);
        S.E[0] = ct * cp; S.E[1] = ct * sp; S.E[2] = st;
        S.E[3] = -st * cp; S.E[4] = -st * sp; S.E[5] = ct;
        S.E[6] = -sp; S.E[7] = cp; S.E[8] = 0.0;
        S.Xs[0] = p0 * S.E[0]; S.Xs[1] = p0 * S.E[1]; S.Xs[2] = p0 * S.E[2];
    } else {
        for (int a = 0; a < 9; ++a) S.E[a] = (a % 4 == 0) ? 1.0 : 0.0;
        S.Xs[0] = p0; S.Xs[1] = p1; S.Xs[2] = p2;
    }
    const double xi0 = par[3 * q + 1], eta0 = par[3 * q + 2];
    const double b = 1.0 - 2.0 * xi0, c = 1.0 + 2.0 * xi0, f = 2.0 * eta0;
    const double det = b * c - f * f;
    S.mi11 = c / det; S.mi12 = -f / det; S.mi22 = b / det;
    S.s0 = par[3 * q];
    S.fb[0] = cell_base(G, 0, p0);
    S.fb[1] = cell_base(G, 1, p1);
    S.fb[2] = cell_base(G, 2, p2);
    S.pad = 0;
    out[q] = S;
}

// trilinear cell and weights at a continuous position (clamped to the grid)
__global__ void k_source_params(Geo G, const double* __restrict__ s, const double* __restrict__ xi,
                                const double* __restrict__ eta, const double* __restrict__ pos,
                                double* __restrict__ par, int nsrc) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nsrc) return;
    const Tri t = tri_of(G, pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]);
    double a = 0.0, b = 0.0, c = 0.0;
    for (int c0 = 0; c0 < 2; ++c0)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int c2 = 0; c2 < 2; ++c2) {
                const double w = tri_w(t, c0, c1, c2);
                const long long x = nidx(G, t.b[0] + c0, t.b[1] + c1, t.b[2] + c2);
                a += w * s[x]; b += w * xi[x]; c += w * eta[x];
            }
    par[3 * q] = a; par[3 * q + 1] = b; par[3 * q + 2] = c;
}

__global__ void k_fill(double* __restrict__ p, long long n, double v) {
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x)
        p[x] = v;
}

// initialise a solve: field = init (or v0), fixed nodes = vfix; flags and counters
// init may alias the field: each element is read and then written by one thread
__global__ void k_solve_init(SweepArgs a, const double* init, double v0, double vfix) {
    const int src = blockIdx.y;
    const Src S = a.src[src];
    double* f = a.field + (long long)src * a.G.N;
    const double* ti = init ? init + (long long)src * a.G.N : nullptr;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < a.G.N;
         x += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(x % a.G.n[2]);
        const long long q = x / a.G.n[2];
        const int j = (int)(q % a.G.n[1]), i = (int)(q / a.G.n[1]);
        f[x] = in_fixed(S, i, j, k) ? vfix : (ti ? ti[x] : v0);
    }
    // partial-sum slots start at zero: slots of slab indices a short tile
    // column does not have are never written
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < a.nslots;
         x += (long long)gridDim.x * blockDim.x) {
        a.part[(long long)src * a.nslots + x] = 0.0;
        if (a.part2) a.part2[(long long)src * a.nslots + x] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.active[src] = 1;
        a.iter[src] = 0;
        a.status[src] = 0;
        if (src == 0) *a.counter = a.nsrc;
    }
}

// --------------------------------------------------------- sweep tiles
// Lane-constant context of one tile of one source in directional sweep DIR
// (signs s_a = -1 where bit 2 - a of DIR is set; compile-time, so every
// sign-dependent index folds to adds).
template <int DIR>
struct Dir {
    static constexpr int s0 = (DIR & 4) ? -1 : 1;
    static constexpr int s1 = (DIR & 2) ? -1 : 1;
    static constexpr int s2 = (DIR & 1) ? -1 : 1;
    static constexpr int fam = ((DIR >> 1) ^ DIR) & 1;  // row-coalesced layout family of this sweep
    static constexpr int lay = 2 * fam + (s1 > 0 ? 0 : 1);  // its aligned layout
};

struct TileCtx {
    int TI, TJ, TK, lane, li, lj, ext_i, ext_j;
    int t0, t1;    // wave-uniform walk: steps t0 <= t < t1 (u = TK tk + t)
    int kp0;       // this lane's k' at step 0 (k' = kp0 + t)
    int kplo, kphi;  // record fetch clamp: this lane's k' range in the tile (a valid k' if empty)
    int kq0;       // staged entry (ci, cj, kk) holds k' = kq0 - ci - cj + kk
    int kbase;     // absolute k = kbase + s2 k'
    bool colv, fcol;
    int i, j;
    int rbase, rstep;  // record index of this lane's column at k' = 0, and its change per k'
    // forward fetches: record and axis-2 table index at step 0, and the step
    // range [tlo, thi] that the clamp of k' to [kplo, kphi] allows
    int rr0, tt0, tlo, thi;
    int slot;          // partial-sum slot of the tile within one directional sweep
};

template <int DIR>
__device__ __forceinline__ TileCtx tile_ctx(const Geo& G, const Src& S, int plane, int s0) {
    using D = Dir<DIR>;
    TileCtx c;
    tile_decode(G, plane, s0, blockIdx.y, c.TI, c.TJ, c.TK);
    c.lane = threadIdx.x;
    c.li = c.lane >> 3;
    c.lj = c.lane & 7;
    c.ext_i = min(kBI, G.m[0] - c.TI * kBI);
    c.ext_j = min(kBJ, G.m[1] - c.TJ * kBJ);
    c.colv = c.li < c.ext_i && c.lj < c.ext_j;
    const int ip = c.TI * kBI + (c.colv ? c.li : 0), jp = c.TJ * kBJ + (c.colv ? c.lj : 0);
    c.i = D::s0 > 0 ? 1 + ip : G.n[0] - 2 - ip;
    c.j = D::s1 > 0 ? 1 + jp : G.n[1] - 2 - jp;
    c.fcol = (unsigned)(c.i - S.fb[0]) <= 1u && (unsigned)(c.j - S.fb[1]) <= 1u;
    const int U0 = c.TK * G.tk;
    const int ucol = kBI * (c.TI + c.TJ);  // u of the column's first node (i', j' at the tile corner, k' = 0)
    c.t0 = max(0, ucol - U0);
    c.t1 = min(G.tk, ucol + (c.ext_i - 1) + (c.ext_j - 1) + G.m[2] - U0);
    c.kp0 = U0 - ip - jp;
    // prefetches past the walk re-read the lane's last record of this tile
    // (a cache hit) instead of the next slab's
    c.kplo = max(0, c.kp0 + c.t0);
    c.kphi = min(G.m[2] - 1, c.kp0 + c.t1 - 1);
    if (c.kplo > c.kphi) c.kplo = c.kphi = min(max(c.kp0 + c.t0, 0), G.m[2] - 1);
    c.kq0 = U0 - ucol + 1;
    c.kbase = D::s2 > 0 ? 1 : G.n[2] - 2;
    // record index ((i W + w) n1p + j + joff) in the aligned layout of this sweep,
    // w = j + k (family 0) or j - k + n2 - 1 (family 1), k = kbase + s2 k': linear
    // in k' with slope s1 n1p in both families
    const int w0 = D::fam == 0 ? c.j + c.kbase : c.j - c.kbase + G.n[2] - 1;
    c.rbase = (c.i * G.W + w0) * G.n1p + c.j + G.joff[D::s1 > 0 ? 0 : 1];
    c.rstep = D::s1 * G.n1p;
    c.rr0 = c.rbase + c.rstep * c.kp0;
    c.tt0 = c.kbase + D::s2 * c.kp0;
    c.tlo = c.kplo - c.kp0;
    c.thi = c.kphi - c.kp0;
    c.slot = (c.TI * G.nt[1] + c.TJ) * G.nt[2] + (c.TK - col_tile_lo(G, c.TI + c.TJ));
    return c;
}

// Staged tile: the (8+2) x (8+2) columns of the tile and its i'/j' halo, each
// with the entries kk = 0..tk+1, in LDS as [ci][cj][kk] (ci = li + 1,
// cj = lj + 1; column pitch tk + 2: an odd pitch measured no better and costs
// a tile per CU at some depths).  Entry kk of column (ci, cj) is the node
// k' = kq0 - ci - cj + kk: the column windows are sheared along the tile's
// slab, so at step t lane (li, lj) owns entry t + 1 of its column and finds
// its upstream i'/j'/k' neighbours at entry t and its downstream ones at
// entry t + 2.  Everything a step reads from the field is staged (upstream
// tiles are finished, downstream ones untouched), so the walk touches LDS
// only; staged k' are clamped to the column's nodes [-1, m2] (entries outside
// are never read).  Loads and stores move contiguous column segments.
constexpr int kTC = kBI + 2;

// Staging.  The staged window is always the full (8+2) x (8+2) columns
// (columns past a ragged tile's end are staged from clamped, valid rows and
// never read) of Lp = tile_pitch(tk) slots; slot q of a column holds entry
// kk = q in sweeps with s2 > 0 and kk = Lp - 1 - q in sweeps with s2 < 0, so
// that consecutive slots always hold consecutive nodes in memory (ascending
// k).  The window is loaded with direct global-to-LDS loads of 16 bytes per
// lane (lane l of a load writes the l-th slot pair from the load's LDS
// address): each load covers 64 / (Lp / 2) whole columns, so a lane keeps its
// column offset and slot pair in every load, no data passes through
// registers, every load of the window is in flight at once and the wave waits
// once.  Pairs with no node entry (k' outside [-1, m2]) and pairs of columns
// past a ragged tile's halo are not loaded (their slots are never read); a
// pair with one node entry reads one neighbouring element of the field array
// that is never used (its address is clamped into the array).
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) void lds_void;

// LDS bytes of a staged tile: the window's slot pairs
__host__ __device__ inline int stage_bytes(int tk) { return kTC * kTC * tile_pitch(tk) * 8; }

// LDS slot of entry kk of a column (the mirror for sweeps with s2 < 0)
template <int S2>
__device__ __forceinline__ int slot_of(int kk, int Lp) {
    return S2 > 0 ? kk : Lp - 1 - kk;
}

// Absolute index along axis a of staged column/row ci (0 = upstream halo):
// origin + sgn * ci.
template <int SGN>
__device__ __forceinline__ int stage_origin(const Geo& G, int a, int T) {
    return SGN > 0 ? T * kBI : G.n[a] - 1 - T * kBI;
}

// xlo, xhi: the element range of the field array around fld that may be read.
// Load r covers columns cb = r cpi .. cb + cpi - 1 (cpi = 64 / (Lp / 2));
// lane l takes slots q, q + 1 (q = 2 (l % (Lp / 2))) of column cb + l / (Lp / 2)
// (lanes past cpi whole columns stay idle).  Per lane the loop keeps that
// column's (ci, cj), y = the element of its lower slot, and d = the k' test
// value of the pair, each advanced by a constant per load plus a carry when cj
// wraps.  Offsets are 32-bit: the host keeps N below 2^31, and a loaded pair
// lies in [-1, N] around fld.
template <int DIR>
__device__ __forceinline__ void stage_tile(const Geo& G, const TileCtx& c, const double* __restrict__ fld,
                                           long long xlo, long long xhi, double* lds) {
    using D = Dir<DIR>;
    constexpr int sg = D::s2;
    const int Lp = tile_pitch(G.tk);
    const int hp = Lp >> 1, cpi = 64 / hp;
    const int si = (int)G.si, sj = (int)G.sj;
    const int oi = stage_origin<D::s0>(G, 0, c.TI), oj = stage_origin<D::s1>(G, 1, c.TJ);
    const int lo = (int)(xlo > -1 ? xlo : -1), hi = (int)(xhi < G.N ? xhi : G.N);
    const int dc = c.lane / hp, q = 2 * (c.lane - dc * hp);
    const bool lane_on = dc < cpi;
    int ci = dc / kTC, cj = dc - ci * kTC;
    // lower slot q holds entry kk = q (s2 > 0) or Lp - 1 - q (s2 < 0) of the
    // column, node k' = kq0 - ci - cj + kk at element kbase + s2 k'; the pair
    // holds a node entry iff its lower entry's k' + (2 or 1) lies in [0, m2 + 2]
    const int x0 = c.kbase + sg * c.kq0 + (sg > 0 ? 0 : 1 - Lp);
    const int ka0 = sg > 0 ? c.kq0 + 2 : c.kq0 + Lp;
    // (unsigned: columns outside the grid, never loaded, may leave the int range)
    unsigned y = (unsigned)(oi + D::s0 * ci) * si + (unsigned)(oj + D::s1 * cj) * sj - sg * (ci + cj) + x0 + q;
    int d = ka0 - (ci + cj) + sg * q;
    const unsigned kspan = (unsigned)G.m[2] + 2;
    const int ei = c.ext_i + 2, ej = c.ext_j + 2;
    const unsigned dy = (unsigned)cpi * (unsigned)(D::s1 * sj - sg);
    const unsigned dy_w = (unsigned)(D::s0 * si) - (unsigned)(kTC * D::s1 * sj) + sg * (kTC - 1);
    lds_char* lb = (lds_char*)lds;  // the dynamic shared array, in the LDS address space
    for (int cb = 0; cb < kTC * kTC; cb += cpi) {
        if (lane_on && ci < ei && cj < ej && (unsigned)d <= kspan) {
            const int x = min(max((int)y, lo), hi);
            __builtin_amdgcn_global_load_lds(fld + x, (lds_void*)(lb + 16 * cb * hp), 16, 0, 0);
        }
        cj += cpi;
        y += dy;
        d -= cpi;
        // one wrap (taken as selects) unless cpi >= kTC (pitches below 14)
        const bool wrap = cj >= kTC;
        cj -= wrap ? kTC : 0;
        ci += wrap ? 1 : 0;
        y += wrap ? dy_w : 0u;
        d += wrap ? kTC - 1 : 0;
        if (cpi >= kTC) {
            while (cj >= kTC) {
                cj -= kTC;
                ++ci;
                y += dy_w;
                d += kTC - 1;
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // every load of the window (and any earlier one) has landed
}

// Write back the tile's own nodes: entries 1..tk of its columns whose k' is
// an interior node (the others are halo or outside the column).  The columns
// are taken as the full 8 x 8 (those past a ragged tile's end are skipped)
// in chunks of 16 entries: in chunk ch, lane (g, r) = (lane / 16, lane % 16)
// takes entry q + 1, q = ch + r, of own column (li, lj) = (u / 2, 4 (u % 2) + g)
// at step u = 0..15.  A step's element offset and LDS slot then differ from
// the lane's first ones by a wave-uniform amount, and every LDS read of a
// chunk is issued before its stores.  (Reads of skipped entries stay inside
// the window: their slots lie less than 16 past either end of an own
// column, and the columns beside it in LDS are staged ones.)
template <int DIR>
__device__ __forceinline__ void unstage_tile(const Geo& G, const TileCtx& c, double* __restrict__ fld,
                                             const double* lds, int Lp) {
    using D = Dir<DIR>;
    constexpr int sg = D::s2;
    const int ek = G.tk;
    const int si = D::s0 * (int)G.si, sj = D::s1 * (int)G.sj;
    const int base = (int)nidx(G, stage_origin<D::s0>(G, 0, c.TI) + D::s0, stage_origin<D::s1>(G, 1, c.TJ) + D::s1,
                               c.kbase);
    const unsigned kmax = (unsigned)G.m[2];
    const int g = c.lane >> 4, r = c.lane & 15;
    const bool colj0 = g < c.ext_j, colj1 = g + 4 < c.ext_j;
    // node (li, lj, entry q + 1): element base + li si + lj sj + s2 k', with
    // k' = kq0 - 1 - li - lj + q, and slot ((li + 1) kTC + lj + 1) Lp + q + 1
    // (mirrored: Lp - 2 - q)
    const unsigned xa = (unsigned)(si - sg), xb = 4u * (unsigned)(sj - sg);
    const int la = kTC * Lp, lb = 4 * Lp;
    for (int ch = 0; ch < ek; ch += 16) {
        const int q = ch + r;
        // (unsigned: lanes past the tile's entries, never stored, may leave the int range)
        const unsigned x0 = (unsigned)base + (unsigned)(sg * (c.kq0 - 1 + q)) + (unsigned)g * (unsigned)(sj - sg);
        const int l0 = (kTC + g + 1) * Lp + (sg > 0 ? 1 : Lp - 2) + sg * q;
        const int kp0 = c.kq0 - 1 - g + q;
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            v[u] = lds[l0 + __builtin_amdgcn_readfirstlane((u >> 1) * la + (u & 1) * lb)];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int li = u >> 1, b = u & 1;
            if (li < c.ext_i && (b ? colj1 : colj0) && q < ek && (unsigned)(kp0 - li - 4 * b) < kmax)
                fld[(int)(x0 + (unsigned)__builtin_amdgcn_readfirstlane((int)((unsigned)li * xa + (unsigned)b * xb)))] =
                    v[u];
        }
    }
}

// Forward sweeps: a boundary node on a k face only (its column is interior)
// copies the column's interior end node k' = 0 or m2 - 1 (the boundary rule
// copies the inward neighbour along the last boundary axis, here k).  Nothing
// else in a sweep reads or writes it, so the tile that finalises the end node
// sets it right after its walk, next to the column it has just written back;
// the boundary pass skips those nodes (strided ones: each sits in a cache line
// of its own) and the change joins the tile's convergence sum.  (The adjoint
// keeps them in its boundary pass: its value also needs the node's right-hand
// side and coupling, loaded after the walk, which cost the sweep more than the
// pass saved.)
template <int DIR>
__device__ __forceinline__ void fwd_kface_nodes(const Geo& G, const Src& S, const TileCtx& c, double* __restrict__ fld,
                                                const double* lds, int own, int Lp, double& eps) {
    using D = Dir<DIR>;
    constexpr int sg = D::s2;
    if (!c.colv) return;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int kin = e == 0 ? 0 : G.m[2] - 1;                // the interior end node's k'
        const int t = kin - c.kp0;                              // the step that updated it
        if (t < c.t0 || t >= c.t1) continue;
        const int kb = c.kbase + sg * (e == 0 ? -1 : G.m[2]);  // absolute k of the boundary node
        if (in_fixed(S, c.i, c.j, kb)) continue;
        const int o = sg > 0 ? own + t : own + Lp - 1 - t;
        const double nv = lds[o + sg];                       // entry t + 1: the end node
        const double old = lds[e == 0 ? o : o + 2 * sg];     // entry t or t + 2: the boundary node
        fld[nidx(G, c.i, c.j, kb)] = nv;
        eps += fabs(nv - old);
    }
}

// The per-node records a step needs (model, table) are loaded kPre steps
// ahead into a ring slot indexed by the wave-uniform step number.
constexpr int kPre = 4;       // forward: steps are long (the full update)
constexpr int kPreAdj = 6;    // adjoint: short steps, so look further ahead

struct FwdSlot {
    double sx, ma, mb, mc, c2, s2;  // s, the anisotropy block (1 - 2 xi, 2 eta, 1 + 2 xi), axis-2 table
};

// unconditional: k' is clamped into the lane's range in the tile, so the address is always valid
template <int DIR>
__device__ __forceinline__ void fwd_fetch(const TileCtx& c, const double* __restrict__ mdl,
                                          const double2* __restrict__ t2, int t, FwdSlot& r) {
    // the step clamped to the lane's k' range; |rstep| = n1p < 2^23 and the
    // step is below 64, so the product is a 24-bit one
    const int tc = min(max(t, c.tlo), c.thi);
    const unsigned ri = (unsigned)(c.rr0 + __mul24(c.rstep, tc));
    const double2* m = reinterpret_cast<const double2*>(mdl + (size_t)ri * 4);
    const double2 m0 = m[0], m1 = m[1];
    r.sx = m0.x;
    r.ma = m0.y;
    r.mb = m1.x;
    r.mc = m1.y;
    const double2 tv = t2[(unsigned)(c.tt0 + Dir<DIR>::s2 * tc)];
    r.c2 = tv.x;
    r.s2 = tv.y;
}

// TKC: the tile depth as a compile-time constant (0: read from the geometry),
// so that LDS offsets become immediates and the staging and write-back index
// arithmetic folds; the host picks an instance whose TKC equals the depth.
template <int COORD, int DIR, int TKC>
__global__ void __launch_bounds__(64) k_fwd_sweep(SweepArgs a, int plane, int s0) {
    using D = Dir<DIR>;
    extern __shared__ double lds[];
    const int src = blockIdx.x;
    if (!a.active[src]) return;
    Geo G = a.G;
    if (TKC > 0) G.tk = TKC;
    const Src S = a.src[src];
    const TileCtx c = tile_ctx<DIR>(G, S, plane, s0);
    if (c.t1 <= c.t0) {  // a ragged column's slab with no nodes
        if (c.lane == 0) a.part[(long long)src * a.nslots + DIR * G.ntiles + c.slot] = 0.0;
        return;
    }
    const Col cl = make_col(G, a.T, c.i, c.j);
    const LfCol W = lf_col<COORD>(G, S, cl, a.kappa);
    double* __restrict__ fld = a.field + (long long)src * G.N;
    const double* __restrict__ mdl = a.model + (long long)D::lay * G.Sa * 4;
    const double2* __restrict__ t2 = a.T.t2;
    const int Lp = tile_pitch(G.tk);
    const int kmax = G.m[2];

    FwdSlot ring[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) fwd_fetch<DIR>(c, mdl, t2, c.t0 + u, ring[u]);
    stage_tile<DIR>(G, c, fld, -(long long)src * G.N, (long long)(a.nsrc - src) * G.N - 2, lds);
    __syncthreads();

    const int own = ((c.li + 1) * kTC + c.lj + 1) * Lp;
    double eps = 0.0;
    // the step count is padded to a multiple of kPre: no branch encloses a load
    for (int tb = c.t0; tb < c.t1; tb += kPre) {
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int t = tb + u;
            {
                FwdSlot& r = ring[u];
                const int kp = c.kp0 + t;
                if (c.colv && t < c.t1 && (unsigned)kp < (unsigned)kmax) {
                    const int ka = c.kbase + D::s2 * kp;
                    if (!(c.fcol && (unsigned)(ka - S.fb[2]) <= 1u)) {
                        // sweep-relative neighbours: "up" = already updated this sweep
                        // slot of entry t (mirrored columns when s2 < 0): entry t + 1 is at o + s2
                        constexpr int sg = D::s2;
                        const int o = sg > 0 ? own + t : own + Lp - 1 - t;
                        const double cur = lds[o + sg];
                        const double up_i = lds[o - kTC * Lp], dn_i = lds[o + kTC * Lp + 2 * sg];
                        const double up_j = lds[o - Lp], dn_j = lds[o + Lp + 2 * sg];
                        const double up_k = lds[o], dn_k = lds[o + 2 * sg];
                        const double m0 = D::s0 > 0 ? up_i : dn_i, p0 = D::s0 > 0 ? dn_i : up_i;
                        const double m1 = D::s1 > 0 ? up_j : dn_j, p1 = D::s1 > 0 ? dn_j : up_j;
                        const double m2 = D::s2 > 0 ? up_k : dn_k, p2 = D::s2 > 0 ? dn_k : up_k;
                        const double nv = lf_update<COORD>(G, S, cl, W, r.c2, r.s2, r.sx, r.ma, r.mb, r.mc, cur, m0,
                                                           p0, m1, p1, m2, p2);
                        lds[o + sg] = nv;
                        eps += fabs(nv - cur);
                    }
                }
                fwd_fetch<DIR>(c, mdl, t2, t + kPre, r);
            }
        }
    }
    __syncthreads();
    unstage_tile<DIR>(G, c, fld, lds, Lp);
    fwd_kface_nodes<DIR>(G, S, c, fld, lds, own, Lp, eps);
    eps = wave_sum(eps);
    if (c.lane == 0) a.part[(long long)src * a.nslots + DIR * G.ntiles + c.slot] = eps;
}

// model records (s, 1 - 2 xi, 2 eta, 1 + 2 xi) in the four aligned layouts
__global__ void k_model_records(Geo G, const double* __restrict__ s, const double* __restrict__ xi,
                                const double* __restrict__ eta, double* __restrict__ out) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= G.N) return;
    const int k = (int)(x % G.n[2]);
    const long long q = x / G.n[2];
    const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
    // the lower-right block of M = [[1 - 2 xi, 2 eta], [2 eta, 1 + 2 xi]]
    const double2 v0 = make_double2(s[x], 1.0 - 2.0 * xi[x]), v1 = make_double2(2.0 * eta[x], 1.0 + 2.0 * xi[x]);
    for (int lay = 0; lay < 4; ++lay) {
        double2* o = reinterpret_cast<double2*>(out + ((long long)lay * G.Sa + arec_idx(G, lay, i, j, k)) * 4);
        o[0] = v0;
        o[1] = v1;
    }
}

// Value of node p once the boundary pass is done: interior and fixed nodes as
// stored; a boundary node copies its inward neighbour along its largest
// boundary axis, which has one boundary axis fewer (depth <= 3).
template <int BUDGET>
__device__ __forceinline__ double fwd_bval(const Geo& G, const Src& S, const double* f, int i, int j, int k) {
    const int p[3] = {i, j, k};
    const int as = astar_of(G, p);
    if constexpr (BUDGET == 0) {
        return f[nidx(G, i, j, k)];
    } else {
        if (as < 0 || in_fixed(S, i, j, k)) return f[nidx(G, i, j, k)];
        int q1[3] = {i, j, k};
        q1[as] += (p[as] == 0) ? 1 : -1;
        return fwd_bval<BUDGET - 1>(G, S, f, q1[0], q1[1], q1[2]);
    }
}

__global__ void __launch_bounds__(kBndThreads) k_fwd_bnd(SweepArgs a, int dir) {
    __shared__ double sh[4];
    const int src = blockIdx.y;
    if (!a.active[src]) return;
    const Geo& G = a.G;
    const Src S = a.src[src];
    double* fld = a.field + (long long)src * G.N;
    const long long b = (long long)blockIdx.x * kBndThreads + threadIdx.x;
    double d = 0.0;
    if (b < G.NB) {
        int i, j, k;
        bnd_decode(G, b, i, j, k);
        // (the sweeps set the nodes on a k face only)
        if (!in_fixed(S, i, j, k) && !kface_only(G, i, j)) {
            const double nv = fwd_bval<3>(G, S, fld, i, j, k);
            const long long x = nidx(G, i, j, k);
            d = fabs(nv - fld[x]);
            fld[x] = nv;
        }
    }
    d = block_sum256(d, sh);
    if (threadIdx.x == 0) a.part[(long long)src * a.nslots + 8 * G.ntiles + dir * a.nbblocks + blockIdx.x] = d;
}

__device__ __forceinline__ double fixed_sum(const double* p, int cnt, double* sh) {
    double v = 0.0;
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) v += p[q];
    return block_sum256(v, sh);
}

__device__ __forceinline__ void finish_iteration(const SweepArgs& a, int src, double eps) {
    const int it = a.iter[src] + 1;
    a.iter[src] = it;
    if (a.eps_hist) a.eps_hist[(long long)src * a.hist_stride + (it - 1)] = eps;
    if (eps < a.tol) {
        a.status[src] = it;
        a.active[src] = 0;
        atomicSub(a.counter, 1);
    } else if (it >= a.max_iter) {
        a.status[src] = -it;
        a.active[src] = 0;
        atomicSub(a.counter, 1);
    } else {
        a.status[src] = -it;
    }
}

__global__ void __launch_bounds__(256) k_fwd_finalize(SweepArgs a) {
    __shared__ double sh[4];
    const int src = blockIdx.x;
    if (!a.active[src]) return;
    const double tot = fixed_sum(a.part + (long long)src * a.nslots, a.nslots, sh);
    if (threadIdx.x == 0) finish_iteration(a, src, tot / (double)a.G.N);
}

// --------------------------------------------------------- adjoint solve
// Local state at an arbitrary interior node, loading what it needs.
template <int COORD>
__device__ __forceinline__ void state_at(const Geo& G, const Tabs& T, const Src& S, const double* __restrict__ tau,
                                         const double* __restrict__ xi, const double* __restrict__ eta, int i,
                                         int j, int k, Col& c, Loc& L) {
    c = make_col(G, T, i, j);
    const long long x = nidx(G, i, j, k);
    const double2 t2 = T.t2[k];
    local_state<COORD>(G, S, c, t2.x, t2.y, xi[x], eta[x], tau[x], tau[x - G.si], tau[x + G.si], tau[x - G.sj],
                       tau[x + G.sj], tau[x - 1], tau[x + 1], L);
}

__device__ __forceinline__ double g_of(const Col& c, int a) { return a == 0 ? 1.0 : (a == 1 ? c.g1 : c.g2); }

// J_{x, x + dirn e_a} of an interior non-fixed row x (dirn = +1 or -1):
//   alpha_a - beta_a or -alpha_a - beta_a with alpha_a = T0 g_a (MP)_a / (2 h_a H),
//   beta_a = kappa T0 g_a / (2 h_a).
__device__ __forceinline__ double row_off(const Geo& G, const Col& c, const Loc& L, double kappa, int a, int dirn) {
    const double ga = g_of(c, a);
    const double alpha = L.T0 * ga * L.MP[a] / (2.0 * G.h[a] * L.H);
    const double beta = kappa * L.T0 * ga / (2.0 * G.h[a]);
    return dirn > 0 ? alpha - beta : -alpha - beta;
}

// Adjoint coefficient records: the six couplings of a node's column equation
// divided by its diagonal (48 bytes).  Default: four line-aligned
// row-coalesced layouts per source (arec_idx), so the 8 records a tile row
// reads on one step are whole 128-byte lines in every sweep direction.
// Compact (TT_FLAG_COMPACT_ADJOINT): one copy per source in node order
// [nsrc][N][6], a ninth of the memory at 101^3; a lane's records for
// consecutive steps are then contiguous along its column, but a tile row's
// records lie on different lines.
constexpr int kRec = 6;

// store a node's row {c+_0, c-_0, c+_1, c-_1, c+_2, c-_2, diag, -} divided by
// its diagonal, the diagonal into diag_all, and a zero right-hand side
// (k_adj_rhs adds to it); a zero diagonal (no row) stores a zero record
__device__ __forceinline__ void store_record(const Geo& G, double* __restrict__ coef_all, double* __restrict__ diag_all,
                                             double* __restrict__ rhs_all, int src, long long x, int i, int j, int k,
                                             const double (&out)[8], int compact) {
    const double d = out[6];
    double2 rec[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
        rec[q] = d != 0.0 ? make_double2(out[2 * q] / d, out[2 * q + 1] / d) : make_double2(0.0, 0.0);
    diag_all[(long long)src * G.N + x] = d;
    rhs_all[(long long)src * G.N + x] = 0.0;
    if (compact) {
        double2* cf = reinterpret_cast<double2*>(coef_all + ((long long)src * G.N + x) * kRec);
#pragma unroll
        for (int q = 0; q < 3; ++q) cf[q] = rec[q];
        return;
    }
    for (int lay = 0; lay < 4; ++lay) {
        double2* cf =
            reinterpret_cast<double2*>(coef_all + (((long long)src * 4 + lay) * G.Sa + arec_idx(G, lay, i, j, k)) * kRec);
#pragma unroll
        for (int q = 0; q < 3; ++q) cf[q] = rec[q];
    }
}

// Coefficients of the transposed system at every node of every source, stored
// as the column equation of x divided by its diagonal
// J_xx: record {in+_0, in-_0, in+_1, in-_1, in+_2, in-_2} / J_xx, with
// in+-_a = J_{x +- e_a, x}, the coefficient of lambda(x +- e_a) (zero unless x
// is interior and not fixed).  J_xx goes to diag [nsrc][N] (0 where there is
// no row); the right-hand side, divided likewise, is added to rhs [nsrc][N] by
// k_adj_rhs.  bnd_in[b] = J_{x, b} for each face node b and its interior
// neighbour x (zero when x is fixed).
template <int COORD>
__global__ void __launch_bounds__(256) k_adj_coef(SweepArgs a, const double* __restrict__ tau_all,
                                                  double* __restrict__ coef_all, double* __restrict__ bnd_all,
                                                  double* __restrict__ diag_all, double* __restrict__ rhs_all) {
    const Geo& G = a.G;
    const int src = blockIdx.y;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= G.N) return;
    const Src S = a.src[src];
    const double* tau = tau_all + (long long)src * G.N;
    const int k = (int)(x % G.n[2]);
    const long long q = x / G.n[2];
    const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
    double out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool interior = i > 0 && i < G.n[0] - 1 && j > 0 && j < G.n[1] - 1 && k > 0 && k < G.n[2] - 1;
    if (interior && !in_fixed(S, i, j, k)) {
        Col c;
        Loc L;
        state_at<COORD>(G, a.T, S, tau, a.xi, a.eta, i, j, k, c, L);
        double diag = (L.t[0] * L.MP[0] + L.t[1] * L.MP[1] + L.t[2] * L.MP[2]) / L.H;
        for (int ax = 0; ax < 3; ++ax) diag += 2.0 * (a.kappa * L.T0 * g_of(c, ax) / (2.0 * G.h[ax]));
        out[6] = diag;
        for (int ax = 0; ax < 3; ++ax) {
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int dirn = sgn == 0 ? 1 : -1;
                int y[3] = {i, j, k};
                y[ax] += dirn;
                double v = 0.0;
                if (!in_fixed(S, y[0], y[1], y[2])) {
                    if (on_bnd(G, ax, y[ax])) {
                        v = -1.0;  // the face row of y copies x
                    } else {
                        Col cy;
                        Loc Ly;
                        state_at<COORD>(G, a.T, S, tau, a.xi, a.eta, y[0], y[1], y[2], cy, Ly);
                        v = row_off(G, cy, Ly, a.kappa, ax, -dirn);
                    }
                }
                out[2 * ax + sgn] = v;
                if (on_bnd(G, ax, y[ax]))
                    bnd_all[(long long)src * G.NB + bnd_encode(G, y[0], y[1], y[2])] =
                        row_off(G, c, L, a.kappa, ax, dirn);
            }
        }
    }
    store_record(G, coef_all, diag_all, rhs_all, src, x, i, j, k, out, a.compact);
}

// d chi / d tau = sum_m R_m w_c T0(c) (discrete adjoint), or the point sources
// sum_m R_m w_c of Eq. (5) (continuous adjoint, with_t0 = 0), added in receiver
// order (one thread per source: deterministic)
template <int COORD>
__global__ void k_adj_rhs(SweepArgs a, const double* __restrict__ diag_all, double* __restrict__ rhs_all,
                          int* __restrict__ box_all, int nrec, const double* __restrict__ rec,
                          const double* __restrict__ R, int with_t0) {
    const int src = blockIdx.x * blockDim.x + threadIdx.x;
    if (src >= a.nsrc) return;
    const Geo& G = a.G;
    const Src S = a.src[src];
    const double* dg = diag_all + (long long)src * G.N;
    double* rh = rhs_all + (long long)src * G.N;
    int lo[3] = {G.n[0], G.n[1], G.n[2]}, hi[3] = {-1, -1, -1};
    double* brhs = const_cast<double*>(a.bnd_rhs) + (long long)src * G.NB;
    for (int m = 0; m < nrec; ++m) {
        const Tri t = tri_of(G, rec[3 * m], rec[3 * m + 1], rec[3 * m + 2]);
        const double r = R[(long long)src * nrec + m];
        for (int c0 = 0; c0 < 2; ++c0)
            for (int c1 = 0; c1 < 2; ++c1)
                for (int c2 = 0; c2 < 2; ++c2) {
                    const int i = t.b[0] + c0, j = t.b[1] + c1, k = t.b[2] + c2;
                    const Col c = make_col(G, a.T, i, j);
                    const double2 t2 = a.T.t2[k];
                    double T0, tt[3];
                    factor<COORD>(S, c, t2.x, t2.y, T0, tt);
                    const double v = with_t0 ? r * tri_w(t, c0, c1, c2) * T0 : r * tri_w(t, c0, c1, c2);
                    // divided by the row's diagonal like the records (a row-less node's
                    // value is never read by the sweeps)
                    const long long xn = nidx(G, i, j, k);
                    const double d = dg[xn];
                    rh[xn] += d != 0.0 ? v / d : v;
                    const int id[3] = {i, j, k};
                    for (int ax = 0; ax < 3; ++ax) {
                        lo[ax] = min(lo[ax], id[ax]);
                        hi[ax] = max(hi[ax], id[ax]);
                    }
                    if (on_bnd(G, 0, i) || on_bnd(G, 1, j) || on_bnd(G, 2, k))
                        brhs[bnd_encode(G, i, j, k)] += v;
                }
    }
    for (int ax = 0; ax < 3; ++ax) {
        box_all[src * 6 + 2 * ax] = lo[ax];
        box_all[src * 6 + 2 * ax + 1] = hi[ax];
    }
}

// a step's record (and, in tiles that meet the source's right-hand side, its
// right-hand side value), fetched kPreAdj steps ahead
struct AdjSlot {
    double r[kRec];
    double b;
};

template <int DIR, bool RHS, bool COMPACT>
__device__ __forceinline__ void adj_fetch(const TileCtx& c, const double* __restrict__ cf,
                                          const double* __restrict__ rh, long long xb, int t, AdjSlot& r) {
    using D = Dir<DIR>;
    const int kp = min(max(c.kp0 + t, c.kplo), c.kphi);
    const long long x = xb + D::s2 * kp;
    // |rstep| = n1p < 2^23 and 0 <= kp < n2 <= 8192: a 24-bit product
    const double2* rc =
        reinterpret_cast<const double2*>(cf + (COMPACT ? x : (long long)(c.rbase + __mul24(c.rstep, kp))) * kRec);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double2 v = rc[q];
        r.r[2 * q] = v.x;
        r.r[2 * q + 1] = v.y;
    }
    r.b = RHS ? rh[x] : 0.0;
}

// does the tile (its columns, and the k' range of its slab) meet the index box
// of the source's nonzero right-hand side?
template <int DIR>
__device__ __forceinline__ bool tile_meets_box(const Geo& G, const TileCtx& c, const int* bx) {
    using D = Dir<DIR>;
    const int i0 = 8 * c.TI, i1 = 8 * c.TI + c.ext_i - 1, j0 = 8 * c.TJ, j1 = 8 * c.TJ + c.ext_j - 1;
    const int kq0 = max(0, c.TK * G.tk - i1 - j1), kq1 = min(G.m[2] - 1, c.TK * G.tk + G.tk - 1 - i0 - j0);
    const int ia = D::s0 > 0 ? 1 + i0 : G.n[0] - 2 - i1, ib = D::s0 > 0 ? 1 + i1 : G.n[0] - 2 - i0;
    const int ja = D::s1 > 0 ? 1 + j0 : G.n[1] - 2 - j1, jb = D::s1 > 0 ? 1 + j1 : G.n[1] - 2 - j0;
    const int ka = D::s2 > 0 ? 1 + kq0 : G.n[2] - 2 - kq1, kb = D::s2 > 0 ? 1 + kq1 : G.n[2] - 2 - kq0;
    return ia <= bx[1] && ib >= bx[0] && ja <= bx[3] && jb >= bx[2] && ka <= bx[5] && kb >= bx[4] && kq0 <= kq1;
}

template <int DIR, bool RHS, bool COMPACT>
__device__ __forceinline__ void adj_tile(const SweepArgs& a, const Geo& G, const Src& S, const TileCtx& c, int src,
                                         double* lds) {
    using D = Dir<DIR>;
    constexpr bool last = (DIR == 7);
    double* __restrict__ fld = a.field + (long long)src * G.N;
    const double* __restrict__ cf =
        a.coef + (COMPACT ? (long long)src * G.N : ((long long)src * 4 + D::lay) * G.Sa) * kRec;
    const double* __restrict__ rh = a.rhs + (long long)src * G.N;
    const long long xb = nidx(G, c.i, c.j, c.kbase);
    const int Lp = tile_pitch(G.tk);
    const int kmax = G.m[2];

    AdjSlot ring[kPreAdj];
#pragma unroll
    for (int u = 0; u < kPreAdj; ++u) adj_fetch<DIR, RHS, COMPACT>(c, cf, rh, xb, c.t0 + u, ring[u]);
    stage_tile<DIR>(G, c, fld, -(long long)src * G.N, (long long)(a.nsrc - src) * G.N - 2, lds);
    __syncthreads();

    const int own = ((c.li + 1) * kTC + c.lj + 1) * Lp;
    double dsum = 0.0, asum = 0.0;
    // the step count is padded to a multiple of kPreAdj: no branch encloses a load
    for (int tb = c.t0; tb < c.t1; tb += kPreAdj) {
#pragma unroll
        for (int u = 0; u < kPreAdj; ++u) {
            const int t = tb + u;
            {
                AdjSlot& r = ring[u];
                const int kp = c.kp0 + t;
                if (c.colv && t < c.t1 && (unsigned)kp < (unsigned)kmax) {
                    const int ka = c.kbase + D::s2 * kp;
                    if (!(c.fcol && (unsigned)(ka - S.fb[2]) <= 1u)) {
                        // slot of entry t (mirrored columns when s2 < 0): entry t + 1 is at o + s2
                        constexpr int sg = D::s2;
                        const int o = sg > 0 ? own + t : own + Lp - 1 - t;
                        const double cur = lds[o + sg];
                        const double up_i = lds[o - kTC * Lp], dn_i = lds[o + kTC * Lp + 2 * sg];
                        const double up_j = lds[o - Lp], dn_j = lds[o + Lp + 2 * sg];
                        const double up_k = lds[o], dn_k = lds[o + 2 * sg];
                        // record: coefficients of lambda(x + e_a), lambda(x - e_a) at 2a, 2a + 1,
                        // divided by the diagonal like the right-hand side.  The
                        // sweep-downstream terms (values of the previous sweep) go first, the
                        // upstream ones (updated on the previous step) last.
                        constexpr int di = D::s0 > 0 ? 0 : 1, dj = D::s1 > 0 ? 2 : 3, dk = D::s2 > 0 ? 4 : 5;
                        double acc = r.b;
                        acc -= r.r[di] * dn_i;
                        acc -= r.r[dj] * dn_j;
                        acc -= r.r[dk] * dn_k;
                        acc -= r.r[di ^ 1] * up_i;
                        acc -= r.r[dj ^ 1] * up_j;
                        acc -= r.r[dk ^ 1] * up_k;
                        const double nv = acc;
                        lds[o + sg] = nv;
                        dsum += fabs(nv - cur);
                        if (last) asum += fabs(nv);
                    }
                }
                adj_fetch<DIR, RHS, COMPACT>(c, cf, rh, xb, t + kPreAdj, r);
            }
        }
    }
    __syncthreads();
    unstage_tile<DIR>(G, c, fld, lds, Lp);
    dsum = wave_sum(dsum);
    asum = wave_sum(asum);
    if (c.lane == 0) {
        a.part[(long long)src * a.nslots + DIR * G.ntiles + c.slot] = dsum;
        if (last) a.part2[(long long)src * a.nslots + c.slot] = asum;
    }
}

// TKC: compile-time tile depth as for k_fwd_sweep (0: from the geometry)
template <int COORD, int DIR, bool COMPACT, int TKC>
__global__ void __launch_bounds__(64) k_adj_sweep(SweepArgs a, int plane, int s0) {
    extern __shared__ double lds[];
    const int src = blockIdx.x;
    if (!a.active[src]) return;
    Geo G = a.G;
    if (TKC > 0) G.tk = TKC;
    const Src S = a.src[src];
    const TileCtx c = tile_ctx<DIR>(G, S, plane, s0);
    if (c.t1 <= c.t0) {  // a ragged column's slab with no nodes
        if (c.lane == 0) {
            a.part[(long long)src * a.nslots + DIR * G.ntiles + c.slot] = 0.0;
            if (DIR == 7) a.part2[(long long)src * a.nslots + c.slot] = 0.0;
        }
        return;
    }
    // wave-uniform: only tiles that meet the right-hand side read it
    if (tile_meets_box<DIR>(G, c, a.box + src * 6)) adj_tile<DIR, true, COMPACT>(a, G, S, c, src, lds);
    else adj_tile<DIR, false, COMPACT>(a, G, S, c, src, lds);
}

// Transposed boundary pass: lambda_b = rhs_b - sum_{rows r != b} J_{r, b} lambda_r,
// rhs_b read from the compact per-boundary-node copy (bnd_rhs).
// The rows that reference a boundary node b are its interior neighbour (face
// nodes only, coefficient bnd_in[b]) and boundary rows b' that copy b along an
// axis a' above a*(b) (b' one step outward along a', coefficient -1);
// lambda(b') is evaluated in place (a* grows strictly: depth <= 3).
template <int BUDGET>
__device__ double adj_bval(const Geo& G, const Src& S, const double* lam, const double* brhs, const double* bin,
                           int i, int j, int k) {
    const int p[3] = {i, j, k};
    const int as = astar_of(G, p);
    double acc = brhs[bnd_encode(G, i, j, k)];
    const int nb = (int)on_bnd(G, 0, i) + (int)on_bnd(G, 1, j) + (int)on_bnd(G, 2, k);
    if (nb == 1) {
        int x[3] = {i, j, k};
        x[as] += (p[as] == 0) ? 1 : -1;
        acc -= bin[bnd_encode(G, i, j, k)] * lam[nidx(G, x[0], x[1], x[2])];
    }
    if constexpr (BUDGET > 0) {
        for (int ap = as + 1; ap < 3; ++ap) {
            const int id = p[ap];
            if (on_bnd(G, ap, id)) continue;
            for (int side = 0; side < 2; ++side) {
                const int dist = side == 0 ? id : (G.n[ap] - 1 - id);
                if (dist != 1) continue;
                int q[3] = {i, j, k};
                q[ap] = side == 0 ? 0 : G.n[ap] - 1;
                if (in_fixed(S, q[0], q[1], q[2])) continue;
                acc += adj_bval<BUDGET - 1>(G, S, lam, brhs, bin, q[0], q[1], q[2]);
            }
        }
    }
    return acc;
}

__global__ void __launch_bounds__(kBndThreads) k_adj_bnd(SweepArgs a, int dir) {
    __shared__ double sh[4];
    const int src = blockIdx.y;
    if (!a.active[src]) return;
    const Geo& G = a.G;
    const Src S = a.src[src];
    double* lam = a.field + (long long)src * G.N;
    const double* brhs = a.bnd_rhs + (long long)src * G.NB;
    const double* bin = a.bnd_in + (long long)src * G.NB;
    const long long b = (long long)blockIdx.x * kBndThreads + threadIdx.x;
    double d = 0.0, av = 0.0;
    if (b < G.NB) {
        int i, j, k;
        bnd_decode(G, b, i, j, k);
        if (!in_fixed(S, i, j, k)) {
            const double nv = adj_bval<2>(G, S, lam, brhs, bin, i, j, k);
            const long long x = nidx(G, i, j, k);
            d = fabs(nv - lam[x]);
            av = fabs(nv);
            lam[x] = nv;
        }
    }
    d = block_sum256(d, sh);
    const double as = (dir == 7) ? block_sum256(av, sh) : 0.0;
    if (threadIdx.x == 0) {
        a.part[(long long)src * a.nslots + 8 * G.ntiles + dir * a.nbblocks + blockIdx.x] = d;
        if (dir == 7) a.part2[(long long)src * a.nslots + G.ntiles + blockIdx.x] = as;
    }
}

__global__ void __launch_bounds__(256) k_adj_finalize(SweepArgs a) {
    __shared__ double sh[4];
    const int src = blockIdx.x;
    if (!a.active[src]) return;
    const double dtot = fixed_sum(a.part + (long long)src * a.nslots, a.nslots, sh);
    const double atot = fixed_sum(a.part2 + (long long)src * a.nslots, a.G.ntiles + a.nbblocks, sh);
    if (threadIdx.x == 0) finish_iteration(a, src, dtot / (atot > 1e-300 ? atot : 1e-300));
}

// ------------------------------------------ continuous adjoint (Eq. (5))
// Upwind finite volumes for div(P w) = sum_m R_m delta(x - x_m), w = -M grad T.
// Each node owns the trapezoidal control volume around it; the flux leaves
// through six faces with the face velocity the mean of the two nodal normal
// components (the node's own on a grid face) and carries the upwind node's P.
// P = 0 on the fixed cell (the source absorbs) and outside the grid.

// w = -M p at any node, p the scaled gradient of T = T0 tau: central
// differences of tau along axes where the node is interior, one-sided where
// it lies on the grid face.
template <int COORD>
__device__ __forceinline__ void cadj_vel(const Geo& G, const Tabs& T, const Src& S, const double* __restrict__ tau,
                                         const double* __restrict__ xi, const double* __restrict__ eta, int i, int j,
                                         int k, double w[3]) {
    const Col c = make_col(G, T, i, j);
    const double2 t2 = T.t2[k];
    double T0, t[3];
    factor<COORD>(S, c, t2.x, t2.y, T0, t);
    const long long x = nidx(G, i, j, k);
    const int id[3] = {i, j, k};
    const long long st[3] = {G.si, G.sj, 1};
    const double tx = tau[x];
    double p[3];
#pragma unroll
    for (int a2 = 0; a2 < 3; ++a2) {
        double q;
        if (id[a2] == 0) q = (tau[x + st[a2]] - tx) * G.invh[a2];
        else if (id[a2] == G.n[a2] - 1) q = (tx - tau[x - st[a2]]) * G.invh[a2];
        else q = (tau[x + st[a2]] - tau[x - st[a2]]) * G.inv2h[a2];
        p[a2] = T0 * g_of(c, a2) * q + tx * t[a2];
    }
    const double xv = xi[x], ev = eta[x];
    w[0] = -p[0];
    w[1] = -((1.0 - 2.0 * xv) * p[1] + 2.0 * ev * p[2]);
    w[2] = -(2.0 * ev * p[1] + (1.0 + 2.0 * xv) * p[2]);
}

// control-volume extent of node index idx along axis a
__device__ __forceinline__ double cv_ext(const Geo& G, int a, int idx) {
    return (idx == 0 || idx == G.n[a] - 1) ? 0.5 * G.h[a] : G.h[a];
}

// Area of the face of node (i, j, k) normal to axis a at coordinate xf of that
// axis: r^2 cos(theta) dtheta dphi (r faces), r cos(theta) dr dphi (theta
// faces), r dr dtheta (phi faces); products of the other extents in Cartesian
// coordinates.
__device__ __forceinline__ double cadj_area(const Geo& G, int a, int i, int j, int k, double xf) {
    const int id[3] = {i, j, k};
    double A = 1.0;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if (b != a) A *= cv_ext(G, b, id[b]);
    if (G.coord == 1) {
        const double r = G.o[0] + i * G.h[0];
        if (a == 0) A *= xf * xf * cos(G.o[1] + j * G.h[1]);
        else if (a == 1) A *= r * cos(xf);
        else A *= r;
    }
    return A;
}

// Records of the continuous system in the adjoint layout (the row divided by
// its diagonal, store_record): c+-_a = A min(u_out, 0) couples P(x +- e_a)
// (0 when that node is fixed or outside), and the diagonal is the outflow
// sum A max(u_out, 0).  A node without outflow gets outflow = inf, so that its
// update is P = 0.
template <int COORD>
__global__ void __launch_bounds__(256) k_cadj_coef(SweepArgs a, const double* __restrict__ tau_all,
                                                   double* __restrict__ coef_all, double* __restrict__ diag_all,
                                                   double* __restrict__ rhs_all) {
    const Geo& G = a.G;
    const int src = blockIdx.y;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= G.N) return;
    const Src S = a.src[src];
    const double* tau = tau_all + (long long)src * G.N;
    const int k = (int)(x % G.n[2]);
    const long long q = x / G.n[2];
    const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
    double out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (!in_fixed(S, i, j, k)) {
        double w[3];
        cadj_vel<COORD>(G, a.T, S, tau, a.xi, a.eta, i, j, k, w);
        const int id[3] = {i, j, k};
        double diag = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const double xa = G.o[ax] + id[ax] * G.h[ax];
            for (int side = 0; side < 2; ++side) {
                const int sg = side == 0 ? 1 : -1;
                const int nb = id[ax] + sg;
                int y[3] = {i, j, k};
                y[ax] = nb;
                double u, A;
                const bool inside = nb >= 0 && nb < G.n[ax];
                if (inside) {
                    double wy[3];
                    cadj_vel<COORD>(G, a.T, S, tau, a.xi, a.eta, y[0], y[1], y[2], wy);
                    u = sg * 0.5 * (w[ax] + wy[ax]);
                    A = cadj_area(G, ax, i, j, k, 0.5 * (xa + (G.o[ax] + nb * G.h[ax])));
                } else {
                    u = sg * w[ax];
                    A = cadj_area(G, ax, i, j, k, xa);
                }
                diag += A * (u > 0.0 ? u : 0.0);
                out[2 * ax + side] = (inside && !in_fixed(S, y[0], y[1], y[2])) ? A * (u < 0.0 ? u : 0.0) : 0.0;
            }
        }
        out[6] = diag > 0.0 ? diag : HUGE_VAL;
    }
    store_record(G, coef_all, diag_all, rhs_all, src, x, i, j, k, out, a.compact);
}

// Boundary pass of the continuous system, Jacobi: every boundary node's new P
// from the values present before the pass, into tmp [nsrc][NB] ...
__global__ void __launch_bounds__(kBndThreads) k_cadj_bnd_calc(SweepArgs a, double* __restrict__ tmp_all) {
    const int src = blockIdx.y;
    if (!a.active[src]) return;
    const Geo& G = a.G;
    const long long b = (long long)blockIdx.x * kBndThreads + threadIdx.x;
    if (b >= G.NB) return;
    const Src S = a.src[src];
    const double* P = a.field + (long long)src * G.N;
    const double* cf = a.coef + (long long)src * (a.compact ? G.N : 4 * G.Sa) * kRec;  // compact, or layout 0
    int i, j, k;
    bnd_decode(G, b, i, j, k);
    double nv = 0.0;
    if (!in_fixed(S, i, j, k)) {
        const long long x = nidx(G, i, j, k);
        const double* r = cf + (a.compact ? x : arec_idx(G, 0, i, j, k)) * kRec;  // the row divided by its diagonal
        const int id[3] = {i, j, k};
        const long long st[3] = {G.si, G.sj, 1};
        double acc = a.rhs[(long long)src * G.N + nidx(G, i, j, k)];
        for (int ax = 0; ax < 3; ++ax) {
            if (r[2 * ax] != 0.0 && id[ax] + 1 < G.n[ax]) acc -= r[2 * ax] * P[x + st[ax]];
            if (r[2 * ax + 1] != 0.0 && id[ax] > 0) acc -= r[2 * ax + 1] * P[x - st[ax]];
        }
        nv = acc;
    }
    tmp_all[(long long)src * G.NB + b] = nv;
}

// ... then written back, with the convergence sums in the boundary slots.
__global__ void __launch_bounds__(kBndThreads) k_cadj_bnd_store(SweepArgs a, const double* __restrict__ tmp_all,
                                                                int dir) {
    __shared__ double sh[4];
    const int src = blockIdx.y;
    if (!a.active[src]) return;
    const Geo& G = a.G;
    double* P = a.field + (long long)src * G.N;
    const long long b = (long long)blockIdx.x * kBndThreads + threadIdx.x;
    double d = 0.0, av = 0.0;
    if (b < G.NB) {
        int i, j, k;
        bnd_decode(G, b, i, j, k);
        const long long x = nidx(G, i, j, k);
        const double nv = tmp_all[(long long)src * G.NB + b];
        d = fabs(nv - P[x]);
        av = fabs(nv);
        P[x] = nv;
    }
    d = block_sum256(d, sh);
    const double as = (dir == 7) ? block_sum256(av, sh) : 0.0;
    if (threadIdx.x == 0) {
        a.part[(long long)src * a.nslots + 8 * G.ntiles + dir * a.nbblocks + blockIdx.x] = d;
        if (dir == 7) a.part2[(long long)src * a.nslots + G.ntiles + blockIdx.x] = as;
    }
}

// The continuous adjoint's P as the derivative it estimates: d chi / d s(x) =
// P s V (Eqs. (6), (9)), V the trapezoidal node volume.
__global__ void __launch_bounds__(256) k_cadj_scale(Geo G, const double* __restrict__ s, double* __restrict__ lam_all,
                                                    int nsrc) {
    const int src = blockIdx.y;
    double* lam = lam_all + (long long)src * G.N;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < G.N;
         x += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(x % G.n[2]);
        const long long q = x / G.n[2];
        const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
        lam[x] *= s[x] * node_volume(G, i, j, k);
    }
    (void)nsrc;
}

// --------------------------------------------------------- sampling etc.
template <int COORD>
__global__ void k_sample(Geo G, Tabs T, const Src* __restrict__ srcs, int nsrc, const double* __restrict__ tau_all,
                         int nrec, const double* __restrict__ rec, double* __restrict__ out) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)nsrc * nrec) return;
    const int src = (int)(q / nrec), m = (int)(q % nrec);
    const Src S = srcs[src];
    const double* tau = tau_all + (long long)src * G.N;
    const Tri t = tri_of(G, rec[3 * m], rec[3 * m + 1], rec[3 * m + 2]);
    double acc = 0.0;
    for (int c0 = 0; c0 < 2; ++c0)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int c2 = 0; c2 < 2; ++c2) {
                const int i = t.b[0] + c0, j = t.b[1] + c1, k = t.b[2] + c2;
                const Col c = make_col(G, T, i, j);
                const double2 t2 = T.t2[k];
                double T0, tt[3];
                factor<COORD>(S, c, t2.x, t2.y, T0, tt);
                acc += tri_w(t, c0, c1, c2) * T0 * tau[nidx(G, i, j, k)];
            }
    out[q] = acc;
}

template <int COORD>
__global__ void __launch_bounds__(256) k_kernel_accum(Geo G, Tabs T, const Src* __restrict__ srcs, int nsrc,
                                                      const double* __restrict__ xi, const double* __restrict__ eta,
                                                      const double* __restrict__ tau_all,
                                                      const double* __restrict__ lam_all, double* __restrict__ grad,
                                                      int accumulate) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= G.N) return;
    const int k = (int)(x % G.n[2]);
    const long long q = x / G.n[2];
    const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
    double gs = 0.0, gx = 0.0, ge = 0.0;
    const bool interior = i > 0 && i < G.n[0] - 1 && j > 0 && j < G.n[1] - 1 && k > 0 && k < G.n[2] - 1;
    if (interior) {
        for (int n = 0; n < nsrc; ++n) {
            const Src S = srcs[n];
            if (in_fixed(S, i, j, k)) continue;
            const double l = lam_all[(long long)n * G.N + x];
            Col c;
            Loc L;
            state_at<COORD>(G, T, S, tau_all + (long long)n * G.N, xi, eta, i, j, k, c, L);
            gs += l;
            gx += l * (L.P[1] * L.P[1] - L.P[2] * L.P[2]) / L.H;
            ge += -2.0 * l * L.P[1] * L.P[2] / L.H;
        }
    }
    if (accumulate) {
        grad[x] += gs; grad[G.N + x] += gx; grad[2 * G.N + x] += ge;
    } else {
        grad[x] = gs; grad[G.N + x] = gx; grad[2 * G.N + x] = ge;
    }
}

// ---------------------------------------------------------------- launchers

SweepArgs make_args(const Plan& P, const double* s, const double* xi, const double* eta, double* field,
                    int32_t* status) {
    SweepArgs a;
    a.G = P.G;
    a.T = P.T;
    a.s = s; a.xi = xi; a.eta = eta;
    a.src = P.src;
    a.field = field;
    a.coef = P.coef;
    a.rhs = P.rhs;
    a.box = P.box;
    a.model = P.model;
    a.bnd_in = P.bnd_in;
    a.bnd_rhs = P.bnd_rhs;
    a.active = P.active;
    a.iter = P.iter;
    a.status = status;
    a.part = P.part;
    a.part2 = P.part2;
    a.counter = P.counter;
    a.eps_hist = P.eps_hist;
    a.nslots = P.nslots;
    a.nbblocks = P.nbblocks;
    a.nsrc = P.nsrc;
    a.compact = P.compact ? 1 : 0;
    a.max_iter = P.max_iter;
    a.hist_stride = P.hist_stride;
    a.kappa = P.kappa;
    a.tol = P.tol;
    return a;
}

void launch_tables(const Plan& P, hipStream_t st) {
    int n = P.G.n[0];
    if (P.G.n[1] > n) n = P.G.n[1];
    if (P.G.n[2] > n) n = P.G.n[2];
    hipLaunchKernelGGL(k_tables, dim3(blocks_for(n, 64)), dim3(64), 0, st, P.G, P.tab0, P.tab1, P.tab2);
}

void launch_src_setup(const Plan& P, const double* pos, const double* par, hipStream_t st) {
    hipLaunchKernelGGL(k_src_setup, dim3(blocks_for(P.nsrc, 64)), dim3(64), 0, st, P.G, pos, par, P.src, P.nsrc);
}

void launch_source_params(const Geo& G, const double* s, const double* xi, const double* eta, const double* pos,
                          double* par, int nsrc, hipStream_t st) {
    hipLaunchKernelGGL(k_source_params, dim3(blocks_for(nsrc, 64)), dim3(64), 0, st, G, s, xi, eta, pos, par, nsrc);
}


void launch_fwd_init(const Plan& P, const SweepArgs& a, const double* tau_init, const double* s, const double* xi,
                     const double* eta, hipStream_t st) {
    hipLaunchKernelGGL(k_model_records, dim3(blocks_for(P.G.N, 256)), dim3(256), 0, st, P.G, s, xi, eta, P.model);
    hipLaunchKernelGGL(k_solve_init, dim3(fill_blocks(P.G.N), P.nsrc), dim3(256), 0, st, a, tau_init, 1.0, 1.0);
}

static size_t tile_lds_bytes(const Geo& G) { return (size_t)stage_bytes(G.tk); }

// Event pair around the tile-plane launches of one directional sweep when
// timing is on; the launch count of the group is recorded with it.
struct TimedLaunch {
    const Plan& P;
    hipStream_t st;
    hipEvent_t e1 = nullptr;
    TimedLaunch(const Plan& p, hipStream_t s, int launches) : P(p), st(s) {
        if (P.timing) {
            hipEvent_t e0;
            if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
                (void)hipEventRecord(e0, st);
                P.timing->push_back({{e0, e1}, launches});
            } else {
                e1 = nullptr;
            }
        }
    }
    ~TimedLaunch() {
        if (P.timing && e1) (void)hipEventRecord(e1, st);
    }
};

// Sweep kernels are instantiated per coordinate system and direction.
typedef void (*SweepFn)(SweepArgs, int, int);

template <int COORD, int TKC, int... DS>
constexpr SweepFn pick_fwd(int d, std::integer_sequence<int, DS...>) {
    SweepFn t[] = {k_fwd_sweep<COORD, DS, TKC>...};
    return t[d];
}

template <int COORD, bool COMPACT, int TKC, int... DS>
constexpr SweepFn pick_adj(int d, std::integer_sequence<int, DS...>) {
    SweepFn t[] = {k_adj_sweep<COORD, DS, COMPACT, TKC>...};
    return t[d];
}

// forward sweep instances with a compile-time tile depth (the autotuner's
// usual choices); other depths run the generic instance
template <int COORD>
SweepFn fwd_sweep_fn_c(int tk, int d) {
    const auto seq = std::make_integer_sequence<int, 8>{};
    switch (tk) {
        case 16: return pick_fwd<COORD, 16>(d, seq);
        case 20: return pick_fwd<COORD, 20>(d, seq);
        case 24: return pick_fwd<COORD, 24>(d, seq);
        case 28: return pick_fwd<COORD, 28>(d, seq);
        default: return pick_fwd<COORD, 0>(d, seq);
    }
}

SweepFn fwd_sweep_fn(int coord, int tk, int d) {
    return coord == 1 ? fwd_sweep_fn_c<1>(tk, d) : fwd_sweep_fn_c<0>(tk, d);
}

// adjoint instances with a compile-time tile depth for the full record
// layouts (the autotuner's usual choices); compact records and other depths
// run the generic instance
template <int COORD>
SweepFn adj_sweep_fn_c(int tk, int d, bool compact) {
    const auto seq = std::make_integer_sequence<int, 8>{};
    if (compact) return pick_adj<COORD, true, 0>(d, seq);
    switch (tk) {
        case 28: return pick_adj<COORD, false, 28>(d, seq);
        case 32: return pick_adj<COORD, false, 32>(d, seq);
        case 40: return pick_adj<COORD, false, 40>(d, seq);
        case 48: return pick_adj<COORD, false, 48>(d, seq);
        default: return pick_adj<COORD, false, 0>(d, seq);
    }
}

SweepFn adj_sweep_fn(int coord, int tk, int d, bool compact) {
    return coord == 1 ? adj_sweep_fn_c<1>(tk, d, compact) : adj_sweep_fn_c<0>(tk, d, compact);
}

void launch_fwd_iteration(const Plan& P, const SweepArgs& a, hipStream_t st) {
    for (int d = 0; d < 8; ++d) {
        {
        TimedLaunch tl(P, st, P.nplanes);
        const SweepFn fn = fwd_sweep_fn(P.G.coord, P.G.tk, d);
        for (int p = 0; p < P.nplanes; ++p)
            hipLaunchKernelGGL(fn, dim3(P.nsrc, P.plane_count[p]), dim3(64), tile_lds_bytes(P.G), st, a,
                               P.plane_id[p], P.plane_s0[p]);
        }
        hipLaunchKernelGGL(k_fwd_bnd, dim3(P.nbblocks, P.nsrc), dim3(kBndThreads), 0, st, a, d);
    }
    hipLaunchKernelGGL(k_fwd_finalize, dim3(P.nsrc), dim3(256), 0, st, a);
}

void launch_adj_init(const Plan& P, const SweepArgs& a, const double* tau, int nrec, const double* rec,
                     const double* R, const double* init, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks(2 * P.G.NB * P.nsrc)), dim3(256), 0, st, P.bnd_in,
                       2 * P.G.NB * P.nsrc, 0.0);  // bnd_in and bnd_rhs
    const dim3 grid(blocks_for(P.G.N, 256), P.nsrc);
    const dim3 rgrid(blocks_for(P.nsrc, 64));
    const int t0 = P.continuous ? 0 : 1;
    if (P.G.coord == 1) {
        if (P.continuous) hipLaunchKernelGGL(k_cadj_coef<1>, grid, dim3(256), 0, st, a, tau, P.coef, P.diag, P.rhs);
        else hipLaunchKernelGGL(k_adj_coef<1>, grid, dim3(256), 0, st, a, tau, P.coef, P.bnd_in, P.diag, P.rhs);
        hipLaunchKernelGGL(k_adj_rhs<1>, rgrid, dim3(64), 0, st, a, P.diag, P.rhs, P.box, nrec, rec, R, t0);
    } else {
        if (P.continuous) hipLaunchKernelGGL(k_cadj_coef<0>, grid, dim3(256), 0, st, a, tau, P.coef, P.diag, P.rhs);
        else hipLaunchKernelGGL(k_adj_coef<0>, grid, dim3(256), 0, st, a, tau, P.coef, P.bnd_in, P.diag, P.rhs);
        hipLaunchKernelGGL(k_adj_rhs<0>, rgrid, dim3(64), 0, st, a, P.diag, P.rhs, P.box, nrec, rec, R, t0);
    }
    hipLaunchKernelGGL(k_solve_init, dim3(fill_blocks(P.G.N), P.nsrc), dim3(256), 0, st, a, init, 0.0, 0.0);
}

void launch_adj_iteration(const Plan& P, const SweepArgs& a, hipStream_t st) {
    for (int d = 0; d < 8; ++d) {
        {
        TimedLaunch tl(P, st, P.nplanes);
        const SweepFn fn = adj_sweep_fn(P.G.coord, P.G.tk, d, P.compact);
        for (int p = 0; p < P.nplanes; ++p)
            hipLaunchKernelGGL(fn, dim3(P.nsrc, P.plane_count[p]), dim3(64), tile_lds_bytes(P.G), st, a,
                               P.plane_id[p], P.plane_s0[p]);
        }
        if (P.continuous) {
            hipLaunchKernelGGL(k_cadj_bnd_calc, dim3(P.nbblocks, P.nsrc), dim3(kBndThreads), 0, st, a, P.bnd_in);
            hipLaunchKernelGGL(k_cadj_bnd_store, dim3(P.nbblocks, P.nsrc), dim3(kBndThreads), 0, st, a, P.bnd_in, d);
        } else {
            hipLaunchKernelGGL(k_adj_bnd, dim3(P.nbblocks, P.nsrc), dim3(kBndThreads), 0, st, a, d);
        }
    }
    hipLaunchKernelGGL(k_adj_finalize, dim3(P.nsrc), dim3(256), 0, st, a);
}

void launch_cadj_scale(const Plan& P, const double* s, double* lam, hipStream_t st) {
    hipLaunchKernelGGL(k_cadj_scale, dim3(fill_blocks(P.G.N), P.nsrc), dim3(256), 0, st, P.G, s, lam, P.nsrc);
}

void launch_fill(double* p, long long n, double v, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(fill_blocks(n)), dim3(256), 0, st, p, n, v);
}

void launch_sample(const Plan& P, const double* tau, int nrec, const double* rec, double* out, hipStream_t st) {
    const long long tot = (long long)P.nsrc * nrec;
    if (tot == 0) return;
    if (P.G.coord == 1)
        hipLaunchKernelGGL(k_sample<1>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, P.G, P.T, P.src, P.nsrc, tau,
                           nrec, rec, out);
    else
        hipLaunchKernelGGL(k_sample<0>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, P.G, P.T, P.src, P.nsrc, tau,
                           nrec, rec, out);
}

void launch_kernel_accum(const Plan& P, const double* xi, const double* eta, const double* tau, const double* lam,
                         double* grad, int accumulate, hipStream_t st) {
    if (P.G.coord == 1)
        hipLaunchKernelGGL(k_kernel_accum<1>, dim3(blocks_for(P.G.N, 256)), dim3(256), 0, st, P.G, P.T, P.src,
                           P.nsrc, xi, eta, tau, lam, grad, accumulate);
    else
        hipLaunchKernelGGL(k_kernel_accum<0>, dim3(blocks_for(P.G.N, 256)), dim3(256), 0, st, P.G, P.T, P.src,
                           P.nsrc, xi, eta, tau, lam, grad, accumulate);
}

}  // namespace tt

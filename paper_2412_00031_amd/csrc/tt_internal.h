// tt_internal.h -- library-private types and device helpers of libtt.
//
// Numerics (Chen et al., TomoATT, arXiv 2412.00031; Sec. 2.1 Eq. (4), Sec. 3.1):
//   T = T0 * tau with T0 = s0 sqrt(d^T M0^{-1} d), d = x - x_s in the source's
//   local (r^, theta^, phi^) frame; scaled gradient p = (dT/dr, dT/dtheta / r,
//   dT/dphi / (r cos theta)); Lax-Friedrichs update of the factored equation
//   with viscosity sigma_a = kappa T0 g_a.  Everything in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "tt.h"

namespace tt {

// Record a printf-style message for tt_last_error() and return `code`.
int fail(int code, const char* fmt, ...);

constexpr int kBI = 8;        // column block of one wave: 8 x 8 (i, j) columns
constexpr int kBJ = 8;
constexpr int kWave = 64;
constexpr int kBndThreads = 256;
constexpr int kMaxTileK = 62;  // k-extent of a forward sweep tile; the staged column (tk + 2) fits one wave

// Kernel-argument copy of the grid.
struct Geo {
    int n[3];          // nodes per axis
    int m[3];          // interior nodes per axis (n - 2)
    int coord;         // 0 Cartesian, 1 spherical
    int nt[3];         // tile columns along i' and j'; nt[2] = most tiles of one tile column
    int tk;            // hyperplane steps of a tile (its extent along u = i' + j' + k')
    int ntiles;        // nt0 * nt1 * nt2 (partial-sum slots per directional sweep)
    long long N;       // n0 * n1 * n2
    long long si, sj;  // strides of axes 0 and 1 (axis 2 has stride 1)
    long long NB;      // boundary nodes
    int W;             // n1 + n2 - 1: width of the row-coalesced layouts
    int n1p;           // aligned layouts: row pitch (a multiple of 8 records, >= n1 + 7)
    int joff[2];       // aligned layouts: record offset of j in a row for sweeps with s1 > 0, s1 < 0
    long long Sa;      // records per aligned layout: n0 * W * n1p
    double o[3], h[3], inv2h[3], invh[3];
};

// Sheared sweep tiles.  In sweep-relative interior coordinates (i', j', k')
// a tile is the 8 x 8 (i', j') tile column (TI, TJ) intersected with the slab
// TK tk <= u < (TK + 1) tk of the hyperplane index u = i' + j' + k'.  Tile column
// TI + TJ = s spans u in [8 s, 8 s + 14 + m2) (full columns; ragged ones end
// earlier), i.e. slabs lo(s)..hi(s).  A tile reads its upstream neighbours'
// nodes at u - 1 (slabs TK - 1 and TK of the neighbouring columns) and its
// downstream ones' at u + 1 (slabs TK and TK + 1), so all tiles with the same
// tile-plane number TI + TJ + TK are independent and each depends only on
// lower tile-planes.
__host__ __device__ inline int col_tile_lo(const Geo& G, int s) { return (kBI * s) / G.tk; }
__host__ __device__ inline int col_tile_hi(const Geo& G, int s) {
    return (kBI * s + (kBI - 1) + (kBJ - 1) + G.m[2] - 1) / G.tk;
}
// tile columns with TI + TJ = s
__host__ __device__ inline int diag_first(const Geo& G, int s) { return s - (G.nt[1] - 1) > 0 ? s - (G.nt[1] - 1) : 0; }
__host__ __device__ inline int diag_count(const Geo& G, int s) {
    const int hi = s < G.nt[0] - 1 ? s : G.nt[0] - 1;
    return hi - diag_first(G, s) + 1;
}
// tile b of tile-plane p whose first tile column sum is s0 (tiles ordered by s,
// then TI); the host enumerates the planes so that b is always in range
__host__ __device__ inline void tile_decode(const Geo& G, int p, int s0, int b, int& TI, int& TJ, int& TK) {
    const int smax = G.nt[0] + G.nt[1] - 2;
    int s = s0;
    for (; s < smax; ++s) {
        const int c = diag_count(G, s);
        if (b < c) break;
        b -= c;
    }
    TI = diag_first(G, s) + b;
    TJ = s - TI;
    TK = p - s;
}
// LDS doubles per staged column: the tk + 2 entries, rounded up to an even
// count (the window is staged two doubles per lane and load)
__host__ __device__ inline int tile_pitch(int tk) { return (tk + 3) & ~1; }

// Per-source constants, produced on the device by k_src_setup.
struct Src {
    double Xs[3];      // source position in the embedding (spherical) or (z,y,x)
    double E[9];       // rows: source-frame unit vectors r^_s, theta^_s, phi^_s
    double mi11, mi12, mi22;  // lower-right block of M0^{-1}
    double s0;
    int fb[3];         // base corner of the fixed cell
    int pad;
};

// Per-axis tables, built on the device by k_tables into the caller's workspace.
//   tab0[i]  = r (spherical) or z (Cartesian)
//   tab1[j]  = (cos theta, sin theta) (spherical) or (y, 0) (Cartesian)
//   tab2[k]  = (cos phi, sin phi) (spherical) or (x, 0) (Cartesian)
struct Tabs {
    const double* t0;
    const double2* t1;
    const double2* t2;
};

// Lane-constant geometry of an (i, j) column.
struct Col {
    double x0;         // r or z
    double ct, st;     // cos/sin latitude (spherical), y in ct (Cartesian)
    double rct, rst;   // r cos theta, r sin theta
    double g1, g2;     // scaled-gradient factors of axes 1, 2 (g0 = 1)
};

__device__ __forceinline__ Col make_col(const Geo& G, const Tabs& T, int i, int j) {
    Col c;
    c.x0 = T.t0[i];
    double2 a1 = T.t1[j];
    c.ct = a1.x;
    c.st = a1.y;
    if (G.coord == 1) {
        c.rct = c.x0 * c.ct;
        c.rst = c.x0 * c.st;
        c.g1 = 1.0 / c.x0;
        c.g2 = 1.0 / c.rct;
    } else {
        c.rct = c.rst = 0.0;
        c.g1 = c.g2 = 1.0;
    }
    return c;
}

__device__ __forceinline__ bool in_fixed(const Src& S, int i, int j, int k) {
    return (unsigned)(i - S.fb[0]) <= 1u && (unsigned)(j - S.fb[1]) <= 1u && (unsigned)(k - S.fb[2]) <= 1u;
}

// 1/sqrt(x) for x > 0 to about an ulp: the hardware estimate (good to about
// 23 bits) refined by two Newton steps y <- y (3 - x y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y *= fma(-h * y, y, 1.5);
    y *= fma(-h * y, y, 1.5);
    return y;
}

// sqrt(x) for x >= 0 to about an ulp, as x / sqrt(x) without a branch: 0 at
// x = 0, and x / sqrt(DBL_MIN) below the smallest normal double (Hamiltonians
// that small do not occur)
__device__ __forceinline__ double sqrt_nr(double x) { return x * rsqrt_nr(fmax(x, 2.2250738585072014e-308)); }

// T0 and its scaled gradient t at a node of column c with axis-2 table value
// (c2, s2) = (cos phi, sin phi) or (x, 0); rq = 1/sqrt(Q) = s0 / T0 (0 at the
// source itself, where the factor vanishes).  OFF_SOURCE: the caller never
// asks at the source itself (Q > 0; the sweeps skip the fixed cell), so there
// is no branch.
template <int COORD, bool OFF_SOURCE = false>
__device__ __forceinline__ void factor(const Src& S, const Col& c, double c2, double s2, double& T0, double t[3],
                                       double& rq) {
    double d0, d1, d2;
    if (COORD == 1) {
        double D0 = c.rct * c2 - S.Xs[0];
        double D1 = c.rct * s2 - S.Xs[1];
        double D2 = c.rst - S.Xs[2];
        d0 = D0 * S.E[0] + D1 * S.E[1] + D2 * S.E[2];
        d1 = D0 * S.E[3] + D1 * S.E[4] + D2 * S.E[5];
        d2 = D0 * S.E[6] + D1 * S.E[7] + D2 * S.E[8];
    } else {
        d0 = c.x0 - S.Xs[0];
        d1 = c.ct - S.Xs[1];
        d2 = c2 - S.Xs[2];
    }
    double m0 = d0;
    double m1 = S.mi11 * d1 + S.mi12 * d2;
    double m2 = S.mi12 * d1 + S.mi22 * d2;
    double Q = d0 * m0 + d1 * m1 + d2 * m2;
    if (!OFF_SOURCE && !(Q > 0.0)) {
        T0 = 0.0;
        t[0] = t[1] = t[2] = 0.0;
        rq = 0.0;
        return;
    }
    rq = rsqrt_nr(Q);
    T0 = S.s0 * (Q * rq);
    double f = S.s0 * rq;
    if (COORD == 1) {
        // gradient in the embedding, then on the node's local unit vectors
        // r^ = (ct c2, ct s2, st), theta^ = (-st c2, -st s2, ct), phi^ = (-s2, c2, 0)
        double G0 = f * (m0 * S.E[0] + m1 * S.E[3] + m2 * S.E[6]);
        double G1 = f * (m0 * S.E[1] + m1 * S.E[4] + m2 * S.E[7]);
        double G2 = f * (m0 * S.E[2] + m1 * S.E[5] + m2 * S.E[8]);
        double hz = G0 * c2 + G1 * s2;
        t[0] = c.ct * hz + c.st * G2;
        t[1] = c.ct * G2 - c.st * hz;
        t[2] = G1 * c2 - G0 * s2;
    } else {
        t[0] = f * m0;
        t[1] = f * m1;
        t[2] = f * m2;
    }
}

template <int COORD>
__device__ __forceinline__ void factor(const Src& S, const Col& c, double c2, double s2, double& T0, double t[3]) {
    double rq;
    factor<COORD, false>(S, c, c2, s2, T0, t, rq);
}

// Local state of the factored Hamiltonian at an interior node: P, M P, H.
struct Loc {
    double T0, t[3], P[3], MP[3], H;
};

template <int COORD>
__device__ __forceinline__ void local_state(const Geo& G, const Src& S, const Col& c, double c2, double s2,
                                            double xi, double eta, double tx, double up0, double dn0,
                                            double up1, double dn1, double up2, double dn2, Loc& L) {
    // up_a = tau(x - e_a), dn_a = tau(x + e_a) in absolute axis directions
    factor<COORD>(S, c, c2, s2, L.T0, L.t);
    double q0 = (dn0 - up0) * G.inv2h[0];
    double q1 = c.g1 * (dn1 - up1) * G.inv2h[1];
    double q2 = c.g2 * (dn2 - up2) * G.inv2h[2];
    L.P[0] = L.T0 * q0 + tx * L.t[0];
    L.P[1] = L.T0 * q1 + tx * L.t[1];
    L.P[2] = L.T0 * q2 + tx * L.t[2];
    L.MP[0] = L.P[0];
    L.MP[1] = (1.0 - 2.0 * xi) * L.P[1] + 2.0 * eta * L.P[2];
    L.MP[2] = 2.0 * eta * L.P[1] + (1.0 + 2.0 * xi) * L.P[2];
    L.H = sqrt(L.P[0] * L.MP[0] + L.P[1] * L.MP[1] + L.P[2] * L.MP[2]);
}

// Lax-Friedrichs update: the tau(x) that zeroes
//   G_x = H(q, tau_old(x)) - sum_a sigma_a (dn_a - 2 tau(x) + up_a) / (2 h_a) - s(x),
// sigma_a = kappa T0 g_a.  With C = sum_a g_a / h_a (g_0 = 1) it reads
//   tau(x) = (s - H) / (kappa T0 C) + sum_a w_a (up_a + dn_a),  w_a = g_a / (2 h_a C),
// and 1 / (kappa T0 C) = rho / sqrt(Q) with rho = 1 / (kappa s0 C): LfCol holds
// the column's constants, so an update has no division.
//
// The factor enters through T0 = s0 Q rq and its scaled gradient t = s0 rq u
// (rq = 1 / sqrt(Q), u = the gradient direction of the factor() notes without
// the s0 rq), so P_a = T0 q_a + tau t_a = s0 rq R_a with R_a = Q q_a + tau u_a and
// H = s0 rq sqrt(R . M R): the update forms R, not T0 and t.  Along a spherical
// column X = (rct c2, rct s2, rst), so d = E (X - Xs) is d_i = A_i c2 + B_i s2 + C_i
// with column constants A, B, C.
struct LfCol {
    double v1, v2;      // g_a / (2 h_a) of axes 1, 2 (central differences)
    double w0, w1, w2;  // averaging weights w_a
    double rho;
    double A[3], B[3], C[3];  // d_i along the column (spherical); Cartesian: C = (x0, y) - Xs
};

template <int COORD>
__device__ __forceinline__ LfCol lf_col(const Geo& G, const Src& S, const Col& c, double kappa) {
    LfCol W;
    const double iC = 1.0 / (G.invh[0] + c.g1 * G.invh[1] + c.g2 * G.invh[2]);
    W.v1 = c.g1 * G.inv2h[1];
    W.v2 = c.g2 * G.inv2h[2];
    W.w0 = G.inv2h[0] * iC;
    W.w1 = W.v1 * iC;
    W.w2 = W.v2 * iC;
    W.rho = iC / (kappa * S.s0);
    if (COORD == 1) {
        const double D2 = c.rst - S.Xs[2];
        for (int i = 0; i < 3; ++i) {
            W.A[i] = c.rct * S.E[3 * i];
            W.B[i] = c.rct * S.E[3 * i + 1];
            W.C[i] = D2 * S.E[3 * i + 2] - (S.Xs[0] * S.E[3 * i] + S.Xs[1] * S.E[3 * i + 1]);
        }
    } else {
        W.A[0] = W.A[1] = W.A[2] = W.B[0] = W.B[1] = W.B[2] = W.C[2] = 0.0;
        W.C[0] = c.x0 - S.Xs[0];
        W.C[1] = c.ct - S.Xs[1];
    }
    return W;
}

template <int COORD>
__device__ __forceinline__ double lf_update(const Geo& G, const Src& S, const Col& c, const LfCol& W, double c2,
                                            double s2, double sx, double ma, double mb, double mc, double tx,
                                            double up0, double dn0, double up1, double dn1, double up2, double dn2) {
    double d0, d1, d2;
    if (COORD == 1) {
        d0 = fma(c2, W.A[0], fma(s2, W.B[0], W.C[0]));
        d1 = fma(c2, W.A[1], fma(s2, W.B[1], W.C[1]));
        d2 = fma(c2, W.A[2], fma(s2, W.B[2], W.C[2]));
    } else {
        d0 = W.C[0];
        d1 = W.C[1];
        d2 = c2 - S.Xs[2];
    }
    const double m1 = S.mi11 * d1 + S.mi12 * d2;
    const double m2 = S.mi12 * d1 + S.mi22 * d2;
    const double Q = d0 * d0 + d1 * m1 + d2 * m2;  // > 0: the sweeps skip the fixed cell
    const double rq = rsqrt_nr(Q);
    double u0, u1, u2;
    if (COORD == 1) {
        // E^T m in the embedding, then on the node's local unit vectors
        // r^ = (ct c2, ct s2, st), theta^ = (-st c2, -st s2, ct), phi^ = (-s2, c2, 0)
        const double G0 = d0 * S.E[0] + m1 * S.E[3] + m2 * S.E[6];
        const double G1 = d0 * S.E[1] + m1 * S.E[4] + m2 * S.E[7];
        const double G2 = d0 * S.E[2] + m1 * S.E[5] + m2 * S.E[8];
        const double hz = G0 * c2 + G1 * s2;
        u0 = c.ct * hz + c.st * G2;
        u1 = c.ct * G2 - c.st * hz;
        u2 = G1 * c2 - G0 * s2;
    } else {
        u0 = d0;
        u1 = m1;
        u2 = m2;
    }
    const double R0 = Q * ((dn0 - up0) * G.inv2h[0]) + tx * u0;
    const double R1 = Q * ((dn1 - up1) * W.v1) + tx * u1;
    const double R2 = Q * ((dn2 - up2) * W.v2) + tx * u2;
    // (ma, mb, mc) = (1 - 2 xi, 2 eta, 1 + 2 xi): the lower-right block of M
    const double MR1 = ma * R1 + mb * R2;
    const double MR2 = mb * R1 + mc * R2;
    const double H = (S.s0 * rq) * sqrt_nr(R0 * R0 + R1 * MR1 + R2 * MR2);
    return (sx - H) * (W.rho * rq) + ((up0 + dn0) * W.w0 + (up1 + dn1) * W.w1 + (up2 + dn2) * W.w2);
}

// ----- state of one batched solve (host side) -----
struct Plan {
    Geo G;
    Tabs T;
    int nsrc = 0;
    int nplanes = 0;          // non-empty tile-planes per sweep
    int max_plane_tiles = 0;  // largest tile-plane
    int nbblocks = 0;         // boundary-pass blocks per source
    int nslots = 0;           // partial-sum slots per source per iteration
    double kappa = 1.0, tol = 1e-6;
    int max_iter = 1;         // iteration budget of this group
    int hist_stride = 1;      // row length of eps_hist (the call's max_iter)
    double* eps_hist = nullptr;
    // workspace views
    Src* src = nullptr;
    double* tab0 = nullptr;
    double2* tab1 = nullptr;
    double2* tab2 = nullptr;
    int* active = nullptr;
    int* iter = nullptr;
    int* counter = nullptr;
    double* part = nullptr;
    double* part2 = nullptr;
    double* coef = nullptr;   // adjoint: [nsrc][4][Sa][6] (line-aligned row-coalesced layouts) or [nsrc][N][6]
    double* diag = nullptr;   // adjoint: diagonal of each node's row [nsrc][N]
    double* rhs = nullptr;    // adjoint: right-hand side divided by the diagonal [nsrc][N]
    int* box = nullptr;       // adjoint: index box of each source's nonzero rhs [nsrc][6]
    double* model = nullptr;  // forward: [4][Sa][4] = (s, 1 - 2 xi, 2 eta, 1 + 2 xi) (aligned row-coalesced layouts)
    double* bnd_in = nullptr; // adjoint: [nsrc][NB] (continuous adjoint: boundary pass scratch)
    double* bnd_rhs = nullptr; // adjoint: right-hand side of the boundary nodes, [nsrc][NB]
    bool continuous = false;  // adjoint: upwind discretisation of Eq. (5) instead of the exact transpose
    bool compact = false;     // adjoint: one node-order copy of the coefficient records
    std::vector<int> plane_count;  // tiles of each non-empty tile-plane
    std::vector<int> plane_id;     // its tile-plane number TI + TJ + TK
    std::vector<int> plane_s0;     // its first tile column sum TI + TJ
    // optional timing of the sweep kernels: an event pair around the
    // tile-plane launches of each directional sweep, with the launch count
    std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>>* timing = nullptr;
};

// Kernel-argument bundle of the sweep kernels.
struct SweepArgs {
    Geo G;
    Tabs T;
    const double *s, *xi, *eta;
    const Src* src;
    double* field;          // tau or lambda [nsrc][N]
    const double* coef;     // adjoint coefficients [nsrc][4][Sa][6], or [nsrc][N][6] when compact
    const double* rhs;      // adjoint right-hand side / diagonal [nsrc][N]
    const int* box;         // [nsrc][6]: i, j, k ranges of the nonzero rhs (empty: lo > hi)
    const double* model;    // forward model records [4][Sa][4]
    const double* bnd_in;   // adjoint face couplings [nsrc][NB]
    const double* bnd_rhs;  // adjoint right-hand side of the boundary nodes [nsrc][NB]
    int* active;
    int* iter;
    int32_t* status;
    double* part;
    double* part2;
    int* counter;
    double* eps_hist;       // optional [nsrc][hist_stride]
    int nslots, nbblocks, nsrc, max_iter, hist_stride;
    int compact;            // adjoint records in node order (TT_FLAG_COMPACT_ADJOINT)
    double kappa, tol;
};

SweepArgs make_args(const Plan& P, const double* s, const double* xi, const double* eta, double* field,
                    int32_t* status);
void launch_tables(const Plan& P, hipStream_t st);
void launch_src_setup(const Plan& P, const double* src_pos, const double* src_par, hipStream_t st);
void launch_source_params(const Geo& G, const double* s, const double* xi, const double* eta,
                          const double* src_pos, double* src_par, int nsrc, hipStream_t st);
void launch_fwd_init(const Plan& P, const SweepArgs& a, const double* tau_init, const double* s, const double* xi,
                     const double* eta, hipStream_t st);
void launch_fwd_iteration(const Plan& P, const SweepArgs& a, hipStream_t st);
void launch_adj_init(const Plan& P, const SweepArgs& a, const double* tau, int nrec, const double* rec_pos,
                     const double* R, const double* init, hipStream_t st);
void launch_adj_iteration(const Plan& P, const SweepArgs& a, hipStream_t st);
void launch_cadj_scale(const Plan& P, const double* s, double* lam, hipStream_t st);
void launch_sample(const Plan& P, const double* tau, int nrec, const double* rec_pos, double* out,
                   hipStream_t st);
void launch_fill(double* p, long long n, double v, hipStream_t st);
void launch_reloc_times(const Plan& P, const double* tau, int nev, const double* ev, const double* t0, double* out,
                        hipStream_t st);
void launch_reloc_kernel(const Plan& P, const double* tau, int nev, const double* ev, const double* R, double* K,
                         hipStream_t st);
void launch_misfit(int nsrc, int nrec, const double* T, const double* Tobs, const double* w, int npair,
                   const int32_t* pairs, const double* wpair, double alpha, double beta, double* R,
                   double* chi, hipStream_t st);
void launch_misfit_cr(int nsrc, int nrec, const double* T, const double* Tobs, const int32_t* off, const int32_t* pair,
                      const double* wcr, double gamma, double* R, double* chi, hipStream_t st);
// Inversion grids of the multiple-grid parameterisation, flattened for kernel
// arguments: sizes, offsets of each grid's axis coordinates in the
// concatenated coords array, and running sums of m2, m1*m2 and 3*m0*m1*m2.
struct MgGrids {
    int H;
    int ncoord;  // total coordinates of all grids
    int m[TT_MG_MAX_GRIDS][3];
    int coff[TT_MG_MAX_GRIDS][3];
    int s2off[TT_MG_MAX_GRIDS + 1];
    int s12off[TT_MG_MAX_GRIDS + 1];
    long long outoff[TT_MG_MAX_GRIDS + 1];
};

// Projection plan: the separable staged form when its LDS fits, with nch
// row chunks per plane and ws_bytes of partial sums; else one wave per node.
constexpr long long kMgMaxLds = 60 * 1024;  // dynamic LDS of the staged forms (static LDS comes on top)
constexpr long long kMgCoordLds = 32 * 1024;  // coordinates staged in LDS up to this size
struct MgPlan {
    bool separable;
    int nch;
    size_t lds;
    size_t ws_bytes;
};

MgGrids make_mg(int H, const int* m);
MgPlan plan_mg_project(const Geo& G, const MgGrids& Q);
void launch_mg_project(const Geo& G, int H, const int* m, const double* coords, const double* K, double* out,
                       double* ws, hipStream_t st);
void launch_mg_expand(const Geo& G, int H, const int* m, const double* coords, const double* C, double* field,
                      hipStream_t st);
void launch_kernel_density(const Geo& G, const double* s, const double* dens, const double* grad, double eps,
                           double zeta, double* K, double* Kd, hipStream_t st);
void launch_kernel_accum(const Plan& P, const double* xi, const double* eta, const double* tau,
                         const double* lam, double* grad, int accumulate, hipStream_t st);

}  // namespace tt

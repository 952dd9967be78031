/*
 * oracle.c -- plain FP64 CPU oracle for per-source adjoint-state traveltime
 * tomography: the factored anisotropic Eikonal solve by fast sweeping, the
 * exact discrete adjoint of that solve, and the sensitivity kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code, header
 * or table with the HIP library: every quantity is recomputed here in the most
 * direct way (libm cos/sin/sqrt per evaluation, explicit division, nested
 * loops in lexicographic order).  Compile with -O2 -ffp-contract=off.
 *
 * What it follows (Chen, Nagaso, Xu & Tong, "TomoATT", arXiv 2412.00031):
 *   Sec. 2.1 step 1, Eq. (4): anisotropic Eikonal equation
 *       p^T M(xi,eta) p = s^2,   p = (dT/dr, dT/dtheta / r, dT/dphi / (r cos theta)),
 *       M = [[1,0,0],[0,1-2xi,2eta],[0,2eta,1+2xi]],  T(x_s) = 0.
 *   Sec. 3.1: fast sweeping (Zhao 2005), multiplicative factorization
 *       T = T0 * tau (Luo & Qian 2012), spherical coordinates.
 *   Sec. 2.1 step 2, Eq. (5): adjoint equation; its exact discrete
 *       counterpart, the transpose of the Jacobian of the discrete forward
 *       system, and (R14) an upwind finite-volume discretisation of Eq. (5)
 *       itself.
 *   Eqs. (2)-(4), (A2)-(A4): traveltime, common-source and common-receiver
 *       differential misfits and their adjoint sources R = d chi / d T(x_r).
 *   Eq. (10), App. B: relocation kernels from receiver-side fields.
 *   Eqs. (6)-(9): kernels; here the discrete gradients d chi/d s, d chi/d xi,
 *       d chi/d eta, which Eq. (9) relates to K_s, K_xi, K_eta.
 *
 * The paper prints no discrete scheme.  Readings adopted where it is silent:
 *   (R1) axes a = 0,1,2 are (r, theta=latitude, phi=longitude) in spherical
 *        mode (r in km, angles in radians) or (z, y, x) in km in Cartesian mode;
 *        storage [n0][n1][n2], axis 2 fastest.  Scaled-gradient factors
 *        g = (1, 1/r, 1/(r cos theta)) (spherical) or (1,1,1) (Cartesian).
 *   (R2) T0 = s0 * sqrt(d^T M0^{-1} d): d is x - x_s in the source's local
 *        (r^, theta^, phi^) frame (embedding X = r(cos th cos ph, cos th sin ph,
 *        sin th)), s0/xi0/eta0 are the model trilinearly interpolated at x_s and
 *        are treated as constants.  grad T0 is analytic, projected on the local
 *        frame at x.
 *   (R3) fixed set F = the 8 corners of the grid cell that contains x_s
 *        (base index floor((x_s-o)/h) clamped to [0,n-2]); tau = 1 on F.
 *   (R4) first-order Lax-Friedrichs update of the factored equation at interior
 *        non-fixed nodes, viscosity sigma_a = kappa*T0*g_a (see lf_update).
 *   (R5) 8 sweep directions in binary order (+++, ++-, +-+, ..., ---), axis 2
 *        least significant; each sweep is followed by a boundary pass.
 *   (R6) boundary pass: for a boundary node b not in F let a* be the largest
 *        axis on which b lies on the boundary; tau_b = tau(b + nu e_a*), nu the
 *        inward sign (zeroth-order extrapolation of the factor tau); groups
 *        a* = 0, 1, 2 in turn.  Linear extrapolation (2 tau(b+nu e) -
 *        tau(b+2nu e)) was tried first: with it the sweeps diverge for deep
 *        sources of the 101^3 spherical workload, while Sec. 3.1 states that the
 *        method converges unconditionally; with the copy rule every boundary row
 *        is an M-matrix row and both the sweeps and the transposed sweeps
 *        converge.
 *   (R7) iteration = 8 sweeps with their boundary passes; eps = (1/N) sum of
 *        |tau_new - tau_old| over all writes of the iteration; stop at the first
 *        iteration with eps < tol.
 *   (R8) receivers: T(x_r) = sum_c w_c T0(c) tau(c), trilinear weights w_c.
 *   (R9) common-source pairs are an explicit list of unordered pairs, each
 *        counted once.
 *   (R10) adjoint: Gauss-Seidel on J^T lambda = d chi / d tau with the same 8
 *        directions; after each sweep a transposed boundary pass in reverse group
 *        order (a* = 2, 1, 0); lambda = 0 on F (the fixed rows couple to nothing).
 *        eps = sum|d lambda| / max(sum|lambda|, 1e-300).
 *   (R11) kernel density (Eqs. (18)-(19)): the adjoint field of Eq. (5) is
 *        P = (d chi / d s) / (s V) with V the trapezoidal node volume, since
 *        K_s = s (d chi / d s) / V (Eq. (9)) and K_s = P s^2.
 *   (R12) multiple-grid basis (Eqs. (11)-(17)): tents vanish outside each
 *        inversion grid's range; the integral of Eq. (17) is the node
 *        quadrature sum_x K B V; the s-coefficients perturb ds / s (Eq. (9)).
 *   (R13) common-receiver pairs (Eqs. (4) and (A4)): an explicit list of
 *        triples (n, j, m), the unordered source pair {n, j} recorded at
 *        receiver m, each counted once, as in (R9).
 *   (R15) relocation (Eq. (10), App. B): by reciprocity T[n][m] = Gamma_m(x_n)
 *        + t_n with Gamma_m the field of receiver m taken as the source, so
 *        the misfits are those of Eqs. (2)-(4) and d chi / d Gamma_m(x_n) is
 *        the adjoint source R[n][m]; grad Gamma_m(x_n) is the gradient of the
 *        trilinear interpolant that samples Gamma_m (the cell of the sampling),
 *        with respect to the grid coordinates.
 *   (R14) continuous adjoint (Eq. (5), the paper's own route): upwind finite
 *        volumes.  The flux P w with w = -M grad T leaves each trapezoidal
 *        control volume through six faces; the face velocity is the mean of the
 *        two nodal normal components, the upwind side's P is carried, P = 0 on
 *        the fixed set (the source absorbs) and outside the grid, and the point
 *        sources of Eq. (5) enter through the trilinear weights of each
 *        receiver.  grad T = T0 (central or, on a boundary axis, one-sided
 *        differences of tau) + tau grad T0.  A node without outflow keeps
 *        P = 0.  Solve: the 8 directional Gauss-Seidel sweeps over interior
 *        nodes, each followed by one Jacobi pass over the boundary nodes.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_R_EARTH 6371.0

typedef struct {
    int n[3];
    int coord;            /* 0 Cartesian, 1 spherical */
    double o[3], h[3];
    size_t N;
} OGrid;

typedef struct {
    double pos[3];
    double s0, xi0, eta0;
    double Xs[3];         /* source position in the embedding */
    double E[3][3];       /* E[c] = c-th unit vector of the source frame */
    double mi11, mi12, mi22;  /* lower-right 2x2 block of M0^{-1} */
    int fb[3];            /* base corner of the fixed cell */
} OSrc;

static void grid_init(OGrid* g, const int* n, int coord, const double* o, const double* h) {
    for (int a = 0; a < 3; ++a) { g->n[a] = n[a]; g->o[a] = o[a]; g->h[a] = h[a]; }
    g->coord = coord;
    g->N = (size_t)n[0] * (size_t)n[1] * (size_t)n[2];
}

static size_t IDX(const OGrid* g, int i, int j, int k) {
    return ((size_t)i * (size_t)g->n[1] + (size_t)j) * (size_t)g->n[2] + (size_t)k;
}

static double cval(const OGrid* g, int a, int idx) { return g->o[a] + (double)idx * g->h[a]; }

static int cell_base(const OGrid* g, int a, double x) {
    double u = (x - g->o[a]) / g->h[a];
    double fl = floor(u);
    int b;
    if (fl < 0.0) b = 0;
    else if (fl > (double)(g->n[a] - 2)) b = g->n[a] - 2;
    else b = (int)fl;
    return b;
}

/* unit vectors of the local frame at (theta, phi) in the embedding */
static void local_frame(double th, double ph, double er[3], double et[3], double ep[3]) {
    double ct = cos(th), st = sin(th), cp = cos(ph), sp = sin(ph);
    er[0] = ct * cp; er[1] = ct * sp; er[2] = st;
    et[0] = -st * cp; et[1] = -st * sp; et[2] = ct;
    ep[0] = -sp; ep[1] = cp; ep[2] = 0.0;
}

static void src_init(OSrc* S, const OGrid* g, const double* pos, const double* par) {
    for (int a = 0; a < 3; ++a) S->pos[a] = pos[a];
    S->s0 = par[0]; S->xi0 = par[1]; S->eta0 = par[2];
    if (g->coord == 0) {
        for (int a = 0; a < 3; ++a) {
            S->Xs[a] = pos[a];
            for (int c = 0; c < 3; ++c) S->E[a][c] = (a == c) ? 1.0 : 0.0;
        }
    } else {
        double r = pos[0];
        local_frame(pos[1], pos[2], S->E[0], S->E[1], S->E[2]);
        for (int c = 0; c < 3; ++c) S->Xs[c] = r * S->E[0][c];
    }
    /* M0 lower-right block [[b, f], [f, c]] with b = 1-2xi0, c = 1+2xi0, f = 2eta0 */
    double b = 1.0 - 2.0 * S->xi0, c = 1.0 + 2.0 * S->xi0, f = 2.0 * S->eta0;
    double det = b * c - f * f;
    S->mi11 = c / det; S->mi12 = -f / det; S->mi22 = b / det;
    for (int a = 0; a < 3; ++a) S->fb[a] = cell_base(g, a, pos[a]);
}

static int is_fixed(const OSrc* S, int i, int j, int k) {
    return (i == S->fb[0] || i == S->fb[0] + 1) &&
           (j == S->fb[1] || j == S->fb[1] + 1) &&
           (k == S->fb[2] || k == S->fb[2] + 1);
}

static void unidx(const OGrid* g, size_t c, int* i, int* j, int* k) {
    *k = (int)(c % (size_t)g->n[2]);
    size_t q = c / (size_t)g->n[2];
    *j = (int)(q % (size_t)g->n[1]);
    *i = (int)(q / (size_t)g->n[1]);
}

/* scaled-gradient factors g_a at node (i, j) */
static void metric(const OGrid* g, int i, int j, double gm[3]) {
    if (g->coord == 0) { gm[0] = gm[1] = gm[2] = 1.0; return; }
    double r = cval(g, 0, i), th = cval(g, 1, j);
    gm[0] = 1.0;
    gm[1] = 1.0 / r;
    gm[2] = 1.0 / (r * cos(th));
}

/* (R2): T0 and its scaled gradient t_a = g_a dT0/dx_a at node (i,j,k). */
static void factor_at(const OGrid* g, const OSrc* S, int i, int j, int k, double* T0, double t[3]) {
    double x[3] = {cval(g, 0, i), cval(g, 1, j), cval(g, 2, k)};
    double d[3];
    double er[3], et[3], ep[3];
    if (g->coord == 0) {
        for (int a = 0; a < 3; ++a) d[a] = x[a] - S->pos[a];
    } else {
        double r = x[0];
        local_frame(x[1], x[2], er, et, ep);
        double D[3];
        for (int c = 0; c < 3; ++c) D[c] = r * er[c] - S->Xs[c];
        for (int a = 0; a < 3; ++a) d[a] = D[0] * S->E[a][0] + D[1] * S->E[a][1] + D[2] * S->E[a][2];
    }
    double m[3];
    m[0] = d[0];
    m[1] = S->mi11 * d[1] + S->mi12 * d[2];
    m[2] = S->mi12 * d[1] + S->mi22 * d[2];
    double Q = d[0] * m[0] + d[1] * m[1] + d[2] * m[2];
    if (!(Q > 0.0)) { *T0 = 0.0; t[0] = t[1] = t[2] = 0.0; return; }
    double sq = sqrt(Q);
    *T0 = S->s0 * sq;
    if (g->coord == 0) {
        for (int a = 0; a < 3; ++a) t[a] = S->s0 * m[a] / sq;
    } else {
        double G[3];
        for (int c = 0; c < 3; ++c)
            G[c] = S->s0 * (m[0] * S->E[0][c] + m[1] * S->E[1][c] + m[2] * S->E[2][c]) / sq;
        t[0] = G[0] * er[0] + G[1] * er[1] + G[2] * er[2];
        t[1] = G[0] * et[0] + G[1] * et[1] + G[2] * et[2];
        t[2] = G[0] * ep[0] + G[1] * ep[1] + G[2] * ep[2];
    }
}

/* Local quantities of the factored Hamiltonian at an interior node:
 *   q_a = g_a (tau(x+e_a) - tau(x-e_a)) / (2 h_a),  P = T0 q + tau(x) t,
 *   H = sqrt(P^T M P),  MP = M P,  sigma_a = kappa T0 g_a. */
typedef struct {
    double T0, t[3], gm[3], P[3], MP[3], H, sig[3];
} OLocal;

static void local_state(const OGrid* g, const OSrc* S, double kappa, const double* s_unused,
                        const double* xi, const double* eta, const double* tau,
                        int i, int j, int k, OLocal* L) {
    (void)s_unused;
    size_t c = IDX(g, i, j, k);
    size_t st[3] = {(size_t)g->n[1] * g->n[2], (size_t)g->n[2], 1};
    factor_at(g, S, i, j, k, &L->T0, L->t);
    metric(g, i, j, L->gm);
    double tx = tau[c];
    for (int a = 0; a < 3; ++a) {
        double q = L->gm[a] * (tau[c + st[a]] - tau[c - st[a]]) / (2.0 * g->h[a]);
        L->P[a] = L->T0 * q + tx * L->t[a];
        L->sig[a] = kappa * L->T0 * L->gm[a];
    }
    double x_ = xi[c], e_ = eta[c];
    L->MP[0] = L->P[0];
    L->MP[1] = (1.0 - 2.0 * x_) * L->P[1] + 2.0 * e_ * L->P[2];
    L->MP[2] = 2.0 * e_ * L->P[1] + (1.0 + 2.0 * x_) * L->P[2];
    L->H = sqrt(L->P[0] * L->MP[0] + L->P[1] * L->MP[1] + L->P[2] * L->MP[2]);
}

/* (R4) Lax-Friedrichs update: the value of tau(x) that zeroes
 *   G_x = H(q, tau_old(x)) - sum_a sigma_a (tau(x+e_a) - 2 tau(x) + tau(x-e_a)) / (2 h_a) - s(x). */
static double lf_update(const OGrid* g, const OSrc* S, double kappa, const double* s,
                        const double* xi, const double* eta, const double* tau, int i, int j, int k) {
    OLocal L;
    local_state(g, S, kappa, s, xi, eta, tau, i, j, k, &L);
    size_t c = IDX(g, i, j, k);
    size_t st[3] = {(size_t)g->n[1] * g->n[2], (size_t)g->n[2], 1};
    double num = s[c] - L.H, den = 0.0;
    for (int a = 0; a < 3; ++a) {
        num += L.sig[a] * (tau[c + st[a]] + tau[c - st[a]]) / (2.0 * g->h[a]);
        den += L.sig[a] / g->h[a];
    }
    return num / den;
}

/* largest axis on which (i,j,k) lies on the boundary, -1 if interior */
static int astar_of(const OGrid* g, int i, int j, int k) {
    int idx[3] = {i, j, k};
    int as = -1;
    for (int a = 0; a < 3; ++a)
        if (idx[a] == 0 || idx[a] == g->n[a] - 1) as = a;
    return as;
}

/* the inward node copied by the boundary row of boundary node b */
static size_t bnd_ref(const OGrid* g, int i, int j, int k, int as) {
    int idx[3] = {i, j, k};
    int nu = (idx[as] == 0) ? 1 : -1;
    int p1[3] = {i, j, k};
    p1[as] += nu;
    return IDX(g, p1[0], p1[1], p1[2]);
}

/* boundary nodes with a* == as, in storage order; returns the count */
static size_t boundary_group(const OGrid* g, int as, size_t* list) {
    size_t cnt = 0;
    for (int i = 0; i < g->n[0]; ++i) {
        int bi = (i == 0 || i == g->n[0] - 1);
        for (int j = 0; j < g->n[1]; ++j) {
            int bj = (j == 0 || j == g->n[1] - 1);
            int kstep = (bi || bj) ? 1 : (g->n[2] - 1);
            for (int k = 0; k < g->n[2]; k += kstep)
                if (astar_of(g, i, j, k) == as) list[cnt++] = IDX(g, i, j, k);
        }
    }
    return cnt;
}

static size_t boundary_count(const OGrid* g) {
    return g->N - (size_t)(g->n[0] - 2) * (size_t)(g->n[1] - 2) * (size_t)(g->n[2] - 2);
}

/* (R6) forward boundary pass; returns the sum of |changes|.  bl is scratch
 * space for boundary_count() indices. */
static double boundary_pass(const OGrid* g, const OSrc* S, double* tau, size_t* bl) {
    double acc = 0.0;
    for (int as = 0; as < 3; ++as) {
        size_t cnt = boundary_group(g, as, bl);
        for (size_t q = 0; q < cnt; ++q) {
            int i, j, k;
            unidx(g, bl[q], &i, &j, &k);
            if (is_fixed(S, i, j, k)) continue;
            size_t b1 = bnd_ref(g, i, j, k, as);
            double nv = tau[b1];
            acc += fabs(nv - tau[bl[q]]);
            tau[bl[q]] = nv;
        }
    }
    return acc;
}

/* ---------------------------------------------------------------------------
 * Visiting orders of the interior nodes in one directional sweep.
 *   order 0: lexicographic (the reference order);
 *   order 1: hyperplanes i'+j'+k' = L, nodes inside a plane in a seeded random
 *            permutation;
 *   order 2: tiles of 3x4x5 nodes on tile-hyperplanes, tiles of one tile-plane in
 *            descending tile index, nodes inside a tile lexicographic.
 * Orders 1 and 2 exist only to test that every order respecting the sweep's
 * dependencies gives bit-identical results.
 * ------------------------------------------------------------------------- */
static uint64_t lcg_next(uint64_t* st) {
    *st = *st * 6364136223846793005ULL + 1442695040888963407ULL;
    return *st >> 33;
}

/* interior node (i',j',k') in sweep-relative coordinates -> absolute */
static void rel2abs(const OGrid* g, const int sg[3], const int r[3], int out[3]) {
    for (int a = 0; a < 3; ++a) out[a] = (sg[a] > 0) ? 1 + r[a] : g->n[a] - 2 - r[a];
}

static size_t build_order(const OGrid* g, const OSrc* S, const int sg[3], int order, uint64_t seed,
                          size_t* list) {
    int m[3] = {g->n[0] - 2, g->n[1] - 2, g->n[2] - 2};
    size_t cnt = 0;
    if (order == 1) {
        uint64_t st = seed;
        for (int L = 0; L <= m[0] + m[1] + m[2] - 3; ++L) {
            size_t start = cnt;
            for (int r0 = 0; r0 < m[0]; ++r0)
                for (int r1 = 0; r1 < m[1]; ++r1) {
                    int r2 = L - r0 - r1;
                    if (r2 < 0 || r2 >= m[2]) continue;
                    int r[3] = {r0, r1, r2}, x[3];
                    rel2abs(g, sg, r, x);
                    if (is_fixed(S, x[0], x[1], x[2])) continue;
                    list[cnt++] = IDX(g, x[0], x[1], x[2]);
                }
            for (size_t q = cnt - start; q > 1; --q) {   /* Fisher-Yates */
                size_t p = (size_t)(lcg_next(&st) % q);
                size_t tmp = list[start + q - 1];
                list[start + q - 1] = list[start + p];
                list[start + p] = tmp;
            }
        }
    } else {
        int tb[3] = {3, 4, 5};
        int nt[3];
        for (int a = 0; a < 3; ++a) nt[a] = (m[a] + tb[a] - 1) / tb[a];
        for (int TL = 0; TL <= nt[0] + nt[1] + nt[2] - 3; ++TL)
            for (int T0 = nt[0] - 1; T0 >= 0; --T0)
                for (int T1 = nt[1] - 1; T1 >= 0; --T1) {
                    int T2 = TL - T0 - T1;
                    if (T2 < 0 || T2 >= nt[2]) continue;
                    for (int r0 = T0 * tb[0]; r0 < m[0] && r0 < (T0 + 1) * tb[0]; ++r0)
                        for (int r1 = T1 * tb[1]; r1 < m[1] && r1 < (T1 + 1) * tb[1]; ++r1)
                            for (int r2 = T2 * tb[2]; r2 < m[2] && r2 < (T2 + 1) * tb[2]; ++r2) {
                                int r[3] = {r0, r1, r2}, x[3];
                                rel2abs(g, sg, r, x);
                                if (is_fixed(S, x[0], x[1], x[2])) continue;
                                list[cnt++] = IDX(g, x[0], x[1], x[2]);
                            }
                }
    }
    return cnt;
}

static void dir_signs(int d, int sg[3]) {
    sg[0] = (d & 4) ? -1 : 1;
    sg[1] = (d & 2) ? -1 : 1;
    sg[2] = (d & 1) ? -1 : 1;
}

static int check_grid(const OGrid* g) {
    for (int a = 0; a < 3; ++a)
        if (g->n[a] < 4 || !(g->h[a] > 0.0)) return -1;
    return 0;
}

/* ---------------------------------------------------------------------------
 * Forward solve, one source.  Returns 0 on success (converged or not), -1 on
 * bad arguments.  *iters = iterations done, *converged = 1 if eps < tol.
 * ------------------------------------------------------------------------- */
int tto_forward(const int* n, int coord, const double* o, const double* h,
                const double* s, const double* xi, const double* eta,
                const double* src_pos, const double* src_par, double kappa, double tol,
                int max_iter, int order, const double* tau_init, double* tau,
                int* iters, int* converged, double* eps_hist) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    if (check_grid(&g) || max_iter < 1) return -1;
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    for (size_t c = 0; c < g.N; ++c) tau[c] = tau_init ? tau_init[c] : 1.0;
    for (int i = S.fb[0]; i <= S.fb[0] + 1; ++i)
        for (int j = S.fb[1]; j <= S.fb[1] + 1; ++j)
            for (int k = S.fb[2]; k <= S.fb[2] + 1; ++k) tau[IDX(&g, i, j, k)] = 1.0;
    size_t* list = NULL;
    size_t* bl = (size_t*)malloc(sizeof(size_t) * boundary_count(&g));
    if (!bl) return -1;
    if (order != 0) {
        list = (size_t*)malloc(sizeof(size_t) * g.N);
        if (!list) { free(bl); return -1; }
    }
    *converged = 0;
    int it;
    for (it = 1; it <= max_iter; ++it) {
        double acc = 0.0;
        for (int d = 0; d < 8; ++d) {
            int sg[3];
            dir_signs(d, sg);
            if (order == 0) {
                for (int a0 = 0; a0 < g.n[0] - 2; ++a0) {
                    int i = sg[0] > 0 ? 1 + a0 : g.n[0] - 2 - a0;
                    for (int a1 = 0; a1 < g.n[1] - 2; ++a1) {
                        int j = sg[1] > 0 ? 1 + a1 : g.n[1] - 2 - a1;
                        for (int a2 = 0; a2 < g.n[2] - 2; ++a2) {
                            int k = sg[2] > 0 ? 1 + a2 : g.n[2] - 2 - a2;
                            if (is_fixed(&S, i, j, k)) continue;
                            size_t c = IDX(&g, i, j, k);
                            double nv = lf_update(&g, &S, kappa, s, xi, eta, tau, i, j, k);
                            acc += fabs(nv - tau[c]);
                            tau[c] = nv;
                        }
                    }
                }
            } else {
                size_t cnt = build_order(&g, &S, sg, order, 0x9E3779B97F4A7C15ULL + 977ULL * (uint64_t)(it * 8 + d), list);
                for (size_t q = 0; q < cnt; ++q) {
                    int i, j, k;
                    unidx(&g, list[q], &i, &j, &k);
                    double nv = lf_update(&g, &S, kappa, s, xi, eta, tau, i, j, k);
                    acc += fabs(nv - tau[list[q]]);
                    tau[list[q]] = nv;
                }
            }
            acc += boundary_pass(&g, &S, tau, bl);
        }
        double eps = acc / (double)g.N;
        if (eps_hist) eps_hist[it - 1] = eps;
        if (eps < tol) { *converged = 1; break; }
    }
    *iters = (it > max_iter) ? max_iter : it;
    free(list);
    free(bl);
    return 0;
}

/* one forward Lax-Friedrichs update at (i,j,k), exposed for tests */
double tto_lf_update(const int* n, int coord, const double* o, const double* h,
                     const double* s, const double* xi, const double* eta,
                     const double* src_pos, const double* src_par, double kappa,
                     const double* tau, int i, int j, int k) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    return lf_update(&g, &S, kappa, s, xi, eta, tau, i, j, k);
}

/* T0 and its scaled gradient at every node: T0[N], t[3][N] (tests) */
void tto_factor_field(const int* n, int coord, const double* o, const double* h,
                      const double* src_pos, const double* src_par, double* T0, double* t) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    for (int i = 0; i < g.n[0]; ++i)
        for (int j = 0; j < g.n[1]; ++j)
            for (int k = 0; k < g.n[2]; ++k) {
                size_t c = IDX(&g, i, j, k);
                double tt[3];
                factor_at(&g, &S, i, j, k, &T0[c], tt);
                for (int a = 0; a < 3; ++a) t[(size_t)a * g.N + c] = tt[a];
            }
}

/* fixed-cell base corner (tests) */
void tto_fixed_base(const int* n, int coord, const double* o, const double* h,
                    const double* src_pos, int* fb) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    for (int a = 0; a < 3; ++a) fb[a] = cell_base(&g, a, src_pos[a]);
}

/* ---------------------------------------------------------------------------
 * Trilinear interpolation at a continuous position.
 * ------------------------------------------------------------------------- */
static int trilinear(const OGrid* g, const double* x, size_t cidx[8], double w[8]) {
    int b[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double lo = g->o[a], hi = g->o[a] + (double)(g->n[a] - 1) * g->h[a];
        if (!(x[a] >= lo && x[a] <= hi)) return -1;
        b[a] = cell_base(g, a, x[a]);
        f[a] = (x[a] - g->o[a]) / g->h[a] - (double)b[a];
    }
    int q = 0;
    for (int c0 = 0; c0 < 2; ++c0)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int c2 = 0; c2 < 2; ++c2) {
                cidx[q] = IDX(g, b[0] + c0, b[1] + c1, b[2] + c2);
                w[q] = (c0 ? f[0] : 1.0 - f[0]) * (c1 ? f[1] : 1.0 - f[1]) * (c2 ? f[2] : 1.0 - f[2]);
                ++q;
            }
    return 0;
}

/* C2: s0, xi0, eta0 = model trilinearly interpolated at the source */
int tto_source_params(const int* n, int coord, const double* o, const double* h,
                      const double* s, const double* xi, const double* eta,
                      int nsrc, const double* src_pos, double* src_par) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    for (int q = 0; q < nsrc; ++q) {
        size_t ci[8];
        double w[8];
        if (trilinear(&g, src_pos + 3 * q, ci, w)) return -1;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int p = 0; p < 8; ++p) { a += w[p] * s[ci[p]]; b += w[p] * xi[ci[p]]; c += w[p] * eta[ci[p]]; }
        src_par[3 * q + 0] = a; src_par[3 * q + 1] = b; src_par[3 * q + 2] = c;
    }
    return 0;
}

/* (R8) T at receivers for one source: T_rec[m] = sum_c w_c T0(c) tau(c) */
int tto_sample(const int* n, int coord, const double* o, const double* h,
               const double* src_pos, const double* src_par, const double* tau,
               int nrec, const double* rec_pos, double* T_rec) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    for (int m = 0; m < nrec; ++m) {
        size_t ci[8];
        double w[8];
        if (trilinear(&g, rec_pos + 3 * m, ci, w)) return -1;
        double acc = 0.0;
        for (int p = 0; p < 8; ++p) {
            int i, j, k;
            unidx(&g, ci[p], &i, &j, &k);
            double T0, t[3];
            factor_at(&g, &S, i, j, k, &T0, t);
            acc += w[p] * T0 * tau[ci[p]];
        }
        T_rec[m] = acc;
    }
    return 0;
}

/* Eqs. (1)-(3), (A2), (A3): chi = alpha*chi_t + beta*chi_cs and R = d chi / d T.
 * T, T_obs, w: [nsrc][nrec]; pairs [npair][2] shared by all sources (R9);
 * wpair [nsrc][npair].  NULL weights mean 1. */
double tto_misfit(int nsrc, int nrec, const double* T, const double* T_obs, const double* w,
                  int npair, const int* pairs, const double* wpair, double alpha, double beta,
                  double* R) {
    double chi = 0.0;
    for (int q = 0; q < nsrc; ++q) {
        for (int m = 0; m < nrec; ++m) {
            size_t c = (size_t)q * nrec + m;
            double ww = w ? w[c] : 1.0;
            double r = T[c] - T_obs[c];
            chi += alpha * 0.5 * ww * r * r;
            R[c] = alpha * ww * r;
        }
        for (int p = 0; p < npair; ++p) {
            int m = pairs[2 * p], i = pairs[2 * p + 1];
            size_t cm = (size_t)q * nrec + m, ci = (size_t)q * nrec + i;
            double ww = wpair ? wpair[(size_t)q * npair + p] : 1.0;
            double r = (T[cm] - T[ci]) - (T_obs[cm] - T_obs[ci]);
            chi += beta * 0.5 * ww * r * r;
            R[cm] += beta * ww * r;
            R[ci] -= beta * ww * r;
        }
    }
    return chi;
}

/* Common-receiver differential misfit gamma * chi_cr (Eq. (4), third misfit)
 * and its adjoint sources (Eq. (A4)), added to R.  T, T_obs, R: [nsrc][nrec];
 * tri [ntri][3] = (n, j, m), the source pair {n, j} at receiver m, each
 * unordered pair listed once (R13); wtri [ntri] or NULL (= 1).  Triples are
 * taken in list order.  Returns gamma * chi_cr, or NAN if an index is out of
 * range. */
double tto_misfit_cr(int nsrc, int nrec, const double* T, const double* T_obs, int ntri, const int* tri,
                     const double* wtri, double gamma, double* R) {
    double chi = 0.0;
    for (int p = 0; p < ntri; ++p) {
        int n = tri[3 * p], j = tri[3 * p + 1], m = tri[3 * p + 2];
        if (n < 0 || n >= nsrc || j < 0 || j >= nsrc || m < 0 || m >= nrec) return NAN;
        size_t cn = (size_t)n * nrec + m, cj = (size_t)j * nrec + m;
        double ww = wtri ? wtri[p] : 1.0;
        /* residual of the differential time T_n - T_j at receiver m */
        double r = (T[cn] - T[cj]) - (T_obs[cn] - T_obs[cj]);
        chi += gamma * 0.5 * ww * r * r;
        R[cn] += gamma * ww * r;
        R[cj] -= gamma * ww * r;
    }
    return chi;
}

/* d chi / d tau for one source: g_c = sum_m R_m w_c(m) T0(c) (dense, [N]) */
int tto_adjoint_rhs(const int* n, int coord, const double* o, const double* h,
                    const double* src_pos, const double* src_par, int nrec, const double* rec_pos,
                    const double* R, double* gr) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    memset(gr, 0, sizeof(double) * g.N);
    for (int m = 0; m < nrec; ++m) {
        size_t ci[8];
        double w[8];
        if (trilinear(&g, rec_pos + 3 * m, ci, w)) return -1;
        for (int p = 0; p < 8; ++p) {
            int i, j, k;
            unidx(&g, ci[p], &i, &j, &k);
            double T0, t[3];
            factor_at(&g, &S, i, j, k, &T0, t);
            gr[ci[p]] += R[m] * w[p] * T0;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint.  Rows of the Jacobian J of the discrete forward system:
 *   fixed node f:       tau_f - 1 = 0                       -> J_ff = 1
 *   boundary node b:    tau_b - tau_b1 = 0                  -> 1, -1
 *   interior node x:    G_x (see lf_update)                 ->
 *       J_xx        = t.MP / H + sum_a 2 beta_a,
 *       J_x,x+e_a   =  alpha_a - beta_a,
 *       J_x,x-e_a   = -alpha_a - beta_a,
 *   alpha_a = T0 g_a (MP)_a / (2 h_a H),  beta_a = sigma_a / (2 h_a).
 * ------------------------------------------------------------------------- */
typedef struct {
    double alpha[3], beta[3], diag;   /* interior rows only */
} OCoef;

static void interior_coef(const OGrid* g, const OSrc* S, double kappa, const double* s,
                          const double* xi, const double* eta, const double* tau,
                          int i, int j, int k, OCoef* C, OLocal* Lout) {
    OLocal L;
    local_state(g, S, kappa, s, xi, eta, tau, i, j, k, &L);
    double dHdt = (L.t[0] * L.MP[0] + L.t[1] * L.MP[1] + L.t[2] * L.MP[2]) / L.H;
    C->diag = dHdt;
    for (int a = 0; a < 3; ++a) {
        C->alpha[a] = L.T0 * L.gm[a] * L.MP[a] / (2.0 * g->h[a] * L.H);
        C->beta[a] = L.sig[a] / (2.0 * g->h[a]);
        C->diag += 2.0 * C->beta[a];
    }
    if (Lout) *Lout = L;
}

/* entries of row x of J: returns the count, fills column indices and values */
static int jac_row(const OGrid* g, const OSrc* S, const OCoef* coef, int i, int j, int k,
                   size_t* col, double* val) {
    size_t c = IDX(g, i, j, k);
    if (is_fixed(S, i, j, k)) { col[0] = c; val[0] = 1.0; return 1; }
    int as = astar_of(g, i, j, k);
    if (as >= 0) {
        col[0] = c; val[0] = 1.0;
        col[1] = bnd_ref(g, i, j, k, as); val[1] = -1.0;
        return 2;
    }
    size_t st[3] = {(size_t)g->n[1] * g->n[2], (size_t)g->n[2], 1};
    const OCoef* C = &coef[c];
    col[0] = c; val[0] = C->diag;
    int q = 1;
    for (int a = 0; a < 3; ++a) {
        col[q] = c + st[a]; val[q] = C->alpha[a] - C->beta[a]; ++q;
        col[q] = c - st[a]; val[q] = -C->alpha[a] - C->beta[a]; ++q;
    }
    return q;
}

/* column equation of J^T lambda = rhs at node y, solved for lambda_y:
 * every row that can reference y lies within distance 1 of y along one axis
 * (candidates up to distance 2 are scanned; jac_row decides). */
static double transposed_update(const OGrid* g, const OSrc* S, const OCoef* coef,
                                const double* rhs, const double* lam, int i, int j, int k) {
    size_t y = IDX(g, i, j, k);
    double acc = rhs[y], diag = 0.0;
    int base[3] = {i, j, k};
    for (int cand = 0; cand < 13; ++cand) {
        int x[3] = {i, j, k};
        if (cand > 0) {
            int a = (cand - 1) / 4, which = (cand - 1) % 4;
            static const int off[4] = {1, -1, 2, -2};
            x[a] = base[a] + off[which];
            if (x[a] < 0 || x[a] >= g->n[a]) continue;
        }
        size_t cols[7];
        double vals[7];
        int cnt = jac_row(g, S, coef, x[0], x[1], x[2], cols, vals);
        size_t xc = IDX(g, x[0], x[1], x[2]);
        for (int p = 0; p < cnt; ++p) {
            if (cols[p] != y) continue;
            if (xc == y) diag += vals[p];
            else acc -= vals[p] * lam[xc];
        }
    }
    return acc / diag;
}

/* adjoint coefficients of every interior non-fixed node from converged tau.
 * Layout of out: [7][N] = alpha0..2, beta0..2, diag (zero elsewhere). */
void tto_adjoint_coeffs(const int* n, int coord, const double* o, const double* h,
                        const double* s, const double* xi, const double* eta,
                        const double* src_pos, const double* src_par, double kappa,
                        const double* tau, double* out) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    memset(out, 0, sizeof(double) * 7 * g.N);
    for (int i = 1; i < g.n[0] - 1; ++i)
        for (int j = 1; j < g.n[1] - 1; ++j)
            for (int k = 1; k < g.n[2] - 1; ++k) {
                if (is_fixed(&S, i, j, k)) continue;
                OCoef C;
                interior_coef(&g, &S, kappa, s, xi, eta, tau, i, j, k, &C, NULL);
                size_t c = IDX(&g, i, j, k);
                for (int a = 0; a < 3; ++a) {
                    out[(size_t)a * g.N + c] = C.alpha[a];
                    out[(size_t)(3 + a) * g.N + c] = C.beta[a];
                }
                out[(size_t)6 * g.N + c] = C.diag;
            }
}

int tto_adjoint(const int* n, int coord, const double* o, const double* h,
                const double* s, const double* xi, const double* eta,
                const double* src_pos, const double* src_par, double kappa,
                const double* tau, const double* rhs, double tol, int max_iter, int order,
                double* lam, int* iters, int* converged, double* eps_hist) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    if (check_grid(&g) || max_iter < 1) return -1;
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    OCoef* coef = (OCoef*)calloc(g.N, sizeof(OCoef));
    size_t* list = NULL;
    size_t* bl = (size_t*)malloc(sizeof(size_t) * boundary_count(&g));
    if (!coef || !bl) { free(coef); free(bl); return -1; }
    if (order != 0) {
        list = (size_t*)malloc(sizeof(size_t) * g.N);
        if (!list) { free(coef); free(bl); return -1; }
    }
    for (int i = 1; i < g.n[0] - 1; ++i)
        for (int j = 1; j < g.n[1] - 1; ++j)
            for (int k = 1; k < g.n[2] - 1; ++k) {
                if (is_fixed(&S, i, j, k)) continue;
                interior_coef(&g, &S, kappa, s, xi, eta, tau, i, j, k, &coef[IDX(&g, i, j, k)], NULL);
            }
    memset(lam, 0, sizeof(double) * g.N);
    *converged = 0;
    int it;
    for (it = 1; it <= max_iter; ++it) {
        double dsum = 0.0;
        for (int d = 0; d < 8; ++d) {
            int sg[3];
            dir_signs(d, sg);
            if (order == 0) {
                for (int a0 = 0; a0 < g.n[0] - 2; ++a0) {
                    int i = sg[0] > 0 ? 1 + a0 : g.n[0] - 2 - a0;
                    for (int a1 = 0; a1 < g.n[1] - 2; ++a1) {
                        int j = sg[1] > 0 ? 1 + a1 : g.n[1] - 2 - a1;
                        for (int a2 = 0; a2 < g.n[2] - 2; ++a2) {
                            int k = sg[2] > 0 ? 1 + a2 : g.n[2] - 2 - a2;
                            if (is_fixed(&S, i, j, k)) continue;
                            size_t c = IDX(&g, i, j, k);
                            double nv = transposed_update(&g, &S, coef, rhs, lam, i, j, k);
                            dsum += fabs(nv - lam[c]);
                            lam[c] = nv;
                        }
                    }
                }
            } else {
                size_t cnt = build_order(&g, &S, sg, order, 0xD1B54A32D192ED03ULL + 131ULL * (uint64_t)(it * 8 + d), list);
                for (size_t q = 0; q < cnt; ++q) {
                    int i, j, k;
                    unidx(&g, list[q], &i, &j, &k);
                    double nv = transposed_update(&g, &S, coef, rhs, lam, i, j, k);
                    dsum += fabs(nv - lam[list[q]]);
                    lam[list[q]] = nv;
                }
            }
            /* transposed boundary pass, groups a* = 2, 1, 0 */
            for (int as = 2; as >= 0; --as) {
                size_t cnt = boundary_group(&g, as, bl);
                for (size_t q = 0; q < cnt; ++q) {
                    int i, j, k;
                    unidx(&g, bl[q], &i, &j, &k);
                    if (is_fixed(&S, i, j, k)) continue;
                    double nv = transposed_update(&g, &S, coef, rhs, lam, i, j, k);
                    dsum += fabs(nv - lam[bl[q]]);
                    lam[bl[q]] = nv;
                }
            }
        }
        double asum = 0.0;
        for (size_t c = 0; c < g.N; ++c) asum += fabs(lam[c]);
        double eps = dsum / (asum > 1e-300 ? asum : 1e-300);
        if (eps_hist) eps_hist[it - 1] = eps;
        if (eps < tol) { *converged = 1; break; }
    }
    *iters = (it > max_iter) ? max_iter : it;
    free(coef);
    free(list);
    free(bl);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Earthquake relocation, Eq. (10) and App. B (R15).
 * ------------------------------------------------------------------------- */

/* corners of the cell holding x (as trilinear) and the gradient of each
 * corner's weight with respect to the grid coordinates */
static int trilinear_grad(const OGrid* g, const double* x, size_t cidx[8], double dw[8][3]) {
    int b[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double lo = g->o[a], hi = g->o[a] + (double)(g->n[a] - 1) * g->h[a];
        if (!(x[a] >= lo && x[a] <= hi)) return -1;
        b[a] = cell_base(g, a, x[a]);
        f[a] = (x[a] - g->o[a]) / g->h[a] - (double)b[a];
    }
    int q = 0;
    for (int c0 = 0; c0 < 2; ++c0)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int c2 = 0; c2 < 2; ++c2) {
                int c[3] = {c0, c1, c2};
                cidx[q] = IDX(g, b[0] + c0, b[1] + c1, b[2] + c2);
                for (int a = 0; a < 3; ++a) {
                    double v = (c[a] ? 1.0 : -1.0) / g->h[a];
                    for (int e = 0; e < 3; ++e)
                        if (e != a) v *= c[e] ? f[e] : 1.0 - f[e];
                    dw[q][a] = v;
                }
                ++q;
            }
    return 0;
}

/* T[n][m] = Gamma_m(x_n) + t_n for nev earthquakes and nfield receiver fields
 * (field m: source at field_pos[m], constants field_par[m], tau [N]);
 * ev_t0 [nev] or NULL (= 0).  -1 if an earthquake lies outside the grid. */
int tto_reloc_times(const int* n, int coord, const double* o, const double* h, int nfield,
                    const double* field_pos, const double* field_par, const double* tau, int nev,
                    const double* ev_pos, const double* ev_t0, double* T) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    for (int m = 0; m < nfield; ++m) {
        double col[1];
        for (int q = 0; q < nev; ++q) {
            if (tto_sample(n, coord, o, h, field_pos + 3 * m, field_par + 3 * m, tau + (size_t)m * g.N, 1,
                           ev_pos + 3 * q, col))
                return -1;
            T[(size_t)q * nfield + m] = col[0] + (ev_t0 ? ev_t0[q] : 0.0);
        }
    }
    return 0;
}

/* Eq. (10): K[n] = (sum_m R[n][m] dGamma_m/dx_a(x_n) for a = 0, 1, 2,
 * sum_m R[n][m]), R [nev][nfield] the adjoint sources of the misfit in
 * T[n][m] (tto_misfit, tto_misfit_cr); K [nev][4]. */
int tto_reloc_kernel(const int* n, int coord, const double* o, const double* h, int nfield,
                     const double* field_pos, const double* field_par, const double* tau, int nev,
                     const double* ev_pos, const double* R, double* K) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    for (int q = 0; q < nev; ++q) {
        size_t ci[8];
        double dw[8][3];
        if (trilinear_grad(&g, ev_pos + 3 * q, ci, dw)) return -1;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int m = 0; m < nfield; ++m) {
            OSrc S;
            src_init(&S, &g, field_pos + 3 * m, field_par + 3 * m);
            double gr[3] = {0.0, 0.0, 0.0};
            for (int p = 0; p < 8; ++p) {
                int i, j, k;
                unidx(&g, ci[p], &i, &j, &k);
                double T0, t[3];
                factor_at(&g, &S, i, j, k, &T0, t);
                double Gc = T0 * tau[(size_t)m * g.N + ci[p]];
                for (int a = 0; a < 3; ++a) gr[a] += dw[p][a] * Gc;
            }
            double r = R[(size_t)q * nfield + m];
            for (int a = 0; a < 3; ++a) acc[a] += r * gr[a];
            acc[3] += r;
        }
        for (int a = 0; a < 4; ++a) K[(size_t)q * 4 + a] = acc[a];
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Continuous adjoint of Eq. (5), (R14).
 * ------------------------------------------------------------------------- */

/* scaled gradient p of T = T0 tau at any node: central differences of tau on
 * axes where the node is interior, one-sided where it is on the boundary */
static void grad_T_any(const OGrid* g, const OSrc* S, const double* tau, int i, int j, int k, double p[3]) {
    double T0, t[3], gm[3];
    factor_at(g, S, i, j, k, &T0, t);
    metric(g, i, j, gm);
    int id[3] = {i, j, k};
    size_t c = IDX(g, i, j, k);
    size_t st[3] = {(size_t)g->n[1] * g->n[2], (size_t)g->n[2], 1};
    for (int a = 0; a < 3; ++a) {
        double q;
        if (id[a] == 0) q = (tau[c + st[a]] - tau[c]) / g->h[a];
        else if (id[a] == g->n[a] - 1) q = (tau[c] - tau[c - st[a]]) / g->h[a];
        else q = (tau[c + st[a]] - tau[c - st[a]]) / (2.0 * g->h[a]);
        p[a] = T0 * gm[a] * q + tau[c] * t[a];
    }
}

/* w = -M p at every node (the transport velocity of Eq. (5)), stored [3][N] */
static void velocity_field(const OGrid* g, const OSrc* S, const double* xi, const double* eta, const double* tau,
                           double* w) {
    for (int i = 0; i < g->n[0]; ++i)
        for (int j = 0; j < g->n[1]; ++j)
            for (int k = 0; k < g->n[2]; ++k) {
                size_t c = IDX(g, i, j, k);
                double p[3];
                grad_T_any(g, S, tau, i, j, k, p);
                w[c] = -p[0];
                w[g->N + c] = -((1.0 - 2.0 * xi[c]) * p[1] + 2.0 * eta[c] * p[2]);
                w[2 * g->N + c] = -(2.0 * eta[c] * p[1] + (1.0 + 2.0 * xi[c]) * p[2]);
            }
}

/* The velocity field w [3][N] that tto_adjoint_cont transports P with, for a
 * given tau (any field, not only a converged one).  Returns -1 on bad input. */
int tto_cont_velocity(const int* n, int coord, const double* o, const double* h, const double* xi,
                      const double* eta, const double* src_pos, const double* src_par, const double* tau, double* w) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    if (check_grid(&g)) return -1;
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    velocity_field(&g, &S, xi, eta, tau, w);
    return 0;
}

/* control-volume extent of node index idx along axis a (coordinate units) */
static double cv_extent(const OGrid* g, int a, int idx) {
    return (idx == 0 || idx == g->n[a] - 1) ? 0.5 * g->h[a] : g->h[a];
}

/* area of the face of node (i,j,k) normal to axis a at coordinate xf of that
 * axis (the face midpoint between two nodes, or the node itself on a grid face) */
static double face_area(const OGrid* g, int a, int i, int j, int k, double xf) {
    int id[3] = {i, j, k};
    double A = 1.0;
    for (int b = 0; b < 3; ++b)
        if (b != a) A *= cv_extent(g, b, id[b]);
    if (g->coord == 1) {
        double r = cval(g, 0, i), th = cval(g, 1, j);
        if (a == 0) A *= xf * xf * cos(th);   /* r = const:     r^2 cos(theta) dtheta dphi */
        else if (a == 1) A *= r * cos(xf);    /* theta = const: r cos(theta) dr dphi */
        else A *= r;                          /* phi = const:   r dr dtheta */
    }
    return A;
}

/* The finite-volume row of node x, solved by Gauss-Seidel:
 *   diag = sum over faces of A max(u_out, 0)          (outflow),
 *   off[2a + side] = A min(u_out, 0) for the neighbour x + (side ? -1 : +1) e_a
 *                    (0 if it is fixed or outside),
 * u_out the outward normal velocity of the face. */
typedef struct {
    double diag, off[6];
} OCRow;

static void cont_row(const OGrid* g, const OSrc* S, const double* w, int i, int j, int k, OCRow* R) {
    int id[3] = {i, j, k};
    size_t c = IDX(g, i, j, k);
    size_t st[3] = {(size_t)g->n[1] * g->n[2], (size_t)g->n[2], 1};
    R->diag = 0.0;
    for (int a = 0; a < 3; ++a) {
        for (int side = 0; side < 2; ++side) {
            int sg = side == 0 ? 1 : -1;
            int nbi = id[a] + sg;
            double xa = cval(g, a, id[a]);
            double u, A;
            int inside = nbi >= 0 && nbi < g->n[a];
            if (inside) {
                size_t nb = sg > 0 ? c + st[a] : c - st[a];
                u = sg * 0.5 * (w[(size_t)a * g->N + c] + w[(size_t)a * g->N + nb]);
                A = face_area(g, a, i, j, k, 0.5 * (xa + cval(g, a, nbi)));
            } else {
                u = sg * w[(size_t)a * g->N + c];
                A = face_area(g, a, i, j, k, xa);
            }
            R->diag += A * (u > 0.0 ? u : 0.0);
            double off = 0.0;
            if (inside) {
                int q[3] = {i, j, k};
                q[a] = nbi;
                if (!is_fixed(S, q[0], q[1], q[2])) off = A * (u < 0.0 ? u : 0.0);
            }
            R->off[2 * a + side] = off;
        }
    }
}

static double cont_update(const OGrid* g, const OCRow* R, const double* b, const double* P, size_t c) {
    size_t st[3] = {(size_t)g->n[1] * g->n[2], (size_t)g->n[2], 1};
    if (!(R->diag > 0.0)) return 0.0;
    double acc = b[c];
    for (int a = 0; a < 3; ++a) {
        if (R->off[2 * a] != 0.0) acc -= R->off[2 * a] * P[c + st[a]];
        if (R->off[2 * a + 1] != 0.0) acc -= R->off[2 * a + 1] * P[c - st[a]];
    }
    return acc / R->diag;
}

/* P of Eq. (5) for one source at the converged tau.  Receivers inject
 * b_x = sum_m R_m w_x(m) (trilinear weights).  Iteration as tto_adjoint:
 * eps = sum |dP| / max(sum |P|, 1e-300).  Returns -1 on bad input or a
 * receiver outside the grid. */
int tto_adjoint_cont(const int* n, int coord, const double* o, const double* h,
                     const double* s, const double* xi, const double* eta,
                     const double* src_pos, const double* src_par, const double* tau,
                     int nrec, const double* rec_pos, const double* Rm, double tol, int max_iter,
                     double* P, int* iters, int* converged, double* eps_hist) {
    (void)s;
    OGrid g;
    grid_init(&g, n, coord, o, h);
    if (check_grid(&g) || max_iter < 1) return -1;
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    double* w = (double*)malloc(sizeof(double) * 3 * g.N);
    double* b = (double*)calloc(g.N, sizeof(double));
    OCRow* rows = (OCRow*)calloc(g.N, sizeof(OCRow));
    size_t nbnd = boundary_count(&g);
    size_t* bl = (size_t*)malloc(sizeof(size_t) * nbnd);
    double* tmp = (double*)malloc(sizeof(double) * nbnd);
    if (!w || !b || !rows || !bl || !tmp) { free(w); free(b); free(rows); free(bl); free(tmp); return -1; }
    velocity_field(&g, &S, xi, eta, tau, w);
    for (int m = 0; m < nrec; ++m) {
        size_t ci[8];
        double wt[8];
        if (trilinear(&g, rec_pos + 3 * m, ci, wt)) { free(w); free(b); free(rows); free(bl); free(tmp); return -1; }
        for (int q = 0; q < 8; ++q) b[ci[q]] += Rm[m] * wt[q];
    }
    for (int i = 0; i < g.n[0]; ++i)
        for (int j = 0; j < g.n[1]; ++j)
            for (int k = 0; k < g.n[2]; ++k)
                if (!is_fixed(&S, i, j, k)) cont_row(&g, &S, w, i, j, k, &rows[IDX(&g, i, j, k)]);
    /* boundary nodes in index order */
    size_t nb = 0;
    for (int i = 0; i < g.n[0]; ++i)
        for (int j = 0; j < g.n[1]; ++j)
            for (int k = 0; k < g.n[2]; ++k)
                if (astar_of(&g, i, j, k) >= 0) bl[nb++] = IDX(&g, i, j, k);
    memset(P, 0, sizeof(double) * g.N);
    *converged = 0;
    int it;
    for (it = 1; it <= max_iter; ++it) {
        double dsum = 0.0;
        for (int d = 0; d < 8; ++d) {
            int sg[3];
            dir_signs(d, sg);
            for (int a0 = 0; a0 < g.n[0] - 2; ++a0) {
                int i = sg[0] > 0 ? 1 + a0 : g.n[0] - 2 - a0;
                for (int a1 = 0; a1 < g.n[1] - 2; ++a1) {
                    int j = sg[1] > 0 ? 1 + a1 : g.n[1] - 2 - a1;
                    for (int a2 = 0; a2 < g.n[2] - 2; ++a2) {
                        int k = sg[2] > 0 ? 1 + a2 : g.n[2] - 2 - a2;
                        if (is_fixed(&S, i, j, k)) continue;
                        size_t c = IDX(&g, i, j, k);
                        double nv = cont_update(&g, &rows[c], b, P, c);
                        dsum += fabs(nv - P[c]);
                        P[c] = nv;
                    }
                }
            }
            /* Jacobi pass over the boundary nodes: every new value from the
             * values present before the pass */
            for (size_t q = 0; q < nb; ++q) {
                int i, j, k;
                unidx(&g, bl[q], &i, &j, &k);
                tmp[q] = is_fixed(&S, i, j, k) ? 0.0 : cont_update(&g, &rows[bl[q]], b, P, bl[q]);
            }
            for (size_t q = 0; q < nb; ++q) {
                dsum += fabs(tmp[q] - P[bl[q]]);
                P[bl[q]] = tmp[q];
            }
        }
        double asum = 0.0;
        for (size_t c = 0; c < g.N; ++c) asum += fabs(P[c]);
        double eps = dsum / (asum > 1e-300 ? asum : 1e-300);
        if (eps_hist) eps_hist[it - 1] = eps;
        if (eps < tol) { *converged = 1; break; }
    }
    *iters = (it > max_iter) ? max_iter : it;
    free(w); free(b); free(rows); free(bl); free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Discrete gradients (the kernels of Eqs. (6)-(8) before the Eq. (9)
 * normalisation): at interior non-fixed nodes
 *   d chi/d s   = lambda,
 *   d chi/d xi  = lambda (P_theta^2 - P_phi^2) / H,
 *   d chi/d eta = -2 lambda P_theta P_phi / H,
 * with P, H the local quantities at the converged tau.  grad is [3][N];
 * accumulate != 0 adds to it.
 * ------------------------------------------------------------------------- */
void tto_kernel(const int* n, int coord, const double* o, const double* h,
                const double* s, const double* xi, const double* eta,
                const double* src_pos, const double* src_par, double kappa,
                const double* tau, const double* lam, double* grad, int accumulate) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    OSrc S;
    src_init(&S, &g, src_pos, src_par);
    if (!accumulate) memset(grad, 0, sizeof(double) * 3 * g.N);
    for (int i = 1; i < g.n[0] - 1; ++i)
        for (int j = 1; j < g.n[1] - 1; ++j)
            for (int k = 1; k < g.n[2] - 1; ++k) {
                if (is_fixed(&S, i, j, k)) continue;
                OLocal L;
                local_state(&g, &S, kappa, s, xi, eta, tau, i, j, k, &L);
                size_t c = IDX(&g, i, j, k);
                double l = lam[c];
                grad[c] += l;
                grad[g.N + c] += l * (L.P[1] * L.P[1] - L.P[2] * L.P[2]) / L.H;
                grad[2 * g.N + c] += -2.0 * l * L.P[1] * L.P[2] / L.H;
            }
}

/* Eq. (9) quadrature volume of each node (trapezoid weights: 1/2 per axis on
 * which the node is on the boundary); spherical volume element r^2 cos(theta). */
void tto_node_volume(const int* n, int coord, const double* o, const double* h, double* V) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    for (int i = 0; i < g.n[0]; ++i)
        for (int j = 0; j < g.n[1]; ++j)
            for (int k = 0; k < g.n[2]; ++k) {
                double v = g.h[0] * g.h[1] * g.h[2];
                if (g.coord == 1) {
                    double r = cval(&g, 0, i), th = cval(&g, 1, j);
                    v *= r * r * cos(th);
                }
                if (i == 0 || i == g.n[0] - 1) v *= 0.5;
                if (j == 0 || j == g.n[1] - 1) v *= 0.5;
                if (k == 0 || k == g.n[2] - 1) v *= 0.5;
                V[IDX(&g, i, j, k)] = v;
            }
}

/* Kernel-density normalisation (Eqs. (18)-(19)).
 * The density of the event kernels is the adjoint field P_hat of Eq. (5) with
 * every adjoint source R = 1, summed over sources.  In this discretisation the
 * s-gradient of a source's misfit is its adjoint field at the interior
 * non-fixed nodes (zero elsewhere: the model enters only the interior
 * equations), and K_s = s (d chi / d s) / V (Eq. (9)) with K_s = P s^2, so
 * P = (d chi / d s) / (s V).  Given dens = the s-gradient summed over sources of
 * the R = 1 adjoint fields, and grad [3][N] = the summed discrete gradients of
 * the misfit, per node x:
 *   Kd(x)   = dens(x) / (s(x) V(x))
 *   K_s(x)  = s(x) grad_s(x) / V(x) / (Kd(x) + eps)^zeta
 *   K_xi(x) = grad_xi(x) / V(x) / (Kd(x) + eps)^zeta,  K_eta likewise. */
void tto_kernel_density(const int* n, int coord, const double* o, const double* h, const double* s,
                        const double* dens, const double* grad, double eps, double zeta, double* K, double* Kd) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    const long N = (long)g.n[0] * g.n[1] * g.n[2];
    double* V = (double*)malloc(sizeof(double) * (size_t)N);
    tto_node_volume(n, coord, o, h, V);
    for (long x = 0; x < N; ++x) {
        const double d = dens[x] / (s[x] * V[x]);
        const double w = pow(d + eps, zeta);
        Kd[x] = d;
        K[x] = s[x] * grad[x] / V[x] / w;
        K[N + x] = grad[N + x] / V[x] / w;
        K[2 * N + x] = grad[2 * N + x] / V[x] / w;
    }
    free(V);
}

/* Multiple-grid parameterisation (Eqs. (11)-(17)).
 * H inversion grids; grid h has ascending node coordinates c_a^h[0..m_a-1] on
 * each axis a (r, theta, phi or z, y, x).  One-dimensional tent functions
 * (Eqs. (12)-(14)): node i is (x - c[i-1]) / (c[i] - c[i-1]) on [c[i-1], c[i]]
 * (i > 0), (c[i+1] - x) / (c[i+1] - c[i]) on [c[i], c[i+1]] (i < m - 1), and 0
 * elsewhere, in particular outside [c[0], c[m-1]].  B_l^h = u_i v_j w_k / H
 * (Eq. (11)); the coefficient index l of the paper is stored as [i][j][k]
 * (k fastest), grid after grid.  Coordinates of all grids are concatenated:
 * grid h's r, theta, phi arrays in turn; m holds m_a^h as [H][3]. */
static double tent(const double* c, int m, int i, double x) {
    if (i > 0 && x >= c[i - 1] && x <= c[i]) return (x - c[i - 1]) / (c[i] - c[i - 1]);
    if (i < m - 1 && x >= c[i] && x <= c[i + 1]) return (c[i + 1] - x) / (c[i + 1] - c[i]);
    if (m == 1 && x == c[0]) return 1.0;
    return 0.0;
}

/* Projection of kernels onto the basis (Eq. (17)), by node quadrature:
 * out[h][p][i][j][k] = sum_x K[p](x) B_(i,j,k)^h(x) V(x), p = s, xi, eta. */
void tto_mg_project(const int* n, int coord, const double* o, const double* h, int H, const int* m,
                    const double* coords, const double* K, double* out) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    const long N = (long)g.N;
    double* V = (double*)malloc(sizeof(double) * (size_t)N);
    tto_node_volume(n, coord, o, h, V);
    const double* cg = coords;
    double* og = out;
    for (int q = 0; q < H; ++q) {
        const int* mq = m + 3 * q;
        const double *c0 = cg, *c1 = cg + mq[0], *c2 = cg + mq[0] + mq[1];
        const long M = (long)mq[0] * mq[1] * mq[2];
        for (long e = 0; e < 3 * M; ++e) og[e] = 0.0;
        for (int ci = 0; ci < mq[0]; ++ci)
            for (int cj = 0; cj < mq[1]; ++cj)
                for (int ck = 0; ck < mq[2]; ++ck) {
                    double acc[3] = {0.0, 0.0, 0.0};
                    for (int i = 0; i < g.n[0]; ++i) {
                        const double u = tent(c0, mq[0], ci, cval(&g, 0, i));
                        if (u == 0.0) continue;
                        for (int j = 0; j < g.n[1]; ++j) {
                            const double v = tent(c1, mq[1], cj, cval(&g, 1, j));
                            if (v == 0.0) continue;
                            for (int k = 0; k < g.n[2]; ++k) {
                                const double w = tent(c2, mq[2], ck, cval(&g, 2, k));
                                if (w == 0.0) continue;
                                const long x = IDX(&g, i, j, k);
                                const double b = u * v * w / H * V[x];
                                for (int p = 0; p < 3; ++p) acc[p] += K[p * N + x] * b;
                            }
                        }
                    }
                    const long l = ((long)ci * mq[1] + cj) * mq[2] + ck;
                    for (int p = 0; p < 3; ++p) og[p * M + l] = acc[p];
                }
        cg += mq[0] + mq[1] + mq[2];
        og += 3 * M;
    }
    free(V);
}

/* Expansion of coefficients into fields (Eq. (15)):
 * field[p](x) = sum_h sum_(i,j,k) C[h][p][i][j][k] B_(i,j,k)^h(x). */
void tto_mg_expand(const int* n, int coord, const double* o, const double* h, int H, const int* m,
                   const double* coords, const double* C, double* field) {
    OGrid g;
    grid_init(&g, n, coord, o, h);
    const long N = (long)g.N;
    for (long e = 0; e < 3 * N; ++e) field[e] = 0.0;
    const double* cg = coords;
    const double* Cg = C;
    for (int q = 0; q < H; ++q) {
        const int* mq = m + 3 * q;
        const double *c0 = cg, *c1 = cg + mq[0], *c2 = cg + mq[0] + mq[1];
        const long M = (long)mq[0] * mq[1] * mq[2];
        for (int i = 0; i < g.n[0]; ++i)
            for (int j = 0; j < g.n[1]; ++j)
                for (int k = 0; k < g.n[2]; ++k) {
                    const long x = IDX(&g, i, j, k);
                    for (int ci = 0; ci < mq[0]; ++ci) {
                        const double u = tent(c0, mq[0], ci, cval(&g, 0, i));
                        if (u == 0.0) continue;
                        for (int cj = 0; cj < mq[1]; ++cj) {
                            const double v = tent(c1, mq[1], cj, cval(&g, 1, j));
                            if (v == 0.0) continue;
                            for (int ck = 0; ck < mq[2]; ++ck) {
                                const double w = tent(c2, mq[2], ck, cval(&g, 2, k));
                                if (w == 0.0) continue;
                                const long l = ((long)ci * mq[1] + cj) * mq[2] + ck;
                                for (int p = 0; p < 3; ++p) field[p * N + x] += Cg[p * M + l] * u * v * w / H;
                            }
                        }
                    }
                }
        cg += mq[0] + mq[1] + mq[2];
        Cg += 3 * M;
    }
}

// tt_aux.hip -- CDNA4 (gfx950) kernels of libtt that run once per inversion
// step outside the solves: misfits and adjoint sources (Eqs. (1)-(4),
// (A2)-(A4)), relocation kernels (Eq. (10), App. B), the multiple-grid
// parameterisation (Eqs. (11)-(17)) and the kernel-density normalisation
// (Eqs. (18)-(19)).  All reductions run in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

__global__ void __launch_bounds__(256) k_misfit(int nsrc, int nrec, const double* __restrict__ T,
                                                const double* __restrict__ Tobs, const double* __restrict__ w,
                                                int npair, const int32_t* __restrict__ pairs,
                                                const double* __restrict__ wpair, double alpha, double beta,
                                                double* __restrict__ R, double* __restrict__ chi) {
    __shared__ double sh[4];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    double part = 0.0;
    for (int q = threadIdx.x; q < nsrc; q += blockDim.x) {
        const long long base = (long long)q * nrec;
        for (int m = 0; m < nrec; ++m) {
            const double ww = w ? w[base + m] : 1.0;
            const double r = T[base + m] - Tobs[base + m];
            part += alpha * 0.5 * ww * r * r;
            R[base + m] = alpha * ww * r;
        }
        for (int p = 0; p < npair; ++p) {
            const int m = pairs[2 * p], i = pairs[2 * p + 1];
            if (m < 0 || m >= nrec || i < 0 || i >= nrec) {
                bad = 1;
                continue;
            }
            const double ww = wpair ? wpair[(long long)q * npair + p] : 1.0;
            const double r = (T[base + m] - T[base + i]) - (Tobs[base + m] - Tobs[base + i]);
            part += beta * 0.5 * ww * r * r;
            R[base + m] += beta * ww * r;
            R[base + i] -= beta * ww * r;
        }
    }
    const double tot = block_sum256(part, sh);
    if (threadIdx.x == 0) *chi = bad ? __builtin_nan("") : tot;
}

// Common-receiver differential misfit (Eq. (4), third misfit) and its adjoint
// sources (Eq. (A4)), added to R and chi.
//
// Adjoint sources: one wave per receiver m.  The wave stages 64 of the
// receiver's pairs at a time (indices and gamma w r in LDS); lane l owns source
// n = base + l and adds the staged contributions that name it, in list order,
// to its R[n][m] -- the additions each element receives come in the order of
// the pair list, as in the plain definition, and no two lanes write one
// element.
constexpr int kCrStage = 64;

__global__ void __launch_bounds__(64) k_misfit_cr_R(int nsrc, int nrec, const double* __restrict__ T,
                                                    const double* __restrict__ Tobs, const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ pair, const double* __restrict__ wcr,
                                                    double gamma, double* __restrict__ R) {
    __shared__ int sn[kCrStage], sj[kCrStage];
    __shared__ double sg[kCrStage];
    const int m = blockIdx.x;
    const int p0 = off[m], p1 = off[m + 1];
    if (p0 < 0 || p1 <= p0 || !pair) return;  // nothing to add (malformed offsets: chi reports it)
    for (int base = 0; base < nsrc; base += kCrStage) {
        const int n = base + (int)threadIdx.x;
        const long long cn = (long long)n * nrec + m;
        double acc = n < nsrc ? R[cn] : 0.0;
        bool touched = false;
        for (int pc = p0; pc < p1; pc += kCrStage) {
            const int p = pc + (int)threadIdx.x;
            int a = -1, b = -1;
            double g = 0.0;
            if (p < p1) {
                a = pair[2 * p];
                b = pair[2 * p + 1];
                if (a >= 0 && a < nsrc && b >= 0 && b < nsrc) {
                    const long long ca = (long long)a * nrec + m, cb = (long long)b * nrec + m;
                    const double ww = wcr ? wcr[p] : 1.0;
                    g = gamma * ww * ((T[ca] - T[cb]) - (Tobs[ca] - Tobs[cb]));
                } else {
                    a = b = -1;
                }
            }
            sn[threadIdx.x] = a;
            sj[threadIdx.x] = b;
            sg[threadIdx.x] = g;
            __syncthreads();
            const int cnt = min(kCrStage, p1 - pc);
            for (int q = 0; q < cnt; ++q) {
                if (sn[q] == n) {
                    acc += sg[q];
                    touched = true;
                }
                if (sj[q] == n) {
                    acc -= sg[q];
                    touched = true;
                }
            }
            __syncthreads();
        }
        if (n < nsrc && touched) R[cn] = acc;
    }
}

// gamma chi_cr over all pairs: one block, pair p of the flat list taken by
// thread p mod 1024 (its receiver found by binary search in the offsets, staged
// in LDS when they fit), fixed-order block reduction; malformed offsets or
// indices make chi NaN.
constexpr int kCrOffLds = 8192;

__global__ void __launch_bounds__(1024) k_misfit_cr_chi(int nsrc, int nrec, const double* __restrict__ T,
                                                        const double* __restrict__ Tobs,
                                                        const int32_t* __restrict__ off_g,
                                                        const int32_t* __restrict__ pair,
                                                        const double* __restrict__ wcr, double gamma,
                                                        double* __restrict__ chi) {
    __shared__ double sh[16];
    __shared__ int bad;
    __shared__ int offl[kCrOffLds];
    const bool staged = nrec + 1 <= kCrOffLds;
    if (staged)
        for (int m = threadIdx.x; m <= nrec; m += blockDim.x) offl[m] = off_g[m];
    if (threadIdx.x == 0) bad = (off_g[0] != 0);
    __syncthreads();
    const int32_t* off = staged ? offl : off_g;
    for (int m = threadIdx.x; m < nrec; m += blockDim.x)
        if (off[m + 1] < off[m]) bad = 1;
    __syncthreads();
    const int total = bad ? 0 : off[nrec];
    if (total > 0 && !pair) bad = 1;
    double part = 0.0;
    if (!bad) {
        for (int p = threadIdx.x; p < total; p += blockDim.x) {
            int lo = 0, hi = nrec;  // off[lo] <= p < off[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (off[mid] <= p) lo = mid;
                else hi = mid;
            }
            const int n = pair[2 * p], j = pair[2 * p + 1];
            if (n < 0 || n >= nsrc || j < 0 || j >= nsrc) {
                bad = 1;
                continue;
            }
            const long long cn = (long long)n * nrec + lo, cj = (long long)j * nrec + lo;
            const double ww = wcr ? wcr[p] : 1.0;
            const double r = (T[cn] - T[cj]) - (Tobs[cn] - Tobs[cj]);
            part += gamma * 0.5 * ww * r * r;
        }
    }
    part = wave_sum(part);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int q = 0; q < 16; ++q) tot += sh[q];
        *chi = bad ? __builtin_nan("") : *chi + tot;
    }
}

// ------------------------------------------------ relocation (Eq. (10), App. B)
// T[n][m] = Gamma_m(x_n) + t_n: field m (receiver m taken as the source) sampled
// at earthquake n by its trilinear interpolant, plus the origin-time shift.
template <int COORD>
__global__ void __launch_bounds__(256) k_reloc_times(Geo G, Tabs T, const Src* __restrict__ fsrc, int nfield,
                                                     const double* __restrict__ tau_all, int nev,
                                                     const double* __restrict__ ev, const double* __restrict__ t0,
                                                     double* __restrict__ out) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)nev * nfield) return;
    const int n = (int)(q / nfield), m = (int)(q % nfield);
    const Src S = fsrc[m];
    const double* tau = tau_all + (long long)m * G.N;
    const Tri t = tri_of(G, ev[3 * n], ev[3 * n + 1], ev[3 * n + 2]);
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
    out[q] = acc + (t0 ? t0[n] : 0.0);
}

// Eq. (10): one wave per earthquake n, lanes over the fields m:
// K[n] = (sum_m R[n][m] dGamma_m/dx_a(x_n), a = 0..2, sum_m R[n][m]), the
// gradient being that of the trilinear interpolant in grid coordinates.  Lane
// partial sums in ascending m, then a fixed butterfly: deterministic.
template <int COORD>
__global__ void __launch_bounds__(64) k_reloc_kernel(Geo G, Tabs T, const Src* __restrict__ fsrc, int nfield,
                                                     const double* __restrict__ tau_all,
                                                     const double* __restrict__ ev, const double* __restrict__ R,
                                                     double* __restrict__ K) {
    const int n = blockIdx.x;
    const Tri t = tri_of(G, ev[3 * n], ev[3 * n + 1], ev[3 * n + 2]);
    long long ci[8];
    double dw[8][3];
    int q = 0;
    for (int c0 = 0; c0 < 2; ++c0)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int c2 = 0; c2 < 2; ++c2) {
                const int c[3] = {c0, c1, c2};
                ci[q] = nidx(G, t.b[0] + c0, t.b[1] + c1, t.b[2] + c2);
                for (int a = 0; a < 3; ++a) {
                    double v = (c[a] ? 1.0 : -1.0) * G.invh[a];
                    for (int e = 0; e < 3; ++e)
                        if (e != a) v *= c[e] ? t.f[e] : 1.0 - t.f[e];
                    dw[q][a] = v;
                }
                ++q;
            }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = threadIdx.x; m < nfield; m += 64) {
        const Src S = fsrc[m];
        const double* tau = tau_all + (long long)m * G.N;
        double gr[3] = {0.0, 0.0, 0.0};
        q = 0;
        for (int c0 = 0; c0 < 2; ++c0)
            for (int c1 = 0; c1 < 2; ++c1)
                for (int c2 = 0; c2 < 2; ++c2) {
                    const Col c = make_col(G, T, t.b[0] + c0, t.b[1] + c1);
                    const double2 t2 = T.t2[t.b[2] + c2];
                    double T0, tt[3];
                    factor<COORD>(S, c, t2.x, t2.y, T0, tt);
                    const double Gc = T0 * tau[ci[q]];
                    for (int a = 0; a < 3; ++a) gr[a] += dw[q][a] * Gc;
                    ++q;
                }
        const double r = R[(long long)n * nfield + m];
        for (int a = 0; a < 3; ++a) acc[a] += r * gr[a];
        acc[3] += r;
    }
    for (int a = 0; a < 4; ++a) acc[a] = wave_sum(acc[a]);
    if (threadIdx.x == 0)
        for (int a = 0; a < 4; ++a) K[(long long)n * 4 + a] = acc[a];
}

void launch_reloc_times(const Plan& P, const double* tau, int nev, const double* ev, const double* t0, double* out,
                        hipStream_t st) {
    const long long tot = (long long)P.nsrc * nev;
    if (tot == 0) return;
    if (P.G.coord == 1)
        hipLaunchKernelGGL(k_reloc_times<1>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, P.G, P.T, P.src, P.nsrc,
                           tau, nev, ev, t0, out);
    else
        hipLaunchKernelGGL(k_reloc_times<0>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, P.G, P.T, P.src, P.nsrc,
                           tau, nev, ev, t0, out);
}

void launch_reloc_kernel(const Plan& P, const double* tau, int nev, const double* ev, const double* R, double* K,
                         hipStream_t st) {
    if (nev == 0) return;
    if (P.G.coord == 1)
        hipLaunchKernelGGL(k_reloc_kernel<1>, dim3(nev), dim3(64), 0, st, P.G, P.T, P.src, P.nsrc, tau, ev, R, K);
    else
        hipLaunchKernelGGL(k_reloc_kernel<0>, dim3(nev), dim3(64), 0, st, P.G, P.T, P.src, P.nsrc, tau, ev, R, K);
}

void launch_misfit(int nsrc, int nrec, const double* T, const double* Tobs, const double* w, int npair,
                   const int32_t* pairs, const double* wpair, double alpha, double beta, double* R, double* chi,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_misfit, dim3(1), dim3(256), 0, st, nsrc, nrec, T, Tobs, w, npair, pairs, wpair, alpha, beta,
                       R, chi);
}

void launch_misfit_cr(int nsrc, int nrec, const double* T, const double* Tobs, const int32_t* off, const int32_t* pair,
                      const double* wcr, double gamma, double* R, double* chi, hipStream_t st) {
    hipLaunchKernelGGL(k_misfit_cr_R, dim3(nrec), dim3(64), 0, st, nsrc, nrec, T, Tobs, off, pair, wcr, gamma, R);
    hipLaunchKernelGGL(k_misfit_cr_chi, dim3(1), dim3(1024), 0, st, nsrc, nrec, T, Tobs, off, pair, wcr, gamma, chi);
}

// ------------------------------------------- multiple-grid parameterisation
// Coordinate of node i on axis a, rounded as o + i h is by definition (product,
// then sum; no fused multiply-add).  A tent ends abruptly at the first and last
// inversion node, so a node lying on such an end must land on the same side
// of it whoever evaluates the basis.
__device__ __forceinline__ double node_coord(const Geo& G, int a, int i) {
#pragma clang fp contract(off)
    return G.o[a] + (double)i * G.h[a];
}

// One-dimensional tent of inversion node i (ascending coordinates c[0..m-1])
// at x (Eqs. (12)-(14)); zero outside [c[0], c[m-1]].
__device__ __forceinline__ double mg_tent(const double* c, int m, int i, double x) {
    if (i > 0 && x >= c[i - 1] && x <= c[i]) return (x - c[i - 1]) / (c[i] - c[i - 1]);
    if (i < m - 1 && x >= c[i] && x <= c[i + 1]) return (c[i + 1] - x) / (c[i + 1] - c[i]);
    if (m == 1 && x == c[0]) return 1.0;
    return 0.0;
}

// Forward-grid index range [lo, hi] of axis a that can lie under the tent of
// inversion node i (one node of margin each side: the tent itself decides).
__device__ __forceinline__ void mg_range(const Geo& G, int a, const double* c, int m, int i, int& lo, int& hi) {
    const double x0 = c[i > 0 ? i - 1 : i], x1 = c[i < m - 1 ? i + 1 : i];
    lo = (int)floor((x0 - G.o[a]) / G.h[a]) - 1;
    hi = (int)ceil((x1 - G.o[a]) / G.h[a]) + 1;
    lo = lo < 0 ? 0 : lo;
    hi = hi > G.n[a] - 1 ? G.n[a] - 1 : hi;
}

// Eq. (17): one wave per inversion node (blockIdx.x = (ci m1 + cj) m2 + ck) of
// one grid; lanes share the node's support box in a fixed pattern and the
// partial sums are combined by a fixed shuffle tree (deterministic).
// out [3][m0][m1][m2] = sum_x K[p](x) B(x) V(x), B = u v w / H.
__global__ void __launch_bounds__(64) k_mg_project(Geo G, int H, int m0, int m1, int m2,
                                                   const double* __restrict__ c0, const double* __restrict__ c1,
                                                   const double* __restrict__ c2, const double* __restrict__ K,
                                                   double* __restrict__ out) {
    const long long M = (long long)m0 * m1 * m2;
    const long long l = blockIdx.x;
    const int ck = (int)(l % m2), cj = (int)((l / m2) % m1), ci = (int)(l / ((long long)m1 * m2));
    int ilo, ihi, jlo, jhi, klo, khi;
    mg_range(G, 0, c0, m0, ci, ilo, ihi);
    mg_range(G, 1, c1, m1, cj, jlo, jhi);
    mg_range(G, 2, c2, m2, ck, klo, khi);
    const int ni = ihi - ilo + 1, nj = jhi - jlo + 1, nk = khi - klo + 1;
    const long long box = (ni > 0 && nj > 0 && nk > 0) ? (long long)ni * nj * nk : 0;
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long e = threadIdx.x; e < box; e += 64) {
        const int k = klo + (int)(e % nk);
        const int j = jlo + (int)((e / nk) % nj);
        const int i = ilo + (int)(e / ((long long)nk * nj));
        const double u = mg_tent(c0, m0, ci, node_coord(G, 0, i));
        const double v = mg_tent(c1, m1, cj, node_coord(G, 1, j));
        const double w = mg_tent(c2, m2, ck, node_coord(G, 2, k));
        const double b = u * v * w / H * node_volume(G, i, j, k);
        if (b != 0.0) {
            const long long x = ((long long)i * G.n[1] + j) * G.n[2] + k;
            for (int p = 0; p < 3; ++p) acc[p] += K[p * G.N + x] * b;
        }
    }
    for (int p = 0; p < 3; ++p) acc[p] = wave_sum(acc[p]);
    if (threadIdx.x == 0)
        for (int p = 0; p < 3; ++p) out[p * M + l] = acc[p];
}

// Nonzero tents of one axis at x: at most two inversion nodes, in ascending
// node order.  With ascending coordinates only the last node at or below x and
// the one after it can be nonzero, so a binary search finds them.
__device__ __forceinline__ int mg_axis(const double* c, int m, double x, int idx[2], double wt[2]) {
    int lo = -1, hi = m;  // c[lo] <= x < c[hi], with c[-1] = -inf and c[m] = +inf
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] <= x) lo = mid;
        else hi = mid;
    }
    int cnt = 0;
    for (int i = lo; i <= lo + 1; ++i) {
        if (i < 0 || i >= m) continue;
        const double t = mg_tent(c, m, i, x);
        if (t != 0.0) {
            idx[cnt] = i;
            wt[cnt] = t;
            ++cnt;
        }
    }
    return cnt;
}

// Factor of the trapezoidal node volume along axis a (node_volume is the
// product of the three): h_a, times r^2 (radius) or cos(theta) (latitude) in
// spherical coordinates, halved on the two end nodes.
__device__ __forceinline__ double vol_axis(const Geo& G, int a, int i) {
    double v = G.h[a];
    if (G.coord == 1) {
        if (a == 0) {
            const double r = G.o[0] + i * G.h[0];
            v *= r * r;
        } else if (a == 1) {
            v *= cos(G.o[1] + i * G.h[1]);
        }
    }
    if (i == 0 || i == G.n[a] - 1) v *= 0.5;
    return v;
}

// The two nonzero tents of one axis at a forward node, weights pre-multiplied
// by that axis's volume factor (index -1: no tent).
struct MgTab {
    int i0, i1;
    double w0, w1;
};

__device__ __forceinline__ MgTab mg_tab(const double* c, int m, double x, double f) {
    int idx[2];
    double wt[2];
    const int n = mg_axis(c, m, x, idx, wt);
    MgTab t;
    t.i0 = n > 0 ? idx[0] : -1;
    t.w0 = n > 0 ? wt[0] * f : 0.0;
    t.i1 = n > 1 ? idx[1] : -1;
    t.w1 = n > 1 ? wt[1] * f : 0.0;
    return t;
}

__device__ __forceinline__ double mg_w(const MgTab& t, int c) { return t.i0 == c ? t.w0 : (t.i1 == c ? t.w1 : 0.0); }

// Separable projection (Eq. (17)): B and V both factor over the axes, so
//   d chi / d C[ci][cj][ck] = (1/H) sum_i W0[ci](i) sum_j W1[cj](j) sum_k W2[ck](k) K(i,j,k)
// with W_a = tent x volume factor.  Stage 1+2, one block per (plane i, row p of
// K, chunk of j): rows of the plane are staged in LDS, contracted over k for
// every (grid, ck) (stage 1), then accumulated over the chunk's j into
// partial[grid][cj][ck] (stage 2) in ascending j.  K is read once.  The
// inversion coordinates, the tent tables of axes 1 and 2 and the k range of
// every (grid, ck) are built in LDS first.
constexpr int kMgRows = 8;
// 8 waves per block share one copy of the tent tables in LDS
constexpr int kMgPlaneThreads = 512;

// k range and owner of one stage-1 output column
struct MgCol {
    int klo, khi, h, ck;
};

__device__ __forceinline__ int mg_grid_of(const int* off, int H, int e) {
    int h = 0;
    while (h + 1 < H && e >= off[h + 1]) ++h;
    return h;
}

__global__ void __launch_bounds__(kMgPlaneThreads) k_mg_proj_planes(Geo G, MgGrids Q, const double* __restrict__ coords,
                                                        const double* __restrict__ K, double* __restrict__ part,
                                                        int nch) {
    extern __shared__ double lds[];
    __shared__ MgGrids QL;  // per-grid sizes and offsets, indexed per lane below
    if (threadIdx.x == 0) QL = Q;
    const int H = Q.H, n1 = G.n[1], n2 = G.n[2];
    const int S2 = Q.s2off[H], S12 = Q.s12off[H];
    double* cl = lds;
    MgTab* tab1 = reinterpret_cast<MgTab*>(cl + Q.ncoord);
    MgTab* tab2 = tab1 + H * n1;
    MgCol* cols = reinterpret_cast<MgCol*>(tab2 + H * n2);
    int* off12 = reinterpret_cast<int*>(cols + S2);
    double* rows = reinterpret_cast<double*>(off12 + 2 * (TT_MG_MAX_GRIDS + 1));
    double* A = rows + kMgRows * n2;
    double* acc = A + kMgRows * S2;
    const int ch = blockIdx.x % nch, p = (blockIdx.x / nch) % 3, i = blockIdx.x / (3 * nch);
    for (int e = threadIdx.x; e < Q.ncoord; e += blockDim.x) cl[e] = coords[e];
    for (int e = threadIdx.x; e <= H; e += blockDim.x) off12[e] = Q.s12off[e];
    __syncthreads();  // QL, cl, off12
    for (int e = threadIdx.x; e < H * n1; e += blockDim.x) {
        const int h = e / n1, j = e % n1;
        tab1[e] = mg_tab(cl + QL.coff[h][1], QL.m[h][1], node_coord(G, 1, j), vol_axis(G, 1, j));
    }
    for (int e = threadIdx.x; e < H * n2; e += blockDim.x) {
        const int h = e / n2, k = e % n2;
        tab2[e] = mg_tab(cl + QL.coff[h][2], QL.m[h][2], node_coord(G, 2, k), vol_axis(G, 2, k));
    }
    for (int q = threadIdx.x; q < S2; q += blockDim.x) {
        MgCol c;
        c.h = 0;
        while (c.h + 1 < H && q >= QL.s2off[c.h + 1]) ++c.h;
        c.ck = q - QL.s2off[c.h];
        mg_range(G, 2, cl + QL.coff[c.h][2], QL.m[c.h][2], c.ck, c.klo, c.khi);
        cols[q] = c;
    }
    for (int e = threadIdx.x; e < S12; e += blockDim.x) acc[e] = 0.0;
    __syncthreads();
    const int j0 = (int)((long long)ch * n1 / nch), j1 = (int)((long long)(ch + 1) * n1 / nch);
    const double* Kp = K + (long long)p * G.N + (long long)i * n1 * n2;
    for (int jb = j0; jb < j1; jb += kMgRows) {
        const int nr = min(kMgRows, j1 - jb);
        for (int e = threadIdx.x; e < nr * n2; e += blockDim.x) rows[e] = Kp[(long long)jb * n2 + e];
        __syncthreads();
        for (int e = threadIdx.x; e < nr * S2; e += blockDim.x) {
            const int r = e / S2, q = e % S2;
            const MgCol c = cols[q];
            const MgTab* t2 = tab2 + c.h * n2;
            const double* row = rows + r * n2;
            double a = 0.0;
            for (int k = c.klo; k <= c.khi; ++k) a += mg_w(t2[k], c.ck) * row[k];
            A[r * S2 + q] = a;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < S12; e += blockDim.x) {
            const int h = mg_grid_of(off12, H, e);
            const int m2 = QL.m[h][2], q = e - off12[h];
            const int cj = q / m2, ck = q % m2;
            const MgTab* t1 = tab1 + h * n1 + jb;
            const double* Ac = A + QL.s2off[h] + ck;
            double v = acc[e];
            for (int r = 0; r < nr; ++r) {
                const double w = mg_w(t1[r], cj);
                if (w != 0.0) v += w * Ac[r * S2];
            }
            acc[e] = v;
        }
        __syncthreads();
    }
    double* out = part + ((long long)(i * 3 + p) * nch + ch) * S12;
    for (int e = threadIdx.x; e < S12; e += blockDim.x) out[e] = acc[e];
}

// Stage 3: kMgFinalLanes lanes per coefficient, contraction over the planes i
// under its tent (lane l takes the planes ilo + l, ilo + l + kMgFinalLanes, ...
// in ascending order, j-chunks summed in order), a fixed xor-shuffle tree over
// the lanes, then the 1/H of Eq. (11).  The grid sizes and (CLDS) the
// inversion coordinates are staged in LDS.
constexpr int kMgFinalLanes = 8;

template <bool CLDS>
__global__ void __launch_bounds__(256) k_mg_proj_final(Geo G, MgGrids Q, const double* __restrict__ coords,
                                                       const double* __restrict__ part, int nch,
                                                       double* __restrict__ out) {
    extern __shared__ double lds[];
    __shared__ MgGrids QL;
    if (threadIdx.x == 0) QL = Q;
    if (CLDS)
        for (int e = threadIdx.x; e < Q.ncoord; e += blockDim.x) lds[e] = coords[e];
    __syncthreads();
    const double* cb = CLDS ? lds : coords;
    const long long total = Q.outoff[Q.H];
    const int S12 = Q.s12off[Q.H];
    const int sub = (int)(threadIdx.x % kMgFinalLanes);
    // the lanes of one coefficient share e, so they leave the loop together
    for (long long e = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kMgFinalLanes; e < total;
         e += (long long)gridDim.x * blockDim.x / kMgFinalLanes) {
        int h = 0;
        while (h + 1 < Q.H && e >= QL.outoff[h + 1]) ++h;
        const int m0 = QL.m[h][0], m1 = QL.m[h][1], m2 = QL.m[h][2];
        const long long M = (long long)m0 * m1 * m2, q = e - QL.outoff[h];
        const int p = (int)(q / M);
        const long long l = q % M;
        const int ck = (int)(l % m2), cj = (int)((l / m2) % m1), ci = (int)(l / ((long long)m1 * m2));
        const double* c0 = cb + QL.coff[h][0];
        int ilo, ihi;
        mg_range(G, 0, c0, m0, ci, ilo, ihi);
        const long long col = QL.s12off[h] + (long long)cj * m2 + ck;
        double a = 0.0;
        for (int i = ilo + sub; i <= ihi; i += kMgFinalLanes) {
            const double u = mg_tent(c0, m0, ci, node_coord(G, 0, i));
            if (u == 0.0) continue;
            const double* pi = part + (long long)(i * 3 + p) * nch * S12 + col;
            double b = 0.0;
            for (int c = 0; c < nch; ++c) b += pi[(long long)c * S12];
            a += u * vol_axis(G, 0, i) * b;
        }
#pragma unroll
        for (int off = kMgFinalLanes / 2; off >= 1; off >>= 1) a += __shfl_xor(a, off, kMgFinalLanes);
        if (sub == 0) out[e] = a / Q.H;
    }
}

// Eq. (15), staged form: one block per (plane i, chunk of j).  With at most two
// nonzero tents per axis and grid, the block first contracts the coefficients
// over axis 0 at its plane, E[p][grid][cj][ck] = sum_ci u_ci(i) C[grid][p][ci][cj][ck],
// in LDS, then each thread forms field(i, j, k) from at most 4 terms of E per
// grid (tables of the axis-1 and axis-2 tents in LDS), summed over the grids in
// order and written once.
__global__ void __launch_bounds__(kMgPlaneThreads) k_mg_expand_planes(Geo G, MgGrids Q, const double* __restrict__ coords,
                                                          const double* __restrict__ C, double* __restrict__ field,
                                                          int nch) {
    extern __shared__ double lds[];
    __shared__ MgGrids QL;
    __shared__ MgTab tab0[TT_MG_MAX_GRIDS];
    if (threadIdx.x == 0) QL = Q;
    const int H = Q.H, n1 = G.n[1], n2 = G.n[2];
    const int S12 = Q.s12off[H];
    double* cl = lds;
    MgTab* tab1 = reinterpret_cast<MgTab*>(cl + Q.ncoord);
    MgTab* tab2 = tab1 + H * n1;
    double* E = reinterpret_cast<double*>(tab2 + H * n2);
    const int ch = blockIdx.x % nch, i = blockIdx.x / nch;
    for (int e = threadIdx.x; e < Q.ncoord; e += blockDim.x) cl[e] = coords[e];
    __syncthreads();  // QL, cl
    for (int h = threadIdx.x; h < H; h += blockDim.x)
        tab0[h] = mg_tab(cl + QL.coff[h][0], QL.m[h][0], node_coord(G, 0, i), 1.0);
    for (int e = threadIdx.x; e < H * n1; e += blockDim.x) {
        const int h = e / n1, j = e % n1;
        tab1[e] = mg_tab(cl + QL.coff[h][1], QL.m[h][1], node_coord(G, 1, j), 1.0);
    }
    for (int e = threadIdx.x; e < H * n2; e += blockDim.x) {
        const int h = e / n2, k = e % n2;
        tab2[e] = mg_tab(cl + QL.coff[h][2], QL.m[h][2], node_coord(G, 2, k), 1.0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * S12; e += blockDim.x) {
        const int p = e / S12, q = e % S12;
        int h = 0;
        while (h + 1 < H && q >= QL.s12off[h + 1]) ++h;
        const long long M12 = (long long)QL.m[h][1] * QL.m[h][2];
        const double* Cp = C + QL.outoff[h] + (long long)p * QL.m[h][0] * M12 + (q - QL.s12off[h]);
        const MgTab t = tab0[h];
        double v = 0.0;
        if (t.i0 >= 0) v += t.w0 * Cp[(long long)t.i0 * M12];
        if (t.i1 >= 0) v += t.w1 * Cp[(long long)t.i1 * M12];
        E[e] = v;
    }
    __syncthreads();
    const int j0 = (int)((long long)ch * n1 / nch), j1 = (int)((long long)(ch + 1) * n1 / nch);
    const long long base = (long long)i * n1 * n2;
    for (int e = threadIdx.x; e < (j1 - j0) * n2; e += blockDim.x) {
        const int j = j0 + e / n2, k = e % n2;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int h = 0; h < H; ++h) {
            const MgTab t1 = tab1[h * n1 + j], t2 = tab2[h * n2 + k];
            const int m2 = QL.m[h][2], o12 = QL.s12off[h];
            const int cj[2] = {t1.i0, t1.i1}, ck[2] = {t2.i0, t2.i1};
            const double wj[2] = {t1.w0, t1.w1}, wk[2] = {t2.w0, t2.w1};
            for (int a = 0; a < 2; ++a) {
                if (cj[a] < 0) continue;
                for (int b = 0; b < 2; ++b) {
                    if (ck[b] < 0) continue;
                    const double bw = wj[a] * wk[b] / H;
                    const int q = o12 + cj[a] * m2 + ck[b];
                    for (int p = 0; p < 3; ++p) acc[p] += E[p * S12 + q] * bw;
                }
            }
        }
        const long long x = base + (long long)j * n2 + k;
        for (int p = 0; p < 3; ++p) field[p * G.N + x] = acc[p];
    }
}

// Eq. (15) for grids whose staging does not fit in LDS: one thread per forward
// node; field[p](x) = sum over the grids of C B over the (at most 8 per grid)
// nonzero basis functions, accumulated in grid order and written once.
__global__ void __launch_bounds__(256) k_mg_expand(Geo G, MgGrids Q, const double* __restrict__ coords,
                                                   const double* __restrict__ C, double* __restrict__ field) {
    __shared__ MgGrids QL;
    if (threadIdx.x == 0) QL = Q;
    __syncthreads();
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < G.N;
         x += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(x % G.n[2]);
        const long long q = x / G.n[2];
        const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
        const double xi = node_coord(G, 0, i), xj = node_coord(G, 1, j), xk = node_coord(G, 2, k);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int h = 0; h < QL.H; ++h) {
            const int m1 = QL.m[h][1], m2 = QL.m[h][2];
            const long long M = (long long)QL.m[h][0] * m1 * m2;
            int ii[2], jj[2], kk[2];
            double wi[2], wj[2], wk[2];
            const int na = mg_axis(coords + QL.coff[h][0], QL.m[h][0], xi, ii, wi);
            const int nb = mg_axis(coords + QL.coff[h][1], m1, xj, jj, wj);
            const int nc = mg_axis(coords + QL.coff[h][2], m2, xk, kk, wk);
            const double* Ch = C + QL.outoff[h];
            for (int a = 0; a < na; ++a)
                for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c) {
                        const long long l = ((long long)ii[a] * m1 + jj[b]) * m2 + kk[c];
                        const double bw = wi[a] * wj[b] * wk[c] / QL.H;
                        for (int p = 0; p < 3; ++p) acc[p] += Ch[p * M + l] * bw;
                    }
        }
        for (int p = 0; p < 3; ++p) field[p * G.N + x] = acc[p];
    }
}

// Kernel-density normalisation (Eqs. (18)-(19)), one thread per node:
// Kd = dens / (s V), K = (s grad_s, grad_xi, grad_eta) / V / (Kd + eps)^zeta with
// V the trapezoidal node volume.
__global__ void k_kernel_density(Geo G, const double* __restrict__ s, const double* __restrict__ dens,
                                 const double* __restrict__ grad, double eps, double zeta, double* __restrict__ K,
                                 double* __restrict__ Kd) {
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < G.N;
         x += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(x % G.n[2]);
        const long long q = x / G.n[2];
        const int j = (int)(q % G.n[1]), i = (int)(q / G.n[1]);
        const double v = node_volume(G, i, j, k);
        const double d = dens[x] / (s[x] * v);
        const double w = pow(d + eps, zeta);
        if (Kd) Kd[x] = d;
        K[x] = s[x] * grad[x] / v / w;
        K[G.N + x] = grad[G.N + x] / v / w;
        K[2 * G.N + x] = grad[2 * G.N + x] / v / w;
    }
}

void launch_kernel_density(const Geo& G, const double* s, const double* dens, const double* grad, double eps,
                           double zeta, double* K, double* Kd, hipStream_t st) {
    hipLaunchKernelGGL(k_kernel_density, dim3(fill_blocks(G.N)), dim3(256), 0, st, G, s, dens, grad, eps, zeta, K,
                       Kd);
}

MgGrids make_mg(int H, const int* m) {
    MgGrids Q{};
    Q.H = H;
    int c = 0;
    for (int h = 0; h < H; ++h) {
        for (int a = 0; a < 3; ++a) {
            Q.m[h][a] = m[3 * h + a];
            Q.coff[h][a] = c;
            c += m[3 * h + a];
        }
        Q.s2off[h + 1] = Q.s2off[h] + m[3 * h + 2];
        Q.s12off[h + 1] = Q.s12off[h] + m[3 * h + 1] * m[3 * h + 2];
        Q.outoff[h + 1] = Q.outoff[h] + 3LL * m[3 * h] * m[3 * h + 1] * m[3 * h + 2];
    }
    Q.ncoord = c;
    return Q;
}

MgPlan plan_mg_project(const Geo& G, const MgGrids& Q) {
    MgPlan P{};
    const long long H = Q.H, S2 = Q.s2off[Q.H], S12 = Q.s12off[Q.H];
    const long long lds = 8LL * Q.ncoord + (long long)sizeof(MgTab) * H * (G.n[1] + G.n[2]) +
                          (long long)sizeof(MgCol) * S2 + 8LL * (TT_MG_MAX_GRIDS + 1) +
                          8LL * (kMgRows * (long long)G.n[2] + kMgRows * S2 + S12);
    P.lds = (size_t)lds;
    P.separable = lds <= kMgMaxLds;
    if (P.separable) {
        // split each plane's rows into chunks for about 512 blocks: every block
        // rebuilds the tent tables, so more chunks cost more than the parallelism
        // they add (101^3, five 11 x 13 x 13 grids: 0.159 ms at 2 chunks per plane,
        // 0.182 ms at 4, 0.218 ms at 8)
        P.nch = (int)std::min<long long>(std::max<long long>((512 + 3LL * G.n[0] - 1) / (3LL * G.n[0]), 1),
                                         std::min(8, G.n[1]));
        P.ws_bytes = 8ULL * G.n[0] * 3ULL * P.nch * (unsigned long long)S12;
    }
    return P;
}

void launch_mg_project(const Geo& G, int H, const int* m, const double* coords, const double* K, double* out,
                       double* ws, hipStream_t st) {
    const MgGrids Q = make_mg(H, m);
    const MgPlan P = plan_mg_project(G, Q);
    if (P.separable) {
        hipLaunchKernelGGL(k_mg_proj_planes, dim3((unsigned)(G.n[0] * 3 * P.nch)), dim3(kMgPlaneThreads), P.lds, st, G, Q,
                           coords, K, ws, P.nch);
        const dim3 fb(fill_blocks(Q.outoff[H] * kMgFinalLanes));
        if (8LL * Q.ncoord <= kMgCoordLds)
            hipLaunchKernelGGL(k_mg_proj_final<true>, fb, dim3(256), 8 * Q.ncoord, st, G, Q, coords, ws, P.nch, out);
        else
            hipLaunchKernelGGL(k_mg_proj_final<false>, fb, dim3(256), 0, st, G, Q, coords, ws, P.nch, out);
        return;
    }
    // grids too large for the staged form: one wave per inversion node
    const double* cg = coords;
    double* og = out;
    for (int q = 0; q < H; ++q) {
        const int* mq = m + 3 * q;
        const long long M = (long long)mq[0] * mq[1] * mq[2];
        hipLaunchKernelGGL(k_mg_project, dim3((unsigned)M), dim3(64), 0, st, G, H, mq[0], mq[1], mq[2], cg,
                           cg + mq[0], cg + mq[0] + mq[1], K, og);
        cg += mq[0] + mq[1] + mq[2];
        og += 3 * M;
    }
}

void launch_mg_expand(const Geo& G, int H, const int* m, const double* coords, const double* C, double* field,
                      hipStream_t st) {
    const MgGrids Q = make_mg(H, m);
    const long long lds = 8LL * Q.ncoord + (long long)sizeof(MgTab) * H * (G.n[1] + G.n[2]) + 8LL * 3 * Q.s12off[H];
    if (lds <= kMgMaxLds) {
        // about 512 blocks of 8 waves (three fit a CU's LDS)
        const int nch = (int)std::min<long long>(std::max<long long>((512 + G.n[0] - 1) / G.n[0], 1), G.n[1]);
        hipLaunchKernelGGL(k_mg_expand_planes, dim3((unsigned)(G.n[0] * nch)), dim3(kMgPlaneThreads), (size_t)lds, st,
                           G, Q, coords, C, field, nch);
        return;
    }
    hipLaunchKernelGGL(k_mg_expand, dim3(fill_blocks(G.N)), dim3(256), 0, st, G, Q, coords, C, field);
}

}  // namespace tt

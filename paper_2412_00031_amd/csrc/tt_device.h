// tt_device.h -- device helpers shared by the solver kernels (tt_kernels.hip)
// and the per-step kernels outside the solves (tt_aux.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "tt_internal.h"

namespace tt {

__device__ __forceinline__ int cell_base(const Geo& G, int a, double x) {
    double u = (x - G.o[a]) / G.h[a];
    double fl = floor(u);
    if (fl < 0.0) return 0;
    if (fl > (double)(G.n[a] - 2)) return G.n[a] - 2;
    return (int)fl;
}

__device__ __forceinline__ long long nidx(const Geo& G, int i, int j, int k) {
    return (long long)i * G.si + (long long)j * G.sj + k;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// fixed-order sum over a 256-thread block (result valid in thread 0)
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

struct Tri {
    int b[3];
    double f[3];
};

__device__ __forceinline__ Tri tri_of(const Geo& G, double p0, double p1, double p2) {
    Tri t;
    const double p[3] = {p0, p1, p2};
    for (int a = 0; a < 3; ++a) {
        t.b[a] = cell_base(G, a, p[a]);
        const double f = (p[a] - G.o[a]) / G.h[a] - (double)t.b[a];
        t.f[a] = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    }
    return t;
}

__device__ __forceinline__ double tri_w(const Tri& t, int c0, int c1, int c2) {
    return (c0 ? t.f[0] : 1.0 - t.f[0]) * (c1 ? t.f[1] : 1.0 - t.f[1]) * (c2 ? t.f[2] : 1.0 - t.f[2]);
}

// Trapezoidal node volume (r^2 cos(theta) dr dtheta dphi in spherical
// coordinates, halved once per boundary axis).
__device__ __forceinline__ double node_volume(const Geo& G, int i, int j, int k) {
    double v = G.h[0] * G.h[1] * G.h[2];
    if (G.coord == 1) {
        const double r = G.o[0] + i * G.h[0];
        v *= r * r * cos(G.o[1] + j * G.h[1]);
    }
    if (i == 0 || i == G.n[0] - 1) v *= 0.5;
    if (j == 0 || j == G.n[1] - 1) v *= 0.5;
    if (k == 0 || k == G.n[2] - 1) v *= 0.5;
    return v;
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// grid-stride launches: enough blocks to fill the chip, at most 2048
inline unsigned fill_blocks(long long n) {
    unsigned nb = blocks_for(n, 256);
    return nb > 2048 ? 2048 : (nb == 0 ? 1 : nb);
}

}  // namespace tt

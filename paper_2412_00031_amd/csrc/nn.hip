// nn.hip -- kernels and C ABI (include/nn.h) of the warm-start 3-D U-Net.
//
// The network predicts the factor tau of T = T0 * tau (multiplicative
// factorisation, Sec. 3.1) from the model so that the sweeps of Eq. (4) start
// near their fixed point.  3^3 convolutions run on the matrix cores
// (v_mfma_f32_16x16x16_bf16: bf16 operands, fp32 accumulation) as implicit
// GEMMs over channels-last activations; pooling, transposed up-sampling, the
// 1x1 head, the loss and Adam are plain vector kernels.  Every reduction runs
// in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "nn.h"
#include "tt_internal.h"

namespace {

using tt::fail;

#define NN_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(TT_EHIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

#define NN_LAUNCHED() NN_HIP(hipGetLastError())

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kMB = 4;  // 16-position blocks of one wave in the convolution

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

unsigned blocks_of(long long n, int per) { return (unsigned)((n + per - 1) / per); }

hipStream_t S(void* st) { return reinterpret_cast<hipStream_t>(st); }

// ------------------------------------------------------------------ casts
__global__ void k_to_bf16(const float* __restrict__ x, long long n, uint16_t* __restrict__ y) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

__global__ void k_from_bf16(const uint16_t* __restrict__ x, long long n, float* __restrict__ y) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = bf2f(x[i]);
}

unsigned grid_stride_blocks(long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

// ------------------------------------------------------- weight fragments
// Operand-B fragment of the 16x16x16 bf16 MFMA: lane l holds B[4(l/16)+v][l%16],
// v = 0..3.  The packed index is (((t*KB + kb)*NB + nb)*64 + lane)*4 + v.
// flip = 0: B[k][n] = W[t][kb*16+k][nb*16+n] (rows >= cin are zero).
// flip = 1: data-gradient weights W'[t][o][i] = W[26-t][i][o].
__global__ void k_conv3_pack(const float* __restrict__ W, int cin, int cout, int KB, int NB, int flip,
                             uint16_t* __restrict__ frag) {
    const long long total = 27LL * KB * NB * 256;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int v = (int)(idx & 3), lane = (int)((idx >> 2) & 63);
        long long rest = idx >> 8;
        const int nb = (int)(rest % NB);
        rest /= NB;
        const int kb = (int)(rest % KB);
        const int t = (int)(rest / KB);
        const int kr = kb * 16 + 4 * (lane >> 4) + v;
        const int nc = nb * 16 + (lane & 15);
        float w;
        if (!flip)
            w = kr < cin ? W[((long long)t * cin + kr) * cout + nc] : 0.0f;
        else
            w = W[((long long)(26 - t) * cin + nc) * cout + kr];
        frag[idx] = f2bf(w);
    }
}

// ---------------------------------------------------------- conv forward
// One wave computes 64 consecutive positions (4 blocks of 16) x all NB*16
// output channels; K runs over 27 taps x cin.  Operand A (lane l: position
// p0 + 16 mb + l%16, channels 4(l/16)..+3 of the k-block) is one 8-byte load
// from the channels-last input; out-of-range neighbours read a clamped
// address and are zeroed.  Result layout: lane l holds rows 4(l/16)+r, col l%16.
template <int NB>
__global__ __launch_bounds__(256) void k_conv3_fwd(const uint16_t* __restrict__ x, int D, int H, int W,
                                                   long long npos, int cxt, int cxo, int KB,
                                                   const uint16_t* __restrict__ frag,
                                                   const float* __restrict__ bias, int relu,
                                                   uint16_t* __restrict__ y, int cyt, int cyo) {
    const int lane = threadIdx.x & 63;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long p0 = wave * (16 * kMB);
    if (p0 >= npos) return;
    const int li = lane & 15, g = lane >> 4;
    int pz[kMB], py[kMB], px[kMB];
    long long pc[kMB];
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) {
        long long p = p0 + 16 * mb + li;
        if (p >= npos) p = npos - 1;
        pc[mb] = p;
        px[mb] = (int)(p % W);
        long long q = p / W;
        py[mb] = (int)(q % H);
        pz[mb] = (int)((q / H) % D);
    }
    f4_t acc[kMB][NB];
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4_t{0.f, 0.f, 0.f, 0.f};
    const s4_t* fr = reinterpret_cast<const s4_t*>(frag) + lane;
    const uint16_t* xb = x + cxo + 4 * g;
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const long long off = ((long long)dz * H + dy) * W + dx;
        const uint16_t* xa[kMB];
        short msk[kMB];
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb) {
            const bool ok = (unsigned)(pz[mb] + dz) < (unsigned)D && (unsigned)(py[mb] + dy) < (unsigned)H &&
                            (unsigned)(px[mb] + dx) < (unsigned)W;
            msk[mb] = ok ? (short)-1 : (short)0;
            xa[mb] = xb + (ok ? pc[mb] + off : pc[mb]) * cxt;
        }
        for (int kb = 0; kb < KB; ++kb) {
            s4_t a[kMB], b[NB];
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb) a[mb] = *reinterpret_cast<const s4_t*>(xa[mb] + kb * 16) & msk[mb];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = fr[((t * KB + kb) * NB + nb) * 64];
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long p = p0 + 16 * mb + 4 * g + r;
            if (p >= npos) continue;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                float v = acc[mb][nb][r] + (bias ? bias[nb * 16 + li] : 0.0f);
                if (relu) v = fmaxf(v, 0.0f);
                y[p * cyt + cyo + nb * 16 + li] = f2bf(v);
            }
        }
}

// --------------------------------------------------------- conv wgrad
// Partial sums of gW[t][i][o] = sum_p x[p + d_t][i] gz[p][o] over the rows
// (n, z, y) of one slice, on the matrix cores with K = positions: A[i][k] =
// x[p_k + d_t][i], B[k][o] = gz[p_k][o], 16 positions of one row per step.
// Block = 4 waves over interleaved rows, combined in wave order through LDS.
// part layout [slice][27][cin][cout].
__global__ __launch_bounds__(256) void k_conv3_wgrad(const uint16_t* __restrict__ x, int D, int H, int W,
                                                     long long nrows, int cxt, int cxo, int cin,
                                                     const uint16_t* __restrict__ gz, int cgt, int cgo,
                                                     int cout, long long rows_per_slice,
                                                     float* __restrict__ part) {
    __shared__ f4_t red[3][16][64];
    const int t = blockIdx.y;
    const long long slice = blockIdx.x;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int IB = (cin + 15) / 16, OB = cout / 16;
    f4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};
    const long long r0 = slice * rows_per_slice;
    const long long r1 = r0 + rows_per_slice < nrows ? r0 + rows_per_slice : nrows;
    int chA[4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
        const int c = ib * 16 + li;
        chA[ib] = c < cin ? c : cin - 1;
    }
    for (long long r = r0 + wv; r < r1; r += 4) {
        const int yy = (int)(r % H);
        const int zz = (int)((r / H) % D);
        if ((unsigned)(zz + dz) >= (unsigned)D || (unsigned)(yy + dy) >= (unsigned)H) continue;
        const long long rowp = r * W;
        const long long nrowp = rowp + ((long long)dz * H + dy) * W;
        for (int x0 = 0; x0 < W; x0 += 16) {
            s4_t a[4], b[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int xk = x0 + 4 * g + v;
                const bool okb = xk < W;
                const bool oka = okb && (unsigned)(xk + dx) < (unsigned)W;
                const long long pa = oka ? nrowp + xk + dx : rowp;
                const long long pb = okb ? rowp + xk : rowp;
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) {
                    if (ib < IB) {
                        const uint16_t va = x[pa * cxt + cxo + chA[ib]];
                        a[ib][v] = (oka && ib * 16 + li < cin) ? (short)va : (short)0;
                    }
                }
#pragma unroll
                for (int ob = 0; ob < 4; ++ob) {
                    if (ob < OB) {
                        const uint16_t vb = gz[pb * cgt + cgo + ob * 16 + li];
                        b[ob][v] = okb ? (short)vb : (short)0;
                    }
                }
            }
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int ob = 0; ob < 4; ++ob)
                    if (ib < IB && ob < OB)
                        acc[ib][ob] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[ib], b[ob], acc[ib][ob], 0, 0, 0);
        }
    }
    if (wv > 0) {
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) red[wv - 1][ib * 4 + ob][lane] = acc[ib][ob];
    }
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            if (ib >= IB || ob >= OB) continue;
            f4_t s = acc[ib][ob];
            for (int w = 0; w < 3; ++w) s += red[w][ib * 4 + ob][lane];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ib * 16 + 4 * g + r;
                if (i < cin)
                    part[((slice * 27 + t) * cin + i) * cout + ob * 16 + li] = s[r];
            }
        }
}

// out[j] = sum over slices (in order) of part[slice][j]
__global__ void k_sum_slices(const float* __restrict__ part, long long nslices, long long n, float* __restrict__ out) {
    for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (long long q = 0; q < nslices; ++q) s += part[q * n + j];
        out[j] = s;
    }
}

// Column sums of a bf16 [npos][ct] block (channels [co, co + c), c <= 64):
// part[block][ch], 4 lane groups per block combined in order.
__global__ __launch_bounds__(256) void k_colsum_part(const uint16_t* __restrict__ g, long long npos, int ct, int co,
                                                     int c, long long chunk, float* __restrict__ part) {
    __shared__ float red[4][64];
    const int ch = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const long long p0 = blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npos ? p0 + chunk : npos;
    float s = 0.0f;
    if (ch < c)
        for (long long p = p0 + grp; p < p1; p += 4) s += bf2f(g[p * ct + co + ch]);
    red[grp][ch] = s;
    __syncthreads();
    if (grp == 0 && ch < c) part[blockIdx.x * (long long)c + ch] = red[0][ch] + red[1][ch] + red[2][ch] + red[3][ch];
}

// ------------------------------------------------------------- relu mask
__global__ void k_relu_mask(const uint16_t* __restrict__ g, const uint16_t* __restrict__ y, long long npos, int ct,
                            int co, int c, uint16_t* __restrict__ go, int cot, int coo) {
    const long long n = npos * c;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long p = e / c;
        const int ch = (int)(e - p * c);
        const uint16_t yv = y[p * ct + co + ch];
        const bool pos = (yv & 0x8000u) == 0 && (yv & 0x7fffu) != 0;  // y > 0
        go[p * cot + coo + ch] = pos ? g[p * ct + co + ch] : (uint16_t)0;
    }
}

// ---------------------------------------------------------------- pooling
__device__ __forceinline__ long long child_pos(long long q, int Dh, int Hh, int Wh, int s) {
    // q indexes the pooled grid [n][Dh][Hh][Wh]; child s = a*4 + b*2 + c
    const int X = (int)(q % Wh);
    long long r = q / Wh;
    const int Y = (int)(r % Hh);
    r /= Hh;
    const int Z = (int)(r % Dh);
    const long long n = r / Dh;
    const int a = s >> 2, b = (s >> 1) & 1, c = s & 1;
    return ((n * (2 * Dh) + 2 * Z + a) * (2 * Hh) + 2 * Y + b) * (long long)(2 * Wh) + 2 * X + c;
}

__global__ void k_pool_fwd(const uint16_t* __restrict__ x, long long nq, int Dh, int Hh, int Wh, int ct, int co, int c,
                           uint16_t* __restrict__ y) {
    const long long n = nq * c;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long q = e / c;
        const int ch = (int)(e - q * c);
        uint16_t best = x[child_pos(q, Dh, Hh, Wh, 0) * ct + co + ch];
        float bv = bf2f(best);
        for (int s = 1; s < 8; ++s) {
            const uint16_t v = x[child_pos(q, Dh, Hh, Wh, s) * ct + co + ch];
            if (bf2f(v) > bv) {
                bv = bf2f(v);
                best = v;
            }
        }
        y[q * c + ch] = best;
    }
}

__global__ void k_pool_bwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ gy, long long nq, int Dh,
                           int Hh, int Wh, int ct, int co, int c, uint16_t* __restrict__ gx, int accumulate) {
    const long long n = nq * c;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long q = e / c;
        const int ch = (int)(e - q * c);
        int arg = 0;
        float bv = bf2f(x[child_pos(q, Dh, Hh, Wh, 0) * ct + co + ch]);
        for (int s = 1; s < 8; ++s) {
            const float v = bf2f(x[child_pos(q, Dh, Hh, Wh, s) * ct + co + ch]);
            if (v > bv) {
                bv = v;
                arg = s;
            }
        }
        const float gv = bf2f(gy[q * c + ch]);
        for (int s = 0; s < 8; ++s) {
            const long long idx = child_pos(q, Dh, Hh, Wh, s) * ct + co + ch;
            const float base = accumulate ? bf2f(gx[idx]) : 0.0f;
            gx[idx] = f2bf(s == arg ? base + gv : base);
        }
    }
}

// ------------------------------------------------- transposed up-sampling
__global__ void k_up_fwd(const uint16_t* __restrict__ x, long long nout, int D, int H, int W, int cin,
                         const float* __restrict__ Wu, const float* __restrict__ b, int cout,
                         uint16_t* __restrict__ y, int cyt, int cyo) {
    const long long n = nout * cout;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long q = e / cout;
        const int o = (int)(e - q * cout);
        const int X = (int)(q % (2 * W));
        long long r = q / (2 * W);
        const int Y = (int)(r % (2 * H));
        r /= 2 * H;
        const int Z = (int)(r % (2 * D));
        const long long nb = r / (2 * D);
        const long long p = ((nb * D + (Z >> 1)) * H + (Y >> 1)) * W + (X >> 1);
        const int s = (Z & 1) * 4 + (Y & 1) * 2 + (X & 1);
        float acc = b[o];
        const uint16_t* xp = x + p * cin;
        const float* wp = Wu + (long long)s * cin * cout + o;
        for (int i = 0; i < cin; ++i) acc += bf2f(xp[i]) * wp[(long long)i * cout];
        y[q * cyt + cyo + o] = f2bf(acc);
    }
}

// gx[p][i] = sum_s sum_o gy[child s of p][o] Wu[s][i][o]
__global__ void k_up_bwd_data(const uint16_t* __restrict__ gy, long long np, int D, int H, int W, int cin, int cout,
                              int cgt, int cgo, const float* __restrict__ Wu, uint16_t* __restrict__ gx) {
    const long long n = np * cin;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long p = e / cin;
        const int i = (int)(e - p * cin);
        float acc = 0.0f;
        for (int s = 0; s < 8; ++s) {
            const long long q = child_pos(p, D, H, W, s);
            const uint16_t* gp = gy + q * cgt + cgo;
            const float* wp = Wu + ((long long)s * cin + i) * cout;
            for (int o = 0; o < cout; ++o) acc += bf2f(gp[o]) * wp[o];
        }
        gx[p * cin + i] = f2bf(acc);
    }
}

// part[slice][s][i][o] = sum over the slice's coarse positions p of x[p][i] gy[child s of p][o]
__global__ __launch_bounds__(256) void k_up_wgrad_part(const uint16_t* __restrict__ x, const uint16_t* __restrict__ gy,
                                                       long long np, int D, int H, int W, int cin, int cout, int cgt,
                                                       int cgo, long long chunk, float* __restrict__ part) {
    const int s = blockIdx.y;
    const long long slice = blockIdx.x;
    const long long p0 = slice * chunk;
    const long long p1 = p0 + chunk < np ? p0 + chunk : np;
    const int npair = cin * cout;
    for (int pr = threadIdx.x; pr < npair; pr += blockDim.x) {
        const int i = pr / cout, o = pr - (pr / cout) * cout;
        float acc = 0.0f;
        for (long long p = p0; p < p1; ++p)
            acc += bf2f(x[p * cin + i]) * bf2f(gy[child_pos(p, D, H, W, s) * cgt + cgo + o]);
        part[((slice * 8 + s) * (long long)cin + i) * cout + o] = acc;
    }
}

// ------------------------------------------------------------------- head
__global__ void k_head_fwd(const uint16_t* __restrict__ x, long long npos, int cin, const float* __restrict__ w,
                           const float* __restrict__ b, float* __restrict__ y) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npos; p += (long long)gridDim.x * blockDim.x) {
        float acc = b[0];
        for (int i = 0; i < cin; ++i) acc += bf2f(x[p * cin + i]) * w[i];
        y[p] = acc;
    }
}

__global__ void k_head_bwd_data(const float* __restrict__ gy, long long npos, int cin, const float* __restrict__ w,
                                uint16_t* __restrict__ gx) {
    const long long n = npos * cin;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long p = e / cin;
        gx[e] = f2bf(gy[p] * w[e - p * cin]);
    }
}

// part[block][col]: col < cin -> sum x[p][col] gy[p]; col == cin -> sum gy[p]
__global__ __launch_bounds__(256) void k_head_wgrad_part(const uint16_t* __restrict__ x, const float* __restrict__ gy,
                                                         long long npos, int cin, long long chunk,
                                                         float* __restrict__ part) {
    __shared__ float red[2][128];
    const int col = threadIdx.x & 127, grp = threadIdx.x >> 7;
    const long long p0 = blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npos ? p0 + chunk : npos;
    float s = 0.0f;
    if (col <= cin)
        for (long long p = p0 + grp; p < p1; p += 2) s += (col < cin ? bf2f(x[p * cin + col]) : 1.0f) * gy[p];
    red[grp][col] = s;
    __syncthreads();
    if (grp == 0 && col <= cin) part[blockIdx.x * (long long)(cin + 1) + col] = red[0][col] + red[1][col];
}

// columns 0..cin-1 of the partials -> gw, column cin -> gb (blocks in order)
__global__ void k_head_finish(const float* __restrict__ part, long long nb, int cin, float* __restrict__ gw,
                              float* __restrict__ gb) {
    const int col = threadIdx.x;
    if (col > cin) return;
    float s = 0.0f;
    for (long long q = 0; q < nb; ++q) s += part[q * (cin + 1) + col];
    if (col < cin)
        gw[col] = s;
    else
        gb[0] = s;
}

// -------------------------------------------------------------------- loss
// part[block] = (sum m, sum m (y - t)^2) over the block's chunk
__global__ __launch_bounds__(256) void k_mse_part(const float* __restrict__ y, const float* __restrict__ t,
                                                  const float* __restrict__ m, long long n, long long chunk,
                                                  float* __restrict__ part) {
    __shared__ float rs[256], rm[256];
    const long long p0 = blockIdx.x * chunk;
    const long long p1 = p0 + chunk < n ? p0 + chunk : n;
    float ss = 0.0f, sm = 0.0f;
    for (long long i = p0 + threadIdx.x; i < p1; i += 256) {
        const float w = m ? m[i] : 1.0f;
        const float r = y[i] - t[i];
        ss += w * r * r;
        sm += w;
    }
    rs[threadIdx.x] = ss;
    rm[threadIdx.x] = sm;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            rs[threadIdx.x] += rs[threadIdx.x + k];
            rm[threadIdx.x] += rm[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rm[0];
        part[2 * blockIdx.x + 1] = rs[0];
    }
}

// loss[0] = sum / max(count, 1); loss[1] = max(count, 1)
__global__ __launch_bounds__(256) void k_mse_final(const float* __restrict__ part, int nb, float* __restrict__ loss) {
    __shared__ float rs[256], rm[256];
    float ss = 0.0f, sm = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) {
        sm += part[2 * b];
        ss += part[2 * b + 1];
    }
    rs[threadIdx.x] = ss;
    rm[threadIdx.x] = sm;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            rs[threadIdx.x] += rs[threadIdx.x + k];
            rm[threadIdx.x] += rm[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float cnt = rm[0] > 1.0f ? rm[0] : 1.0f;
        loss[0] = rs[0] / cnt;
        loss[1] = cnt;
    }
}

__global__ void k_mse_grad(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ m,
                           long long n, const float* __restrict__ loss, float* __restrict__ gy) {
    const float sc = 2.0f / loss[1];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float w = m ? m[i] : 1.0f;
        gy[i] = sc * w * (y[i] - t[i]);
    }
}

// ------------------------------------------------------------------- adam
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// ------------------------------------------------------------- warm start
// Node position in the embedding: spherical (r, lat, lon) -> Cartesian km.
__device__ __forceinline__ void embed(int coord, double a0, double a1, double a2, double X[3]) {
    if (coord == 1) {
        const double ct = cos(a1);
        X[0] = a0 * ct * cos(a2);
        X[1] = a0 * ct * sin(a2);
        X[2] = a0 * sin(a1);
    } else {
        X[0] = a0;
        X[1] = a1;
        X[2] = a2;
    }
}

struct WarmGrid {
    int n[3], coord;
    double o[3], h[3];
};

__global__ void k_warm_features(WarmGrid G, const double* __restrict__ s, const double* __restrict__ xi,
                                const double* __restrict__ eta, const double* __restrict__ src_pos,
                                const double* __restrict__ src_par, int stride, int D, int H, int W,
                                uint16_t* __restrict__ feat) {
    const int q = blockIdx.y;
    const long long npos = (long long)D * H * W;
    double Xs[3];
    embed(G.coord, src_pos[3 * q], src_pos[3 * q + 1], src_pos[3 * q + 2], Xs);
    const double inv_s0 = 1.0 / src_par[3 * q];
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npos; p += (long long)gridDim.x * blockDim.x) {
        const int xx = (int)(p % W);
        const int yy = (int)((p / W) % H);
        const int zz = (int)(p / ((long long)W * H));
        const int i = zz * stride, j = yy * stride, k = xx * stride;
        uint16_t f[4] = {0, 0, 0, 0};
        if (i < G.n[0] && j < G.n[1] && k < G.n[2]) {
            const long long node = ((long long)i * G.n[1] + j) * G.n[2] + k;
            double X[3];
            embed(G.coord, G.o[0] + i * G.h[0], G.o[1] + j * G.h[1], G.o[2] + k * G.h[2], X);
            const double d = sqrt((X[0] - Xs[0]) * (X[0] - Xs[0]) + (X[1] - Xs[1]) * (X[1] - Xs[1]) +
                                  (X[2] - Xs[2]) * (X[2] - Xs[2]));
            f[0] = f2bf((float)((s[node] * inv_s0 - 1.0) * NN_FEAT_S));
            f[1] = f2bf((float)(xi[node] * NN_FEAT_A));
            f[2] = f2bf((float)(eta[node] * NN_FEAT_A));
            f[3] = f2bf((float)(d * NN_FEAT_D));
        }
        uint16_t* o = feat + ((long long)q * npos + p) * 16;
        for (int c = 0; c < 16; ++c) o[c] = c < 4 ? f[c] : (uint16_t)0;
    }
}

__global__ void k_warm_target(WarmGrid G, const double* __restrict__ tau, int stride, int D, int H, int W,
                              float* __restrict__ target, float* __restrict__ mask) {
    const int q = blockIdx.y;
    const long long npos = (long long)D * H * W;
    const long long N = (long long)G.n[0] * G.n[1] * G.n[2];
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npos; p += (long long)gridDim.x * blockDim.x) {
        const int xx = (int)(p % W);
        const int yy = (int)((p / W) % H);
        const int zz = (int)(p / ((long long)W * H));
        const int i = zz * stride, j = yy * stride, k = xx * stride;
        const bool ok = i < G.n[0] && j < G.n[1] && k < G.n[2];
        float tv = 0.0f;
        if (ok) tv = (float)((tau[q * N + ((long long)i * G.n[1] + j) * G.n[2] + k] - 1.0) * NN_TARGET_SCALE);
        target[q * npos + p] = tv;
        if (mask) mask[q * npos + p] = ok ? 1.0f : 0.0f;
    }
}

// tau_init = 1 + pred / NN_TARGET_SCALE, trilinear from the coarse nodes,
// clamped to [NN_TAU_INIT_MIN, NN_TAU_INIT_MAX] (NaN -> 1)
__global__ void k_warm_init(WarmGrid G, const float* __restrict__ pred, int stride, int D, int H, int W,
                            double* __restrict__ tau) {
    const int q = blockIdx.y;
    const long long N = (long long)G.n[0] * G.n[1] * G.n[2];
    const long long npos = (long long)D * H * W;
    const int last[3] = {(G.n[0] - 1) / stride, (G.n[1] - 1) / stride, (G.n[2] - 1) / stride};
    const float* pr = pred + q * npos;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < N; x += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(x % G.n[2]);
        const int j = (int)((x / G.n[2]) % G.n[1]);
        const int i = (int)(x / ((long long)G.n[2] * G.n[1]));
        const int idx[3] = {i, j, k};
        int c0[3], c1[3];
        double w1[3];
        for (int a = 0; a < 3; ++a) {
            int b = idx[a] / stride;
            if (b > last[a]) b = last[a];
            c0[a] = b;
            c1[a] = b + 1 <= last[a] ? b + 1 : b;
            w1[a] = (double)(idx[a] - b * stride) / stride;
            if (c1[a] == c0[a]) w1[a] = 0.0;
        }
        double v = 0.0;
        for (int c = 0; c < 8; ++c) {
            const int a = c >> 2, b = (c >> 1) & 1, d = c & 1;
            const double w = (a ? w1[0] : 1.0 - w1[0]) * (b ? w1[1] : 1.0 - w1[1]) * (d ? w1[2] : 1.0 - w1[2]);
            if (w == 0.0) continue;
            const int zz = a ? c1[0] : c0[0], yy = b ? c1[1] : c0[1], xx = d ? c1[2] : c0[2];
            v += w * (double)pr[((long long)zz * H + yy) * W + xx];
        }
        double t = 1.0 + v / NN_TARGET_SCALE;
        if (t != t)
            t = 1.0;
        else
            t = fmin(fmax(t, NN_TAU_INIT_MIN), NN_TAU_INIT_MAX);
        tau[q * N + x] = t;
    }
}

// ===================================================== host: layer launches
int check_ptr(const void* p, const char* name, size_t align) {
    if (!p) return fail(TT_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % align) return fail(TT_EINVAL, "%s must be %zu-byte aligned", name, align);
    return TT_OK;
}

int check_dims(int nbatch, int D, int H, int W) {
    if (nbatch < 1 || D < 1 || H < 1 || W < 1) return fail(TT_EINVAL, "batch and spatial sizes must be >= 1");
    if ((long long)nbatch * D * H * W > (1LL << 40)) return fail(TT_EINVAL, "too many positions");
    return TT_OK;
}

int check_chan(int ct, int co, int c, const char* name) {
    if (c < 1 || co < 0 || co + c > ct) return fail(TT_EINVAL, "%s: channel range [%d, %d) outside %d", name, co, co + c, ct);
    return TT_OK;
}

int conv3_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int cxt, int cxo, int cin, const uint16_t* frag,
              const float* bias, int cout, int relu, uint16_t* y, int cyt, int cyo, hipStream_t st) {
    const long long npos = (long long)nbatch * D * H * W;
    const unsigned blocks = blocks_of(npos, 4 * 16 * kMB);
    const int KB = cin / 16;
    switch (cout / 16) {
        case 1: hipLaunchKernelGGL(k_conv3_fwd<1>, dim3(blocks), dim3(256), 0, st, x, D, H, W, npos, cxt, cxo, KB, frag, bias, relu, y, cyt, cyo); break;
        case 2: hipLaunchKernelGGL(k_conv3_fwd<2>, dim3(blocks), dim3(256), 0, st, x, D, H, W, npos, cxt, cxo, KB, frag, bias, relu, y, cyt, cyo); break;
        case 3: hipLaunchKernelGGL(k_conv3_fwd<3>, dim3(blocks), dim3(256), 0, st, x, D, H, W, npos, cxt, cxo, KB, frag, bias, relu, y, cyt, cyo); break;
        default: hipLaunchKernelGGL(k_conv3_fwd<4>, dim3(blocks), dim3(256), 0, st, x, D, H, W, npos, cxt, cxo, KB, frag, bias, relu, y, cyt, cyo); break;
    }
    NN_LAUNCHED();
    return TT_OK;
}

long long wgrad_slices(long long nrows) {
    long long s = (nrows + 7) / 8;
    return s < 1 ? 1 : (s > 128 ? 128 : s);
}

size_t conv3_wgrad_floats(long long nrows, int cin, int cout) {
    return (size_t)wgrad_slices(nrows) * 27 * cin * cout;
}

long long colsum_blocks(long long npos) {
    long long b = (npos + 4095) / 4096;
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

int colsum(const uint16_t* g, long long npos, int ct, int co, int c, float* out, float* work, hipStream_t st) {
    const long long nb = colsum_blocks(npos);
    const long long chunk = (npos + nb - 1) / nb;
    hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)nb), dim3(256), 0, st, g, npos, ct, co, c, chunk, work);
    NN_LAUNCHED();
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_of(c, 64)), dim3(64), 0, st, work, nb, (long long)c, out);
    NN_LAUNCHED();
    return TT_OK;
}

int conv3_wgrad(const uint16_t* x, int nbatch, int D, int H, int W, int cxt, int cxo, int cin, const uint16_t* gz,
                int cgt, int cgo, int cout, float* gW, float* gb, float* work, hipStream_t st) {
    const long long nrows = (long long)nbatch * D * H;
    const long long ns = wgrad_slices(nrows);
    const long long rps = (nrows + ns - 1) / ns;
    hipLaunchKernelGGL(k_conv3_wgrad, dim3((unsigned)ns, 27), dim3(256), 0, st, x, D, H, W, nrows, cxt, cxo, cin, gz,
                       cgt, cgo, cout, rps, work);
    NN_LAUNCHED();
    const long long n = 27LL * cin * cout;
    hipLaunchKernelGGL(k_sum_slices, dim3(grid_stride_blocks(n)), dim3(256), 0, st, work, ns, n, gW);
    NN_LAUNCHED();
    if (gb) return colsum(gz, nrows * W, cgt, cgo, cout, gb, work, st);
    return TT_OK;
}

size_t colsum_floats(long long npos, int c) { return (size_t)colsum_blocks(npos) * c; }

long long up_slices(long long np) {
    long long s = (np + 63) / 64;
    return s < 1 ? 1 : (s > 256 ? 256 : s);
}

size_t up_work_floats(long long np, int cin, int cout) {
    const size_t a = (size_t)up_slices(np) * 8 * cin * cout;
    const size_t b = colsum_floats(np * 8, cout);
    return a > b ? a : b;
}

int up_bwd(const uint16_t* x, const uint16_t* gy, int nbatch, int D, int H, int W, int cin, int cout, int cgt, int cgo,
           const float* Wu, uint16_t* gx, float* gW, float* gb, float* work, hipStream_t st) {
    const long long np = (long long)nbatch * D * H * W;
    if (gx) {
        hipLaunchKernelGGL(k_up_bwd_data, dim3(grid_stride_blocks(np * cin)), dim3(256), 0, st, gy, np, D, H, W, cin,
                           cout, cgt, cgo, Wu, gx);
        NN_LAUNCHED();
    }
    const long long ns = up_slices(np);
    const long long chunk = (np + ns - 1) / ns;
    hipLaunchKernelGGL(k_up_wgrad_part, dim3((unsigned)ns, 8), dim3(256), 0, st, x, gy, np, D, H, W, cin, cout, cgt,
                       cgo, chunk, work);
    NN_LAUNCHED();
    const long long n = 8LL * cin * cout;
    hipLaunchKernelGGL(k_sum_slices, dim3(grid_stride_blocks(n)), dim3(256), 0, st, work, ns, n, gW);
    NN_LAUNCHED();
    return colsum(gy, np * 8, cgt, cgo, cout, gb, work, st);
}

long long head_blocks(long long npos) {
    long long b = (npos + 4095) / 4096;
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

size_t head_work_floats(long long npos, int cin) { return (size_t)head_blocks(npos) * (cin + 1); }

int head_bwd(const uint16_t* x, const float* gy, long long npos, int cin, const float* w, uint16_t* gx, float* gw,
             float* gb, float* work, hipStream_t st) {
    if (gx) {
        hipLaunchKernelGGL(k_head_bwd_data, dim3(grid_stride_blocks(npos * cin)), dim3(256), 0, st, gy, npos, cin, w, gx);
        NN_LAUNCHED();
    }
    const long long nb = head_blocks(npos);
    const long long chunk = (npos + nb - 1) / nb;
    hipLaunchKernelGGL(k_head_wgrad_part, dim3((unsigned)nb), dim3(256), 0, st, x, gy, npos, cin, chunk, work);
    NN_LAUNCHED();
    hipLaunchKernelGGL(k_head_finish, dim3(1), dim3(128), 0, st, work, nb, cin, gw, gb);
    NN_LAUNCHED();
    return TT_OK;
}

// ============================================================ U-Net plan
enum { E1A, E1B, E2A, E2B, E3A, E3B, BNA, BNB, D3A, D3B, D2A, D2B, D1A, D1B, NCONV };
enum { U3, U2, U1, NUP };

struct ConvDef {
    int ci, co, cip;     // input channels (real), output channels, padded input channels
    size_t w, b;         // parameter offsets (floats)
    size_t fw, fb;       // fragment offsets: forward, data-gradient (bf16 elements)
};
struct UpDef {
    int ci, co;
    size_t w, b;
};
struct Net {
    int c[4], in_ch;
    ConvDef conv[NCONV];
    UpDef up[NUP];
    size_t head_w, head_b, nparams, nfrag;
};

int make_net(const nn_unet_cfg* cfg, Net& N) {
    if (!cfg) return fail(TT_EINVAL, "cfg is NULL");
    for (int l = 0; l < 4; ++l)
        if (cfg->ch[l] < 16 || cfg->ch[l] % 16 || cfg->ch[l] > 64)
            return fail(TT_EINVAL, "cfg.ch[%d] = %d: channels must be multiples of 16 in [16, 64]", l, cfg->ch[l]);
    for (int l = 0; l < 3; ++l)
        if (2 * cfg->ch[l] > 64) return fail(TT_EINVAL, "decoder convolutions need 2 * ch[%d] <= 64", l);
    if (cfg->in_ch < 1 || cfg->in_ch > 16) return fail(TT_EINVAL, "cfg.in_ch must be in [1, 16]");
    std::memset(&N, 0, sizeof N);
    for (int l = 0; l < 4; ++l) N.c[l] = cfg->ch[l];
    N.in_ch = cfg->in_ch;
    const int c1 = N.c[0], c2 = N.c[1], c3 = N.c[2], c4 = N.c[3];
    const int io[NCONV][2] = {{N.in_ch, c1}, {c1, c1}, {c1, c2}, {c2, c2}, {c2, c3}, {c3, c3}, {c3, c4},
                              {c4, c4},      {2 * c3, c3}, {c3, c3}, {2 * c2, c2}, {c2, c2}, {2 * c1, c1}, {c1, c1}};
    size_t off = 0, fo = 0;
    for (int k = 0; k < NCONV; ++k) {
        ConvDef& C = N.conv[k];
        C.ci = io[k][0];
        C.co = io[k][1];
        C.cip = (C.ci + 15) / 16 * 16;
        C.w = off;
        off += 27 * (size_t)C.ci * C.co;
        C.b = off;
        off += C.co;
        C.fw = fo;
        fo += 27 * (size_t)C.cip * C.co;
        C.fb = fo;
        if (k != E1A) fo += 27 * (size_t)C.ci * C.co;
    }
    const int uio[NUP][2] = {{c4, c3}, {c3, c2}, {c2, c1}};
    for (int k = 0; k < NUP; ++k) {
        UpDef& U = N.up[k];
        U.ci = uio[k][0];
        U.co = uio[k][1];
        U.w = off;
        off += 8 * (size_t)U.ci * U.co;
        U.b = off;
        off += U.co;
    }
    N.head_w = off;
    off += c1;
    N.head_b = off;
    off += 1;
    N.nparams = off;
    N.nfrag = fo;
    return TT_OK;
}

// Activation and gradient buffers of one (batch, D, H, W) in the workspace.
struct Acts {
    long long P[4];
    uint16_t *a1, *cat1, *p1, *a2, *cat2, *p2, *a3, *cat3, *p3, *b1, *b2, *d3a, *d3b, *d2a, *d2b, *d1a, *d1b;
    uint16_t *gA[3], *gZ[3], *gcat[3], *gBa, *gBb, *gZ4, *gP[3];
    float* work;
    size_t bytes;
};

size_t aup(size_t v) { return (v + 255) & ~(size_t)255; }

int check_net_dims(int nbatch, int D, int H, int W) {
    if (check_dims(nbatch, D, H, W)) return TT_EINVAL;
    if (D % 8 || H % 8 || W % 8) return fail(TT_EINVAL, "U-Net spatial sizes must be multiples of 8 (got %d %d %d)", D, H, W);
    return TT_OK;
}

// Lays out the buffers from base (or only measures when base is NULL).
void layout(const Net& N, int nbatch, int D, int H, int W, int train, char* base, Acts& A) {
    std::memset(&A, 0, sizeof A);
    A.P[0] = (long long)nbatch * D * H * W;
    for (int l = 1; l < 4; ++l) A.P[l] = A.P[l - 1] / 8;
    const int c1 = N.c[0], c2 = N.c[1], c3 = N.c[2], c4 = N.c[3];
    size_t off = 0;
    auto take16 = [&](long long np, int c) -> uint16_t* {
        uint16_t* p = base ? reinterpret_cast<uint16_t*>(base + off) : nullptr;
        off += aup((size_t)np * c * sizeof(uint16_t));
        return p;
    };
    A.a1 = take16(A.P[0], c1);
    A.cat1 = take16(A.P[0], 2 * c1);
    A.p1 = take16(A.P[1], c1);
    A.a2 = take16(A.P[1], c2);
    A.cat2 = take16(A.P[1], 2 * c2);
    A.p2 = take16(A.P[2], c2);
    A.a3 = take16(A.P[2], c3);
    A.cat3 = take16(A.P[2], 2 * c3);
    A.p3 = take16(A.P[3], c3);
    A.b1 = take16(A.P[3], c4);
    A.b2 = take16(A.P[3], c4);
    A.d3a = take16(A.P[2], c3);
    A.d3b = take16(A.P[2], c3);
    A.d2a = take16(A.P[1], c2);
    A.d2b = take16(A.P[1], c2);
    A.d1a = take16(A.P[0], c1);
    A.d1b = take16(A.P[0], c1);
    if (train) {
        const int cl[3] = {c1, c2, c3};
        for (int l = 0; l < 3; ++l) {
            A.gA[l] = take16(A.P[l], cl[l]);
            A.gZ[l] = take16(A.P[l], cl[l]);
            A.gcat[l] = take16(A.P[l], 2 * cl[l]);
        }
        A.gBa = take16(A.P[3], c4);
        A.gBb = take16(A.P[3], c4);
        A.gZ4 = take16(A.P[3], c4);
        A.gP[0] = take16(A.P[1], c1);
        A.gP[1] = take16(A.P[2], c2);
        A.gP[2] = take16(A.P[3], c3);
        // reduction scratch: the largest of the layers' needs
        size_t wf = 0;
        const int lev[NCONV] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};
        for (int k = 0; k < NCONV; ++k) {
            const long long np = A.P[lev[k]];
            const long long nrows = np / (W >> lev[k]);  // (n, z, y) rows of the level
            size_t f = conv3_wgrad_floats(nrows, N.conv[k].ci, N.conv[k].co);
            size_t g = colsum_floats(np, N.conv[k].co);
            if (f > wf) wf = f;
            if (g > wf) wf = g;
        }
        for (int k = 0; k < NUP; ++k) {
            const size_t f = up_work_floats(A.P[3 - k], N.up[k].ci, N.up[k].co);
            if (f > wf) wf = f;
        }
        const size_t hf = head_work_floats(A.P[0], c1);
        if (hf > wf) wf = hf;
        A.work = base ? reinterpret_cast<float*>(base + off) : nullptr;
        off += aup(wf * sizeof(float));
    }
    A.bytes = off;
}

int conv_layer_fwd(const Net& N, int k, const float* prm, const uint16_t* frag, const uint16_t* x, int cxt, int cxo,
                   int nbatch, int D, int H, int W, uint16_t* y, int cyt, int cyo, hipStream_t st) {
    const ConvDef& C = N.conv[k];
    return conv3_fwd(x, nbatch, D, H, W, cxt, cxo, C.cip, frag + C.fw, prm + C.b, C.co, 1, y, cyt, cyo, st);
}

int relu_mask(const uint16_t* g, const uint16_t* y, long long npos, int ct, int co, int c, uint16_t* go, int cot,
              int coo, hipStream_t st) {
    hipLaunchKernelGGL(k_relu_mask, dim3(grid_stride_blocks(npos * c)), dim3(256), 0, st, g, y, npos, ct, co, c, go,
                       cot, coo);
    NN_LAUNCHED();
    return TT_OK;
}

int pool_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int ct, int co, int c, uint16_t* y, hipStream_t st) {
    const long long nq = (long long)nbatch * (D / 2) * (H / 2) * (W / 2);
    hipLaunchKernelGGL(k_pool_fwd, dim3(grid_stride_blocks(nq * c)), dim3(256), 0, st, x, nq, D / 2, H / 2, W / 2, ct,
                       co, c, y);
    NN_LAUNCHED();
    return TT_OK;
}

int pool_bwd(const uint16_t* x, const uint16_t* gy, int nbatch, int D, int H, int W, int ct, int co, int c,
             uint16_t* gx, int accumulate, hipStream_t st) {
    const long long nq = (long long)nbatch * (D / 2) * (H / 2) * (W / 2);
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid_stride_blocks(nq * c)), dim3(256), 0, st, x, gy, nq, D / 2, H / 2,
                       W / 2, ct, co, c, gx, accumulate);
    NN_LAUNCHED();
    return TT_OK;
}

int up_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int cin, const float* Wu, const float* b, int cout,
           uint16_t* y, int cyt, int cyo, hipStream_t st) {
    const long long nout = (long long)nbatch * D * H * W * 8;
    hipLaunchKernelGGL(k_up_fwd, dim3(grid_stride_blocks(nout * cout)), dim3(256), 0, st, x, nout, D, H, W, cin, Wu,
                       b, cout, y, cyt, cyo);
    NN_LAUNCHED();
    return TT_OK;
}

#define NN_TRY(expr)          \
    do {                      \
        int rc_ = (expr);     \
        if (rc_) return rc_;  \
    } while (0)

int unet_forward(const Net& N, const float* prm, const uint16_t* frag, const uint16_t* x, int nb, int D, int H, int W,
                 float* y, const Acts& A, hipStream_t st) {
    const int c1 = N.c[0], c2 = N.c[1], c3 = N.c[2], c4 = N.c[3];
    int d = D, h = H, w = W;
    // level 1
    NN_TRY(conv_layer_fwd(N, E1A, prm, frag, x, 16, 0, nb, d, h, w, A.a1, c1, 0, st));
    NN_TRY(conv_layer_fwd(N, E1B, prm, frag, A.a1, c1, 0, nb, d, h, w, A.cat1, 2 * c1, c1, st));
    NN_TRY(pool_fwd(A.cat1, nb, d, h, w, 2 * c1, c1, c1, A.p1, st));
    d /= 2, h /= 2, w /= 2;
    NN_TRY(conv_layer_fwd(N, E2A, prm, frag, A.p1, c1, 0, nb, d, h, w, A.a2, c2, 0, st));
    NN_TRY(conv_layer_fwd(N, E2B, prm, frag, A.a2, c2, 0, nb, d, h, w, A.cat2, 2 * c2, c2, st));
    NN_TRY(pool_fwd(A.cat2, nb, d, h, w, 2 * c2, c2, c2, A.p2, st));
    d /= 2, h /= 2, w /= 2;
    NN_TRY(conv_layer_fwd(N, E3A, prm, frag, A.p2, c2, 0, nb, d, h, w, A.a3, c3, 0, st));
    NN_TRY(conv_layer_fwd(N, E3B, prm, frag, A.a3, c3, 0, nb, d, h, w, A.cat3, 2 * c3, c3, st));
    NN_TRY(pool_fwd(A.cat3, nb, d, h, w, 2 * c3, c3, c3, A.p3, st));
    d /= 2, h /= 2, w /= 2;
    NN_TRY(conv_layer_fwd(N, BNA, prm, frag, A.p3, c3, 0, nb, d, h, w, A.b1, c4, 0, st));
    NN_TRY(conv_layer_fwd(N, BNB, prm, frag, A.b1, c4, 0, nb, d, h, w, A.b2, c4, 0, st));
    // decoder
    NN_TRY(up_fwd(A.b2, nb, d, h, w, c4, prm + N.up[U3].w, prm + N.up[U3].b, c3, A.cat3, 2 * c3, 0, st));
    d *= 2, h *= 2, w *= 2;
    NN_TRY(conv_layer_fwd(N, D3A, prm, frag, A.cat3, 2 * c3, 0, nb, d, h, w, A.d3a, c3, 0, st));
    NN_TRY(conv_layer_fwd(N, D3B, prm, frag, A.d3a, c3, 0, nb, d, h, w, A.d3b, c3, 0, st));
    NN_TRY(up_fwd(A.d3b, nb, d, h, w, c3, prm + N.up[U2].w, prm + N.up[U2].b, c2, A.cat2, 2 * c2, 0, st));
    d *= 2, h *= 2, w *= 2;
    NN_TRY(conv_layer_fwd(N, D2A, prm, frag, A.cat2, 2 * c2, 0, nb, d, h, w, A.d2a, c2, 0, st));
    NN_TRY(conv_layer_fwd(N, D2B, prm, frag, A.d2a, c2, 0, nb, d, h, w, A.d2b, c2, 0, st));
    NN_TRY(up_fwd(A.d2b, nb, d, h, w, c2, prm + N.up[U1].w, prm + N.up[U1].b, c1, A.cat1, 2 * c1, 0, st));
    d *= 2, h *= 2, w *= 2;
    NN_TRY(conv_layer_fwd(N, D1A, prm, frag, A.cat1, 2 * c1, 0, nb, d, h, w, A.d1a, c1, 0, st));
    NN_TRY(conv_layer_fwd(N, D1B, prm, frag, A.d1a, c1, 0, nb, d, h, w, A.d1b, c1, 0, st));
    hipLaunchKernelGGL(k_head_fwd, dim3(grid_stride_blocks(A.P[0])), dim3(256), 0, st, A.d1b, A.P[0], c1,
                       prm + N.head_w, prm + N.head_b, y);
    NN_LAUNCHED();
    return TT_OK;
}

// Backward of one conv + ReLU layer: g_out (gradient of the layer's ReLU
// output, in (gt, go)) -> gZ = g_out * (y > 0); weight and bias gradients from
// the layer input x; data gradient into gin (unless gin is NULL).
int conv_layer_bwd(const Net& N, int k, const uint16_t* frag, float* grad, const uint16_t* g_out, const uint16_t* y,
                   int yt, int yo, const uint16_t* x, int cxt, int cxo, int nb, int D, int H, int W, uint16_t* gZ,
                   uint16_t* gin, int cgt, float* work, hipStream_t st) {
    const ConvDef& C = N.conv[k];
    const long long np = (long long)nb * D * H * W;
    NN_TRY(relu_mask(g_out, y, np, yt, yo, C.co, gZ, C.co, 0, st));
    NN_TRY(conv3_wgrad(x, nb, D, H, W, cxt, cxo, C.ci, gZ, C.co, 0, C.co, grad + C.w, grad + C.b, work, st));
    if (gin) NN_TRY(conv3_fwd(gZ, nb, D, H, W, C.co, 0, C.co, frag + C.fb, nullptr, C.ci, 0, gin, cgt, 0, st));
    return TT_OK;
}

int unet_backward(const Net& N, const float* prm, const uint16_t* frag, const float* gy, const uint16_t* x, int nb,
                  int D, int H, int W, float* grad, const Acts& A, hipStream_t st) {
    const int c1 = N.c[0], c2 = N.c[1], c3 = N.c[2], c4 = N.c[3];
    float* wk = A.work;
    int d = D, h = H, w = W;
    // head
    NN_TRY(head_bwd(A.d1b, gy, A.P[0], c1, prm + N.head_w, A.gA[0], grad + N.head_w, grad + N.head_b, wk, st));
    // level-1 decoder
    NN_TRY(conv_layer_bwd(N, D1B, frag, grad, A.gA[0], A.d1b, c1, 0, A.d1a, c1, 0, nb, d, h, w, A.gZ[0], A.gA[0], c1, wk, st));
    NN_TRY(conv_layer_bwd(N, D1A, frag, grad, A.gA[0], A.d1a, c1, 0, A.cat1, 2 * c1, 0, nb, d, h, w, A.gZ[0], A.gcat[0], 2 * c1, wk, st));
    d /= 2, h /= 2, w /= 2;
    NN_TRY(up_bwd(A.d2b, A.gcat[0], nb, d, h, w, c2, c1, 2 * c1, 0, prm + N.up[U1].w, A.gA[1], grad + N.up[U1].w,
                  grad + N.up[U1].b, wk, st));
    NN_TRY(conv_layer_bwd(N, D2B, frag, grad, A.gA[1], A.d2b, c2, 0, A.d2a, c2, 0, nb, d, h, w, A.gZ[1], A.gA[1], c2, wk, st));
    NN_TRY(conv_layer_bwd(N, D2A, frag, grad, A.gA[1], A.d2a, c2, 0, A.cat2, 2 * c2, 0, nb, d, h, w, A.gZ[1], A.gcat[1], 2 * c2, wk, st));
    d /= 2, h /= 2, w /= 2;
    NN_TRY(up_bwd(A.d3b, A.gcat[1], nb, d, h, w, c3, c2, 2 * c2, 0, prm + N.up[U2].w, A.gA[2], grad + N.up[U2].w,
                  grad + N.up[U2].b, wk, st));
    NN_TRY(conv_layer_bwd(N, D3B, frag, grad, A.gA[2], A.d3b, c3, 0, A.d3a, c3, 0, nb, d, h, w, A.gZ[2], A.gA[2], c3, wk, st));
    NN_TRY(conv_layer_bwd(N, D3A, frag, grad, A.gA[2], A.d3a, c3, 0, A.cat3, 2 * c3, 0, nb, d, h, w, A.gZ[2], A.gcat[2], 2 * c3, wk, st));
    d /= 2, h /= 2, w /= 2;
    NN_TRY(up_bwd(A.b2, A.gcat[2], nb, d, h, w, c4, c3, 2 * c3, 0, prm + N.up[U3].w, A.gBa, grad + N.up[U3].w,
                  grad + N.up[U3].b, wk, st));
    // bottleneck
    NN_TRY(conv_layer_bwd(N, BNB, frag, grad, A.gBa, A.b2, c4, 0, A.b1, c4, 0, nb, d, h, w, A.gZ4, A.gBb, c4, wk, st));
    NN_TRY(conv_layer_bwd(N, BNA, frag, grad, A.gBb, A.b1, c4, 0, A.p3, c3, 0, nb, d, h, w, A.gZ4, A.gP[2], c3, wk, st));
    d *= 2, h *= 2, w *= 2;
    // level 3 encoder: skip gradient + pooled gradient
    NN_TRY(pool_bwd(A.cat3, A.gP[2], nb, d, h, w, 2 * c3, c3, c3, A.gcat[2], 1, st));
    NN_TRY(conv_layer_bwd(N, E3B, frag, grad, A.gcat[2], A.cat3, 2 * c3, c3, A.a3, c3, 0, nb, d, h, w, A.gZ[2], A.gA[2], c3, wk, st));
    NN_TRY(conv_layer_bwd(N, E3A, frag, grad, A.gA[2], A.a3, c3, 0, A.p2, c2, 0, nb, d, h, w, A.gZ[2], A.gP[1], c2, wk, st));
    d *= 2, h *= 2, w *= 2;
    NN_TRY(pool_bwd(A.cat2, A.gP[1], nb, d, h, w, 2 * c2, c2, c2, A.gcat[1], 1, st));
    NN_TRY(conv_layer_bwd(N, E2B, frag, grad, A.gcat[1], A.cat2, 2 * c2, c2, A.a2, c2, 0, nb, d, h, w, A.gZ[1], A.gA[1], c2, wk, st));
    NN_TRY(conv_layer_bwd(N, E2A, frag, grad, A.gA[1], A.a2, c2, 0, A.p1, c1, 0, nb, d, h, w, A.gZ[1], A.gP[0], c1, wk, st));
    d *= 2, h *= 2, w *= 2;
    NN_TRY(pool_bwd(A.cat1, A.gP[0], nb, d, h, w, 2 * c1, c1, c1, A.gcat[0], 1, st));
    NN_TRY(conv_layer_bwd(N, E1B, frag, grad, A.gcat[0], A.cat1, 2 * c1, c1, A.a1, c1, 0, nb, d, h, w, A.gZ[0], A.gA[0], c1, wk, st));
    NN_TRY(conv_layer_bwd(N, E1A, frag, grad, A.gA[0], A.a1, c1, 0, x, 16, 0, nb, d, h, w, A.gZ[0], nullptr, 0, wk, st));
    return TT_OK;
}

int warm_grid(const tt_grid* g, WarmGrid& W) {
    if (!g) return fail(TT_EINVAL, "grid is NULL");
    if (g->coord != 0 && g->coord != 1) return fail(TT_EINVAL, "grid.coord must be 0 or 1");
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1) return fail(TT_EINVAL, "grid.n[%d] must be >= 1", a);
        W.n[a] = g->n[a];
        W.o[a] = g->o[a];
        W.h[a] = g->h[a];
    }
    W.coord = g->coord;
    return TT_OK;
}

int check_coarse(const tt_grid* g, int stride, int D, int H, int W) {
    if (stride < 1) return fail(TT_EINVAL, "stride must be >= 1");
    if (D < 1 || H < 1 || W < 1) return fail(TT_EINVAL, "coarse sizes must be >= 1");
    const int c[3] = {D, H, W};
    for (int a = 0; a < 3; ++a)
        if ((g->n[a] - 1) / stride + 1 > c[a])
            return fail(TT_EINVAL, "coarse axis %d has %d nodes, needs >= %d", a, c[a], (g->n[a] - 1) / stride + 1);
    return TT_OK;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

int nn_to_bf16(const float* x, int64_t n, uint16_t* y, void* stream) {
    if (n < 0) return fail(TT_EINVAL, "n < 0");
    if (n == 0) return TT_OK;
    NN_TRY(check_ptr(x, "x", 4));
    NN_TRY(check_ptr(y, "y", 2));
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_stride_blocks(n)), dim3(256), 0, S(stream), x, (long long)n, y);
    NN_LAUNCHED();
    return TT_OK;
}

int nn_from_bf16(const uint16_t* x, int64_t n, float* y, void* stream) {
    if (n < 0) return fail(TT_EINVAL, "n < 0");
    if (n == 0) return TT_OK;
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(y, "y", 4));
    hipLaunchKernelGGL(k_from_bf16, dim3(grid_stride_blocks(n)), dim3(256), 0, S(stream), x, (long long)n, y);
    NN_LAUNCHED();
    return TT_OK;
}

int nn_conv3_pack(const float* W, int cin, int cout, int flip, uint16_t* frag, void* stream) {
    NN_TRY(check_ptr(W, "W", 4));
    NN_TRY(check_ptr(frag, "frag", 8));
    if (cout < 16 || cout % 16 || cout > 64) return fail(TT_EINVAL, "cout must be a multiple of 16 in [16, 64]");
    if (cin < 1 || cin > 64) return fail(TT_EINVAL, "cin must be in [1, 64]");
    if (flip && cin % 16) return fail(TT_EINVAL, "flip = 1 needs cin a multiple of 16");
    const int KB = flip ? cout / 16 : (cin + 15) / 16;
    const int NB = flip ? cin / 16 : cout / 16;
    hipLaunchKernelGGL(k_conv3_pack, dim3(grid_stride_blocks(27LL * KB * NB * 256)), dim3(256), 0, S(stream), W, cin,
                       cout, KB, NB, flip, frag);
    NN_LAUNCHED();
    return TT_OK;
}

int nn_conv3_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int cx_total, int cx_off, int cin,
                 const uint16_t* frag, const float* bias, int cout, int relu, uint16_t* y, int cy_total, int cy_off,
                 void* stream) {
    NN_TRY(check_dims(nbatch, D, H, W));
    NN_TRY(check_ptr(x, "x", 8));
    NN_TRY(check_ptr(frag, "frag", 8));
    NN_TRY(check_ptr(y, "y", 2));
    if (cin < 16 || cin % 16 || cin > 64) return fail(TT_EINVAL, "cin must be a multiple of 16 in [16, 64]");
    if (cout < 16 || cout % 16 || cout > 64) return fail(TT_EINVAL, "cout must be a multiple of 16 in [16, 64]");
    if (cx_total % 4 || cx_off % 4) return fail(TT_EINVAL, "cx_total and cx_off must be multiples of 4");
    NN_TRY(check_chan(cx_total, cx_off, cin, "x"));
    NN_TRY(check_chan(cy_total, cy_off, cout, "y"));
    return conv3_fwd(x, nbatch, D, H, W, cx_total, cx_off, cin, frag, bias, cout, relu, y, cy_total, cy_off, S(stream));
}

size_t nn_conv3_wgrad_work(int nbatch, int D, int H, int W, int cin, int cout) {
    if (nbatch < 1 || D < 1 || H < 1 || W < 1 || cin < 1 || cout < 1) return 0;
    const long long nrows = (long long)nbatch * D * H;
    const size_t a = conv3_wgrad_floats(nrows, cin, cout), b = colsum_floats(nrows * W, cout);
    return (a > b ? a : b) * sizeof(float);
}

int nn_conv3_wgrad(const uint16_t* x, int nbatch, int D, int H, int W, int cx_total, int cx_off, int cin,
                   const uint16_t* gz, int cg_total, int cg_off, int cout, float* gW, float* gb, float* work,
                   size_t work_bytes, void* stream) {
    NN_TRY(check_dims(nbatch, D, H, W));
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(gz, "gz", 2));
    NN_TRY(check_ptr(gW, "gW", 4));
    NN_TRY(check_ptr(work, "work", 4));
    if (cin < 1 || cin > 64) return fail(TT_EINVAL, "cin must be in [1, 64]");
    if (cout < 16 || cout % 16 || cout > 64) return fail(TT_EINVAL, "cout must be a multiple of 16 in [16, 64]");
    NN_TRY(check_chan(cx_total, cx_off, cin, "x"));
    NN_TRY(check_chan(cg_total, cg_off, cout, "gz"));
    if (work_bytes < nn_conv3_wgrad_work(nbatch, D, H, W, cin, cout)) return fail(TT_EINVAL, "work too small");
    return conv3_wgrad(x, nbatch, D, H, W, cx_total, cx_off, cin, gz, cg_total, cg_off, cout, gW, gb, work, S(stream));
}

int nn_relu_mask(const uint16_t* g, const uint16_t* y, int64_t npos, int c_total, int c_off, int c, uint16_t* g_out,
                 int co_total, int co_off, void* stream) {
    if (npos < 0) return fail(TT_EINVAL, "npos < 0");
    if (npos == 0) return TT_OK;
    NN_TRY(check_ptr(g, "g", 2));
    NN_TRY(check_ptr(y, "y", 2));
    NN_TRY(check_ptr(g_out, "g_out", 2));
    NN_TRY(check_chan(c_total, c_off, c, "g"));
    NN_TRY(check_chan(co_total, co_off, c, "g_out"));
    return relu_mask(g, y, npos, c_total, c_off, c, g_out, co_total, co_off, S(stream));
}

int nn_pool_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int c_total, int c_off, int c, uint16_t* y,
                void* stream) {
    NN_TRY(check_dims(nbatch, D, H, W));
    if (D % 2 || H % 2 || W % 2) return fail(TT_EINVAL, "pooling needs even sizes");
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(y, "y", 2));
    NN_TRY(check_chan(c_total, c_off, c, "x"));
    return pool_fwd(x, nbatch, D, H, W, c_total, c_off, c, y, S(stream));
}

int nn_pool_bwd(const uint16_t* x, const uint16_t* gy, int nbatch, int D, int H, int W, int c_total, int c_off, int c,
                uint16_t* gx, int accumulate, void* stream) {
    NN_TRY(check_dims(nbatch, D, H, W));
    if (D % 2 || H % 2 || W % 2) return fail(TT_EINVAL, "pooling needs even sizes");
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(gy, "gy", 2));
    NN_TRY(check_ptr(gx, "gx", 2));
    NN_TRY(check_chan(c_total, c_off, c, "x"));
    return pool_bwd(x, gy, nbatch, D, H, W, c_total, c_off, c, gx, accumulate, S(stream));
}

int nn_up_fwd(const uint16_t* x, int nbatch, int D, int H, int W, int cin, const float* Wup, const float* b, int cout,
              uint16_t* y, int cy_total, int cy_off, void* stream) {
    NN_TRY(check_dims(nbatch, D, H, W));
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(Wup, "Wup", 4));
    NN_TRY(check_ptr(b, "b", 4));
    NN_TRY(check_ptr(y, "y", 2));
    if (cin < 1 || cout < 1) return fail(TT_EINVAL, "channel counts must be >= 1");
    NN_TRY(check_chan(cy_total, cy_off, cout, "y"));
    return up_fwd(x, nbatch, D, H, W, cin, Wup, b, cout, y, cy_total, cy_off, S(stream));
}

size_t nn_up_wgrad_work(int nbatch, int D, int H, int W, int cin, int cout) {
    if (nbatch < 1 || D < 1 || H < 1 || W < 1 || cin < 1 || cout < 1) return 0;
    return up_work_floats((long long)nbatch * D * H * W, cin, cout) * sizeof(float);
}

int nn_up_bwd(const uint16_t* x, const uint16_t* gy, int nbatch, int D, int H, int W, int cin, int cout, int cg_total,
              int cg_off, const float* Wup, uint16_t* gx, float* gW, float* gb, float* work, size_t work_bytes,
              void* stream) {
    NN_TRY(check_dims(nbatch, D, H, W));
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(gy, "gy", 2));
    NN_TRY(check_ptr(Wup, "Wup", 4));
    NN_TRY(check_ptr(gW, "gW", 4));
    NN_TRY(check_ptr(gb, "gb", 4));
    NN_TRY(check_ptr(work, "work", 4));
    if (cin < 1 || cout < 1 || cout > 64) return fail(TT_EINVAL, "channel counts must be in [1, 64]");
    NN_TRY(check_chan(cg_total, cg_off, cout, "gy"));
    if (work_bytes < nn_up_wgrad_work(nbatch, D, H, W, cin, cout)) return fail(TT_EINVAL, "work too small");
    return up_bwd(x, gy, nbatch, D, H, W, cin, cout, cg_total, cg_off, Wup, gx, gW, gb, work, S(stream));
}

int nn_head_fwd(const uint16_t* x, int64_t npos, int cin, const float* w, const float* b, float* y, void* stream) {
    if (npos < 1 || cin < 1 || cin > 127) return fail(TT_EINVAL, "need npos >= 1 and cin in [1, 127]");
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(w, "w", 4));
    NN_TRY(check_ptr(b, "b", 4));
    NN_TRY(check_ptr(y, "y", 4));
    hipLaunchKernelGGL(k_head_fwd, dim3(grid_stride_blocks(npos)), dim3(256), 0, S(stream), x, (long long)npos, cin, w,
                       b, y);
    NN_LAUNCHED();
    return TT_OK;
}

size_t nn_head_work(int64_t npos, int cin) {
    if (npos < 1 || cin < 1) return 0;
    return head_work_floats(npos, cin) * sizeof(float);
}

int nn_head_bwd(const uint16_t* x, const float* gy, int64_t npos, int cin, const float* w, uint16_t* gx, float* gw,
                float* gb, float* work, size_t work_bytes, void* stream) {
    if (npos < 1 || cin < 1 || cin > 127) return fail(TT_EINVAL, "need npos >= 1 and cin in [1, 127]");
    NN_TRY(check_ptr(x, "x", 2));
    NN_TRY(check_ptr(gy, "gy", 4));
    NN_TRY(check_ptr(w, "w", 4));
    NN_TRY(check_ptr(gw, "gw", 4));
    NN_TRY(check_ptr(gb, "gb", 4));
    NN_TRY(check_ptr(work, "work", 4));
    if (work_bytes < nn_head_work(npos, cin)) return fail(TT_EINVAL, "work too small");
    return head_bwd(x, gy, npos, cin, w, gx, gw, gb, work, S(stream));
}

int nn_mse(const float* y, const float* t, const float* mask, int64_t n, float* loss, float* gy, void* stream) {
    if (n < 1) return fail(TT_EINVAL, "n must be >= 1");
    NN_TRY(check_ptr(y, "y", 4));
    NN_TRY(check_ptr(t, "t", 4));
    NN_TRY(check_ptr(loss, "loss", 4));
    NN_TRY(check_ptr(gy, "gy", 4));
    long long nb = (n + 65535) / 65536;
    if (nb > NN_MSE_MAX_BLOCKS) nb = NN_MSE_MAX_BLOCKS;
    const long long chunk = (n + nb - 1) / nb;
    hipStream_t st = S(stream);
    float* part = loss + 2;
    hipLaunchKernelGGL(k_mse_part, dim3((unsigned)nb), dim3(256), 0, st, y, t, mask, (long long)n, chunk, part);
    NN_LAUNCHED();
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, part, (int)nb, loss);
    NN_LAUNCHED();
    hipLaunchKernelGGL(k_mse_grad, dim3(grid_stride_blocks(n)), dim3(256), 0, st, y, t, mask, (long long)n, loss, gy);
    NN_LAUNCHED();
    return TT_OK;
}

int nn_adam(float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, float beta1, float beta2,
            float eps, void* stream) {
    if (n < 1 || step < 1) return fail(TT_EINVAL, "need n >= 1 and step >= 1");
    NN_TRY(check_ptr(p, "p", 4));
    NN_TRY(check_ptr(g, "g", 4));
    NN_TRY(check_ptr(m, "m", 4));
    NN_TRY(check_ptr(v, "v", 4));
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    hipLaunchKernelGGL(k_adam, dim3(grid_stride_blocks(n)), dim3(256), 0, S(stream), p, g, m, v, (long long)n, lr,
                       beta1, beta2, eps, c1, c2);
    NN_LAUNCHED();
    return TT_OK;
}

size_t nn_unet_nparams(const nn_unet_cfg* cfg) {
    Net N;
    return make_net(cfg, N) ? 0 : N.nparams;
}

size_t nn_unet_nfrag(const nn_unet_cfg* cfg) {
    Net N;
    return make_net(cfg, N) ? 0 : N.nfrag;
}

size_t nn_unet_workspace(const nn_unet_cfg* cfg, int nbatch, int D, int H, int W, int train) {
    Net N;
    if (make_net(cfg, N) || check_net_dims(nbatch, D, H, W)) return 0;
    Acts A;
    layout(N, nbatch, D, H, W, train, nullptr, A);
    return A.bytes;
}

int nn_unet_pack(const nn_unet_cfg* cfg, const float* params, uint16_t* frag, void* stream) {
    Net N;
    NN_TRY(make_net(cfg, N));
    NN_TRY(check_ptr(params, "params", 4));
    NN_TRY(check_ptr(frag, "frag", 8));
    for (int k = 0; k < NCONV; ++k) {
        const ConvDef& C = N.conv[k];
        NN_TRY(nn_conv3_pack(params + C.w, C.ci, C.co, 0, frag + C.fw, stream));
        if (k != E1A) NN_TRY(nn_conv3_pack(params + C.w, C.ci, C.co, 1, frag + C.fb, stream));
    }
    return TT_OK;
}

int nn_unet_forward(const nn_unet_cfg* cfg, const float* params, const uint16_t* frag, const uint16_t* x, int nbatch,
                    int D, int H, int W, float* y, void* ws, size_t ws_bytes, int train, void* stream) {
    Net N;
    NN_TRY(make_net(cfg, N));
    NN_TRY(check_net_dims(nbatch, D, H, W));
    NN_TRY(check_ptr(params, "params", 4));
    NN_TRY(check_ptr(frag, "frag", 8));
    NN_TRY(check_ptr(x, "x", 8));
    NN_TRY(check_ptr(y, "y", 4));
    NN_TRY(check_ptr(ws, "ws", 256));
    Acts A;
    layout(N, nbatch, D, H, W, train, static_cast<char*>(ws), A);
    if (ws_bytes < A.bytes) return fail(TT_EINVAL, "workspace too small: %zu < %zu", ws_bytes, A.bytes);
    return unet_forward(N, params, frag, x, nbatch, D, H, W, y, A, S(stream));
}

int nn_unet_backward(const nn_unet_cfg* cfg, const float* params, const uint16_t* frag, const uint16_t* x,
                     const float* gy, int nbatch, int D, int H, int W, float* grad, void* ws, size_t ws_bytes,
                     void* stream) {
    Net N;
    NN_TRY(make_net(cfg, N));
    NN_TRY(check_net_dims(nbatch, D, H, W));
    NN_TRY(check_ptr(params, "params", 4));
    NN_TRY(check_ptr(frag, "frag", 8));
    NN_TRY(check_ptr(x, "x", 8));
    NN_TRY(check_ptr(gy, "gy", 4));
    NN_TRY(check_ptr(grad, "grad", 4));
    NN_TRY(check_ptr(ws, "ws", 256));
    Acts A;
    layout(N, nbatch, D, H, W, 1, static_cast<char*>(ws), A);
    if (ws_bytes < A.bytes) return fail(TT_EINVAL, "workspace too small: %zu < %zu", ws_bytes, A.bytes);
    return unet_backward(N, params, frag, gy, x, nbatch, D, H, W, grad, A, S(stream));
}

int nn_warm_features(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
                     const double* src_pos, const double* src_par, int32_t stride, int32_t D, int32_t H, int32_t W,
                     uint16_t* feat, void* stream) {
    WarmGrid G;
    NN_TRY(warm_grid(grid, G));
    if (nsrc < 1 || nsrc > 65535) return fail(TT_EINVAL, "nsrc must be in [1, 65535]");
    NN_TRY(check_coarse(grid, stride, D, H, W));
    NN_TRY(check_ptr(s, "s", 8));
    NN_TRY(check_ptr(xi, "xi", 8));
    NN_TRY(check_ptr(eta, "eta", 8));
    NN_TRY(check_ptr(src_pos, "src_pos", 8));
    NN_TRY(check_ptr(src_par, "src_par", 8));
    NN_TRY(check_ptr(feat, "feat", 8));
    const long long npos = (long long)D * H * W;
    unsigned bx = blocks_of(npos, 256);
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(k_warm_features, dim3(bx, nsrc), dim3(256), 0, S(stream), G, s, xi, eta, src_pos, src_par,
                       stride, D, H, W, feat);
    NN_LAUNCHED();
    return TT_OK;
}

int nn_warm_target(const tt_grid* grid, int32_t nsrc, const double* tau, int32_t stride, int32_t D, int32_t H,
                   int32_t W, float* target, float* mask, void* stream) {
    WarmGrid G;
    NN_TRY(warm_grid(grid, G));
    if (nsrc < 1 || nsrc > 65535) return fail(TT_EINVAL, "nsrc must be in [1, 65535]");
    NN_TRY(check_coarse(grid, stride, D, H, W));
    NN_TRY(check_ptr(tau, "tau", 8));
    NN_TRY(check_ptr(target, "target", 4));
    const long long npos = (long long)D * H * W;
    unsigned bx = blocks_of(npos, 256);
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(k_warm_target, dim3(bx, nsrc), dim3(256), 0, S(stream), G, tau, stride, D, H, W, target, mask);
    NN_LAUNCHED();
    return TT_OK;
}

int nn_warm_init(const tt_grid* grid, int32_t nsrc, const float* pred, int32_t stride, int32_t D, int32_t H, int32_t W,
                 double* tau_init, void* stream) {
    WarmGrid G;
    NN_TRY(warm_grid(grid, G));
    if (nsrc < 1 || nsrc > 65535) return fail(TT_EINVAL, "nsrc must be in [1, 65535]");
    NN_TRY(check_coarse(grid, stride, D, H, W));
    NN_TRY(check_ptr(pred, "pred", 4));
    NN_TRY(check_ptr(tau_init, "tau_init", 8));
    const long long N = (long long)G.n[0] * G.n[1] * G.n[2];
    unsigned bx = blocks_of(N, 256);
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(k_warm_init, dim3(bx, nsrc), dim3(256), 0, S(stream), G, pred, stride, D, H, W, tau_init);
    NN_LAUNCHED();
    return TT_OK;
}

}  // extern "C"

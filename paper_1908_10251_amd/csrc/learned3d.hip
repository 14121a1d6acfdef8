// Learned convolutional smoother for the 3D constant-coefficient levels:
// inference inside the V-cycle and training on residuals of plain V-cycles.
//
// The smoothing step is x <- x + N(rho), rho = (f - A x) / D, with
//   z1[c](v) = sum_t W1[c][t] rho(v + t),  h = max(z1, 0) (zero off the
//   interior), N(rho)(v) = sum_{c,t} W2[c][t] h[c](v + t),
// t over the 27 offsets {-1,0,1}^3 (index (dz+1)*9 + (dy+1)*3 + (dx+1)) and
// c over 16 channels.  Both contractions run on the matrix cores as bfloat16
// products with FP32 accumulation (v_mfma_f32_16x16x16_bf16); rho, h and the
// weights are rounded to bfloat16 (nearest even) where they enter them.
//
// Matrix-core operand layout (16x16x16, one wavefront): lane l holds
//   A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16], D[4 (l / 16) + j][l % 16]
// for j = 0..3.
//
// Inference (k_learned_step): a workgroup owns a 16 x 16 column of output
// nodes and marches in z.  Per z slice it loads x with a halo of 3 and f with
// a halo of 2 (one slice ahead, in registers), forms rho on 20 x 20 nodes
// (each thread keeps the last two rho values of its nodes, so it writes the
// z triplet of the slice below as one 8-byte word), the hidden layer on
// 18 x 18 nodes (layer 1: M = channels, K = z triplets of the 9 in-plane
// offsets, N = nodes; its result stays in registers as the next operand),
// then Y[u][t] = sum_c h[u][c] W2[c][t] (layer 2: M = nodes, K = channels,
// N = taps), and gathers N(rho)(v) = sum_t Y[v + t][t] into three running
// output sums held in registers.
//
// Training: loss L = (1/S) sum_s ||r_s - A N(rho_s)||^2 / ||r_s||^2 over
// residual samples; the backward contractions (hidden gradient: M = nodes,
// K = taps, N = channels; weight gradients: M = channels, K = nodes, N = taps)
// run on the matrix cores as well.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace pasm {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline unsigned short f2bf(float f) {
    unsigned u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

// Round-to-nearest-even bfloat16 of two floats in one hardware conversion
// (bits of a in the low half); the same rounding as f2bf for finite values.
__device__ inline unsigned bf16_pair(float a, float b) {
    typedef __bf16 bfv2 __attribute__((ext_vector_type(2)));
    typedef float fv2 __attribute__((ext_vector_type(2)));
    const fv2 v = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bfv2));
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// 16 x 16 x 32: lane l holds A[l % 16][k], B[k][l % 16] for the eight K
// slots of lane group l / 16 (the same slots pair in the product) and D as
// in the 16 x 16 x 16 form.
__device__ inline f32x4 mfma32(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline bf16x8 join8(const bf16x4& lo, const bf16x4& hi) {
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2 w = {__builtin_bit_cast(unsigned long long, lo), __builtin_bit_cast(unsigned long long, hi)};
    return __builtin_bit_cast(bf16x8, w);
}
__device__ inline f32x4 mfma(const bf16x4& a, const bf16x4& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__host__ __device__ inline void tap_off(int t, int& dx, int& dy, int& dz) {
    dx = t % 3 - 1;
    dy = (t / 3) % 3 - 1;
    dz = t / 9 - 1;
}

// ---------------------------------------------------------------------------
// fused inference step
// ---------------------------------------------------------------------------
constexpr int OT = 16;            // output tile edge (x, y)
constexpr int XT = OT + 6;        // x tile edge (halo 3)
constexpr int RT = OT + 4;        // rho tile edge (halo 2)
constexpr int HT = OT + 2;        // hidden tile edge (halo 1)
constexpr int HN = HT * HT;       // hidden nodes per slice (324)
constexpr int HB = (HN + 15) / 16;  // 16-node blocks (21)
constexpr int XRING = 5;          // x slices kept in LDS
constexpr int LT = 256;           // threads per workgroup

// ops (learned_pack_step, 64-bit words): [0, 256) layer-1 operand (2 K-steps
// x 64 lanes x 2 words, the A operand, M = channels), [256, 512) layer-2
// operand (2 K-steps x 64 lanes x 2 words, the B operand).
//
// Both layers run on the 16 x 16 x 32 bfloat16 product.  Layer 1 is
// D[c][v] = sum_k W1'[c][k] P[k][v]: the eight K slots of lane group g in
// K-step s are two groups G = 8 s + 2 g + w (w = 0, 1) of four, group G < 9
// being the in-plane offset (dx, dy) = (G % 3 - 1, G / 3 - 1) and slot jz < 3
// of the group the z offset jz - 1.  So the four values a lane feeds per
// group are one 8-byte word of the "z triplet" tile (rho at z - 1, z, z + 1
// and a zero).  D holds in lane l channels 4 (l / 16) + j of node l % 16: an
// 8-byte word of the hidden tile.
//
// Layer 2 contracts over the x offsets and the channels:
// E[u][col] = sum over dx and channels c of h[u + dx][c] W2[c][3 col + dx + 1]
// for the nine columns col = 3 (dz + 1) + (dy + 1), evaluated on 16-node rows
// u of the hidden tile (18 rows).  Lane group g of K-step s covers x offset
// 2 s + g / 2 - 1 and channels 8 (g % 2) .. + 7: one 16-byte word of the
// hidden tile.  N(rho) at output node v then gathers the nine values
// E[v + (0, dy)][col] of each hidden slice, column (dz, dy) of hidden slice p
// belonging to output slice p - dz.
template <typename T>
__global__ __launch_bounds__(LT, 4) void k_learned_step(Grid g, T w0, const T* __restrict__ x, const T* __restrict__ f,
                                                        T* __restrict__ out, long stride,
                                                        const unsigned long long* __restrict__ ops, int zseg,
                                                        int x_zero) {
    __shared__ T xs[XRING][XT * XT];  // x slices, ring of 5
    __shared__ T fs[RT * RT];         // f slice of the rho tile
    __shared__ bf16x4 tri[RT * RT];   // rho z triplets around the hidden slice
    // hidden slice: [channel half][node], 8 channels in a 16-byte word
    constexpr int HSTR = HB * 16;
    __shared__ bf16x8 hs[2 * HSTR];
    // layer-2 result of the hidden slice: [column][hidden row][x], the column
    // stride padded so that the nine columns a lane group writes spread over
    // the banks
    constexpr int ER = HT, EC = 9, ES = ER * OT + 4;
    __shared__ __attribute__((aligned(16))) float es[EC * ES];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int tiles = (g.m + OT - 1) / OT;
    const int bx = blockIdx.x % tiles, by = blockIdx.x / tiles;
    const int z0 = 1 + blockIdx.y * zseg, z1 = min(g.m + 1, z0 + zseg);  // output slices [z0, z1)
    const long off = (long)blockIdx.z * stride;
    const T* xr = x + off;
    const T* fr = f + off;
    T* outr = out + off;
    const int i0 = bx * OT + 1, j0 = by * OT + 1;  // first output node (interior indices from 1)
    const T invD = T(1) / (T(6) * w0);
    // offsets inside one right-hand side stay below 2^31 (32-bit arithmetic)
    const int zst = (g.n + 1) * g.pitch;  // z stride of the padded layout

    bf16x8 w1[2], w2[2];
    {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
        const u64x2* o2 = reinterpret_cast<const u64x2*>(ops);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            w1[s] = __builtin_bit_cast(bf16x8, o2[s * 64 + lane]);
            w2[s] = __builtin_bit_cast(bf16x8, o2[128 + s * 64 + lane]);
        }
    }
    // layer 1: this lane's triplet offsets for its four K groups
    // G = 8 s + 2 grp + w (groups >= 9 read zeros), and per hidden block
    // (blk = wave + 4 k) its node's triplet base; bit k of hmask says whether
    // that node is interior in x and y
    int toff[4];
#pragma unroll
    for (int sw = 0; sw < 4; ++sw) {
        const int G = min(8 * (sw >> 1) + 2 * grp + (sw & 1), 8);
        toff[sw] = (G / 3) * RT + (G % 3);  // (1 + dy) RT + (1 + dx)
    }
    constexpr int HK = (HB + 3) / 4;  // hidden blocks per wave (the last only for wave 0)
    int tb[HK];
    unsigned hmask = 0;
#pragma unroll
    for (int k = 0; k < HK; ++k) {
        const int v = (wave + 4 * k) * 16 + col;
        const int vc = v < HN ? v : HN - 1;
        const int hx = vc % HT, hy = vc / HT;
        const int i = i0 - 1 + hx, j = j0 - 1 + hy;
        tb[k] = hy * RT + hx;
        if (v < HN && i >= 1 && i <= g.m && j >= 1 && j <= g.m) hmask |= 1u << k;
    }
    constexpr int EK = (ER + 3) / 4;  // layer-2 rows per wave (row wave + 4 k < 18)

    // Global loads run one slice ahead in registers (px, pf), so their
    // latency overlaps the previous slice's work instead of stalling it.
    // They are unconditional, from clamped addresses inside the field, and
    // the values off the tile's valid nodes are replaced by zeros when they
    // enter LDS: no load sits in a branch, so the wait for them can stay at
    // the top of the next iteration.
    constexpr int XPT = (XT * XT + LT - 1) / LT, FPT = (RT * RT + LT - 1) / LT;
    static_assert(FPT == 2, "two rho nodes per thread");
    const T* xsrc = x_zero ? fr : xr;  // x == 0: loads are discarded
    int xoff[XPT], foff[FPT];
    unsigned okmask = 0;  // bit e: x node e valid; bit 8 + e: f node e interior; bit 16: output node interior
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
        const int t = tid + e * LT;
        const int i = i0 - 3 + t % XT, j = j0 - 3 + t / XT;
        if (t < XT * XT && i >= 0 && i <= g.n && j >= 0 && j <= g.n) okmask |= 1u << e;
        xoff[e] = (int)g.idx(min(max(i, 0), g.n), min(max(j, 0), g.n), 0);
    }
#pragma unroll
    for (int e = 0; e < FPT; ++e) {
        const int t = tid + e * LT;
        const int i = i0 - 2 + t % RT, j = j0 - 2 + t / RT;
        if (t < RT * RT && i >= 1 && i <= g.m && j >= 1 && j <= g.m) okmask |= 1u << (8 + e);
        foff[e] = (int)g.idx(min(max(i, 0), g.n), min(max(j, 0), g.n), 0);
    }
    const int ox = tid % OT, oy = tid / OT;  // this thread's output node (LT == OT * OT)
    if (i0 + ox <= g.m && j0 + oy <= g.m) okmask |= 1u << 16;
    const int ooff = (int)g.idx(min(i0 + ox, g.m), min(j0 + oy, g.m), 0);
    T px[XPT], pf[FPT];
    auto fetch_x = [&](int l) {  // x slice l (grid node index)
        const int zo = min(max(l, 0), g.n) * zst;
#pragma unroll
        for (int e = 0; e < XPT; ++e) px[e] = xsrc[(unsigned)(zo + xoff[e])];
    };
    auto fetch_f = [&](int l) {  // f slice l on the rho tile
        const int zo = min(max(l, 0), g.n) * zst;
#pragma unroll
        for (int e = 0; e < FPT; ++e) pf[e] = fr[(unsigned)(zo + foff[e])];
    };
    auto slot = [](int l) { return (l + 2 * XRING) % XRING; };  // l >= -4
    auto put_x = [&](int l) {
        const bool lok = !x_zero && l >= 0 && l <= g.n;
        T* d = xs[slot(l)];
#pragma unroll
        for (int e = 0; e < XPT; ++e)
            if (tid + e * LT < XT * XT) d[tid + e * LT] = (lok && ((okmask >> e) & 1u)) ? px[e] : T(0);
    };
    auto put_f = [&](int l) {
        const bool lok = l >= 1 && l <= g.m;
#pragma unroll
        for (int e = 0; e < FPT; ++e)
            if (tid + e * LT < RT * RT) fs[tid + e * LT] = (lok && ((okmask >> (8 + e)) & 1u)) ? pf[e] : T(0);
    };
    fetch_x(z0 - 3);
    put_x(z0 - 3);
    fetch_x(z0 - 2);
    put_x(z0 - 2);
    fetch_x(z0 - 1);
    fetch_f(z0 - 2);
    unsigned short r1[FPT], r2[FPT];  // bf16 rho of this thread's rho nodes, slices q - 1, q - 2
#pragma unroll
    for (int e = 0; e < FPT; ++e) r1[e] = r2[e] = 0;
    float cm1 = 0.f, c0 = 0.f, cp1 = 0.f;  // running sums of output slices pg - 1, pg, pg + 1
    const float* ebase = es + (oy + 1) * OT + ox;
    // Iteration q: rho of slice q, both layers of hidden slice q - 1 (E to
    // LDS), and the gather of hidden slice q - 2's E, which completes output
    // slice q - 3.
    for (int q = z0 - 2; q <= z1 + 2; ++q) {
        // 1. slices fetched during the previous iteration enter LDS; fetch the next
        put_x(q + 1);
        put_f(q);
        fetch_x(q + 2);
        fetch_f(q + 1);
        __syncthreads();
        // 2. gather E of hidden slice pg = q - 2; output slice pg - 1 is complete
        const int pg = q - 2;
        if (pg >= z0 - 1 && pg <= z1) {  // uniform
#pragma unroll
            for (int cz = 0; cz < EC; ++cz) {
                const int dz = cz / 3 - 1, dy = cz % 3 - 1;
                const float v = ebase[cz * ES + dy * OT];
                if (dz == 1) cm1 += v;
                else if (dz == 0) c0 += v;
                else cp1 += v;
            }
            const int o = pg - 1;
            if (o >= z0 && o < z1 && ((okmask >> 16) & 1u))
                outr[(unsigned)(o * zst + ooff)] = xs[slot(o)][(oy + 3) * XT + ox + 3] + (T)cm1;
            cm1 = c0;
            c0 = cp1;
            cp1 = 0.f;
        }
        // 3. rho slice q on this thread's nodes (zero off the interior); the z
        // triplet centred on slice q - 1 goes to LDS
        {
            const T* xc = xs[slot(q)];
            const T* xq = xs[slot(q - 1)];
            const T* xp = xs[slot(q + 1)];
            float rv[2] = {0.f, 0.f};
#pragma unroll
            for (int e = 0; e < FPT; ++e) {
                const int t = tid + e * LT;
                const int a = t % RT, b = t / RT;
                if (t < RT * RT && q >= 1 && q <= g.m && ((okmask >> (8 + e)) & 1u)) {
                    const int pp = (b + 1) * XT + (a + 1);
                    const T Ax =
                        w0 * (T(6) * xc[pp] - xc[pp - 1] - xc[pp + 1] - xc[pp - XT] - xc[pp + XT] - xq[pp] - xp[pp]);
                    rv[e] = (float)((fs[t] - Ax) * invD);
                }
            }
            const unsigned rp = bf16_pair(rv[0], rv[1]);
#pragma unroll
            for (int e = 0; e < FPT; ++e) {
                const int t = tid + e * LT;
                const unsigned short rq = (unsigned short)(rp >> (16 * e));
                if (t < RT * RT) {
                    bf16x4 w;
                    w[0] = (short)r2[e];
                    w[1] = (short)r1[e];
                    w[2] = (short)rq;
                    w[3] = 0;
                    tri[t] = w;
                }
                r2[e] = r1[e];
                r1[e] = rq;
            }
        }
        __syncthreads();
        const int p = q - 1;  // hidden slice
        if (p < z0 - 1 || p > z1) continue;  // feeds no output slice of this workgroup (uniform)
        // 4. hidden slice p: layer 1, ReLU, zero off the interior, to LDS
        // (the blocks' product chains interleave)
        {
            const bool pin = p >= 1 && p <= g.m;
            const int nhk = wave == 0 ? HK : HK - 1;  // blocks of this wave (uniform)
            f32x4 c[HK];
#pragma unroll
            for (int k = 0; k < HK; ++k) c[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int k = 0; k < HK; ++k)
                    if (k < nhk) {
                        // step 1 holds only group 8 (lane group 0, first
                        // word); the other lanes skip the LDS read
                        bf16x4 b0 = {0, 0, 0, 0}, b1 = {0, 0, 0, 0};
                        if (s == 0 || grp == 0) b0 = tri[tb[k] + toff[2 * s]];
                        if (s == 0) b1 = tri[tb[k] + toff[2 * s + 1]];
                        c[k] = mfma32(w1[s], join8(b0, b1), c[k]);
                    }
            bf16x4* hw = reinterpret_cast<bf16x4*>(hs);
#pragma unroll
            for (int k = 0; k < HK; ++k)
                if (k < nhk) {
                    // ReLU on the rounded values (a negative bfloat16 is a
                    // negative 16-bit integer), then the interior mask
                    typedef short sv2 __attribute__((ext_vector_type(2)));
                    typedef unsigned uv2 __attribute__((ext_vector_type(2)));
                    const sv2 zero2 = {0, 0};
                    const unsigned keep = (pin && ((hmask >> k) & 1u)) ? ~0u : 0u;
                    const sv2 lo = __builtin_elementwise_max(
                        __builtin_bit_cast(sv2, bf16_pair(c[k][0], c[k][1])), zero2);
                    const sv2 hi = __builtin_elementwise_max(
                        __builtin_bit_cast(sv2, bf16_pair(c[k][2], c[k][3])), zero2);
                    const uv2 w = {__builtin_bit_cast(unsigned, lo) & keep, __builtin_bit_cast(unsigned, hi) & keep};
                    hw[((grp >> 1) * HSTR + (wave + 4 * k) * 16 + col) * 2 + (grp & 1)] = __builtin_bit_cast(bf16x4, w);
                }
        }
        __syncthreads();
        // 5. layer 2 on hidden rows r = wave + 4 k (chains interleaved), E to LDS
        {
            const int nek = wave < ER - 4 * (EK - 1) ? EK : EK - 1;  // rows of this wave (uniform)
            f32x4 e[EK];
#pragma unroll
            for (int k = 0; k < EK; ++k) e[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int dx = 2 * s + (grp >> 1) - 1;  // x offset of this lane group (2 in step 1 reads zeros)
                const bf16x8* hp = hs + (grp & 1) * HSTR + wave * HT + col + 1 + min(dx, 1);
#pragma unroll
                for (int k = 0; k < EK; ++k)
                    if (k < nek) {
                        bf16x8 a = {};
                        if (s == 0 || (grp >> 1) == 0) a = hp[4 * k * HT];  // x offset 2 does not exist
                        e[k] = mfma32(a, w2[s], e[k]);
                    }
            }
#pragma unroll
            for (int k = 0; k < EK; ++k)
                if (k < nek && col < EC)
                    *reinterpret_cast<f32x4*>(&es[col * ES + (wave + 4 * k) * OT + 4 * grp]) = e[k];
        }
    }
}

// ---------------------------------------------------------------------------
// training kernels (FP32 fields on an m^3 interior grid, S samples;
// "padded" arrays have one zero node around the interior)
// ---------------------------------------------------------------------------
struct TGrid {
    int m, mp;       // interior edge, padded edge m + 2
    long vol, pvol;  // m^3, (m + 2)^3
    __host__ __device__ inline long pidx(int x, int y, int z) const {
        return ((long)(z + 1) * mp + (y + 1)) * mp + (x + 1);
    }
};

__device__ inline void vox(const TGrid& tg, long u, int& x, int& y, int& z) {
    x = (int)(u % tg.m);
    y = (int)((u / tg.m) % tg.m);
    z = (int)(u / ((long)tg.m * tg.m));
}

// rho = r / D rounded (padded), and ||r||^2 per sample (block partials)
__global__ __launch_bounds__(256) void k_lt_rho(TGrid tg, const float* __restrict__ r, float invD,
                                                unsigned short* __restrict__ rho_p, float* __restrict__ nr_part) {
    __shared__ float sh[4];
    const int s = blockIdx.y;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    float q = 0.f;
    if (u < tg.vol) {
        int x, y, z;
        vox(tg, u, x, y, z);
        const float v = r[s * tg.vol + u];
        rho_p[s * tg.pvol + tg.pidx(x, y, z)] = f2bf(v * invD);
        q = v * v;
    }
    for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) nr_part[(long)s * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// out[u][c] = sum_t src(u + sgn * t) W[c][t] over 16-node blocks of all
// samples (M = nodes, K = taps, N = channels).  Mode 0 (layer 1): stores z1
// and h = bf16(relu) padded.  Mode 1 (hidden gradient): multiplies by the
// ReLU mask of z1 and stores bf16 unpadded.
template <int MODE>
__global__ __launch_bounds__(256) void k_lt_tapconv(TGrid tg, int S, const unsigned short* __restrict__ src_p,
                                                    const unsigned long long* __restrict__ wop, int sgn,
                                                    float* __restrict__ z1, unsigned short* __restrict__ outb) {
    const int lane = threadIdx.x & 63;
    const long nblk = (tg.vol * S + 15) / 16;
    const long blk = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk >= nblk) return;
    bf16x4 b[2];
    for (int ks = 0; ks < 2; ++ks) {
        const unsigned long long w = wop[ks * 64 + lane];
        __builtin_memcpy(&b[ks], &w, 8);
    }
    const long gu = blk * 16 + (lane & 15);
    const bool valid = gu < tg.vol * S;
    const int s = valid ? (int)(gu / tg.vol) : 0;
    int x = 0, y = 0, z = 0;
    if (valid) vox(tg, gu - (long)s * tg.vol, x, y, z);
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        bf16x4 a;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int t = ks * 16 + 4 * (lane >> 4) + jj;
            unsigned short val = 0;
            if (t < 27 && valid) {
                int dx, dy, dz;
                tap_off(t, dx, dy, dz);
                val = src_p[(long)s * tg.pvol + tg.pidx(x + sgn * dx, y + sgn * dy, z + sgn * dz)];
            }
            a[jj] = (short)val;
        }
        c = mfma(a, b[ks], c);
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const long ou = blk * 16 + 4 * (lane >> 4) + jj;
        if (ou >= tg.vol * S) continue;
        const int ch = lane & 15;
        const int os = (int)(ou / tg.vol);
        const long lu = ou - (long)os * tg.vol;
        if (MODE == 0) {
            z1[ou * 16 + ch] = c[jj];
            int ox, oy, oz;
            vox(tg, lu, ox, oy, oz);
            outb[((long)os * tg.pvol + tg.pidx(ox, oy, oz)) * 16 + ch] = f2bf(fmaxf(c[jj], 0.f));
        } else {
            const float v = z1[ou * 16 + ch] > 0.f ? c[jj] : 0.f;
            outb[ou * 16 + ch] = f2bf(v);
        }
    }
}

// Y[u][t] = sum_c h[u][c] W2[c][t] (M = nodes, K = channels, N = taps),
// stored padded [pvol][32] so the gather needs no bounds checks
__global__ __launch_bounds__(256) void k_lt_y(TGrid tg, int S, const unsigned short* __restrict__ h_p,
                                              const unsigned long long* __restrict__ wop, float* __restrict__ y_p) {
    const int lane = threadIdx.x & 63;
    const long nblk = (tg.vol * S + 15) / 16;
    const long blk = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk >= nblk) return;
    const long gu = blk * 16 + (lane & 15);
    const bool valid = gu < tg.vol * S;
    const int s = valid ? (int)(gu / tg.vol) : 0;
    int x = 0, y = 0, z = 0;
    if (valid) vox(tg, gu - (long)s * tg.vol, x, y, z);
    bf16x4 a;
    const long hb = ((long)s * tg.pvol + tg.pidx(x, y, z)) * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) a[jj] = valid ? (short)h_p[hb + jj] : (short)0;
    for (int nb = 0; nb < 2; ++nb) {
        bf16x4 b;
        const unsigned long long w = wop[nb * 64 + lane];
        __builtin_memcpy(&b, &w, 8);
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma(a, b, c);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const long ou = blk * 16 + 4 * (lane >> 4) + jj;
            if (ou >= tg.vol * S) continue;
            const int os = (int)(ou / tg.vol);
            int ox, oy, oz;
            vox(tg, ou - (long)os * tg.vol, ox, oy, oz);
            y_p[((long)os * tg.pvol + tg.pidx(ox, oy, oz)) * 32 + nb * 16 + (lane & 15)] = c[jj];
        }
    }
}

// delta(v) = sum_t Y[v + t][t] (padded output)
__global__ __launch_bounds__(256) void k_lt_delta(TGrid tg, const float* __restrict__ y_p, float* __restrict__ d_p) {
    const int s = blockIdx.y;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    if (u >= tg.vol) return;
    int x, y, z;
    vox(tg, u, x, y, z);
    const float* yb = y_p + (long)s * tg.pvol * 32;
    float acc = 0.f;
    for (int t = 0; t < 27; ++t) {
        int dx, dy, dz;
        tap_off(t, dx, dy, dz);
        acc += yb[tg.pidx(x + dx, y + dy, z + dz) * 32 + t];
    }
    d_p[(long)s * tg.pvol + tg.pidx(x, y, z)] = acc;
}

__device__ inline float lap7(const TGrid& tg, const float* a, long p, float w0) {
    const long sy = tg.mp, sz = (long)tg.mp * tg.mp;
    return w0 * (6.f * a[p] - a[p - 1] - a[p + 1] - a[p - sy] - a[p + sy] - a[p - sz] - a[p + sz]);
}

// res = r - A delta (padded), and block partials of res^2 per sample
__global__ __launch_bounds__(256) void k_lt_res(TGrid tg, const float* __restrict__ r, const float* __restrict__ d_p,
                                                float w0, float* __restrict__ res_p, float* __restrict__ part) {
    __shared__ float sh[4];
    const int s = blockIdx.y;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    float q = 0.f;
    if (u < tg.vol) {
        int x, y, z;
        vox(tg, u, x, y, z);
        const long p = tg.pidx(x, y, z);
        const float v = r[s * tg.vol + u] - lap7(tg, d_p + (long)s * tg.pvol, p, w0);
        res_p[(long)s * tg.pvol + p] = v;
        q = v * v;
    }
    for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) part[(long)s * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// g = coef[s] * A res, rounded (padded)
__global__ __launch_bounds__(256) void k_lt_g(TGrid tg, const float* __restrict__ res_p, const float* __restrict__ coef,
                                              float w0, unsigned short* __restrict__ g_p) {
    const int s = blockIdx.y;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    if (u >= tg.vol) return;
    int x, y, z;
    vox(tg, u, x, y, z);
    const long p = tg.pidx(x, y, z);
    g_p[(long)s * tg.pvol + p] = f2bf(coef[s] * lap7(tg, res_p + (long)s * tg.pvol, p, w0));
}

// dW[c][t] = sum_u X[u][c] src(u + sgn t) (M = channels, K = nodes, N = taps),
// one partial [16][32] per workgroup; X is padded (layer-2 gradient: h) or
// not (layer-1 gradient: hidden gradient)
template <bool XPAD>
__global__ __launch_bounds__(256) void k_lt_dw(TGrid tg, int S, const unsigned short* __restrict__ X,
                                               const unsigned short* __restrict__ src_p, int sgn,
                                               float* __restrict__ part, int kblocks_per_wave) {
    __shared__ float red[4][16 * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long nk = (tg.vol * S + 15) / 16;
    f32x4 c[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    const long kb0 = ((long)blockIdx.x * 4 + wave) * kblocks_per_wave;
    for (long kb = kb0; kb < kb0 + kblocks_per_wave && kb < nk; ++kb) {
        bf16x4 a, b[2];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const long gu = kb * 16 + 4 * (lane >> 4) + jj;  // node of K row 4 (lane / 16) + jj
            unsigned short av = 0, bv0 = 0, bv1 = 0;
            if (gu < tg.vol * S) {
                const int s = (int)(gu / tg.vol);
                int x, y, z;
                vox(tg, gu - (long)s * tg.vol, x, y, z);
                const int ch = lane & 15;
                av = XPAD ? X[((long)s * tg.pvol + tg.pidx(x, y, z)) * 16 + ch] : X[gu * 16 + ch];
                const int t0 = lane & 15, t1 = 16 + (lane & 15);
                int dx, dy, dz;
                tap_off(t0, dx, dy, dz);
                bv0 = src_p[(long)s * tg.pvol + tg.pidx(x + sgn * dx, y + sgn * dy, z + sgn * dz)];
                if (t1 < 27) {
                    tap_off(t1, dx, dy, dz);
                    bv1 = src_p[(long)s * tg.pvol + tg.pidx(x + sgn * dx, y + sgn * dy, z + sgn * dz)];
                }
            }
            // A[c][k]: lane holds row c = lane % 16, columns 4 (lane / 16) + jj:
            // X at node k for channel c -- the same (node, channel) pairs as above
            a[jj] = (short)av;
            b[0][jj] = (short)bv0;
            b[1][jj] = (short)bv1;
        }
        c[0] = mfma(a, b[0], c[0]);
        c[1] = mfma(a, b[1], c[1]);
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) red[wave][(4 * (lane >> 4) + jj) * 32 + nb * 16 + (lane & 15)] = c[nb][jj];
    __syncthreads();
    for (int t = threadIdx.x; t < 16 * 32; t += 256)
        part[(long)blockIdx.x * 512 + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// fixed-order sums of nparts partials of n floats
__global__ __launch_bounds__(256) void k_lt_sum(const float* __restrict__ part, int nparts, int n,
                                                double* __restrict__ out) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(long)p * n + t];
    out[t] = s;
}

__global__ void k_lt_zero_u16(unsigned short* p, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) p[t] = 0;
}
__global__ void k_lt_zero_f(float* p, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) p[t] = 0.f;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Operand words of the inference step (kLearnedStepOps, 8 bfloat16 per lane
// and K-step as two 64-bit words): layer 1 as the A operand of
// (channels x K) x (K x nodes), lane group g of K-step s holding groups
// G = 8 s + 2 g + w, slot jz < 3 of group G < 9 being tap 9 jz + G (the rest
// zero); then layer 2 as the B operand of (nodes x K) x (K x columns), lane
// group g of K-step s holding x offset index dxi = 2 s + g / 2 (< 3) and
// channels 8 (g % 2) .. + 7, column col < 9 being tap 3 col + dxi.
void learned_pack_step(const float* W, unsigned long long* out) {
    for (int s = 0; s < 2; ++s)
        for (int lane = 0; lane < 64; ++lane) {
            unsigned short v[8];
            const int c = lane % 16, gq = lane / 16;
            for (int w = 0; w < 2; ++w) {
                const int G = 8 * s + 2 * gq + w;
                for (int jz = 0; jz < 4; ++jz) v[4 * w + jz] = (G < 9 && jz < 3) ? f2bf(W[c * 27 + 9 * jz + G]) : 0;
            }
            __builtin_memcpy(&out[(s * 64 + lane) * 2], v, 16);
        }
    const float* W2 = W + 16 * 27;
    for (int s = 0; s < 2; ++s)
        for (int lane = 0; lane < 64; ++lane) {
            unsigned short v[8];
            const int cl = lane % 16, gq = lane / 16;
            const int dxi = 2 * s + gq / 2;
            for (int j = 0; j < 8; ++j) {
                const int c = 8 * (gq % 2) + j;
                v[j] = (cl < 9 && dxi < 3) ? f2bf(W2[c * 27 + 3 * cl + dxi]) : 0;
            }
            __builtin_memcpy(&out[256 + (s * 64 + lane) * 2], v, 16);
        }
}

// Operand words (4 bfloat16 per 64-bit word, lane order) of a [16][27]
// weight array as the B operand of a (nodes x taps) x (taps x channels)
// product: B[t][c] = W[c][t], K-steps of 16 taps (taps >= 27 are zero).
void learned_pack_taps_by_channel(const float* W, unsigned long long* out) {
    for (int ks = 0; ks < 2; ++ks)
        for (int lane = 0; lane < 64; ++lane) {
            unsigned short v[4];
            for (int j = 0; j < 4; ++j) {
                const int t = ks * 16 + 4 * (lane / 16) + j, c = lane % 16;
                v[j] = t < 27 ? f2bf(W[c * 27 + t]) : 0;
            }
            __builtin_memcpy(&out[ks * 64 + lane], v, 8);
        }
}
// ... as the B operand of a (nodes x channels) x (channels x taps) product:
// B[c][t] = W[c][t], N-blocks of 16 taps.
void learned_pack_channels_by_tap(const float* W, unsigned long long* out) {
    for (int nb = 0; nb < 2; ++nb)
        for (int lane = 0; lane < 64; ++lane) {
            unsigned short v[4];
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * (lane / 16) + j, t = nb * 16 + lane % 16;
                v[j] = t < 27 ? f2bf(W[c * 27 + t]) : 0;
            }
            __builtin_memcpy(&out[nb * 64 + lane], v, 8);
        }
}

constexpr int kLearnedZseg = 32;

template <typename T>
void launch_learned_step(const Grid& g, T w0, const T* x, const T* f, T* out, int nrhs, long stride,
                         const unsigned long long* ops, bool x_zero, hipStream_t st) {
    if (g.dim != 3) throw Error(PASM_E_INVALID, "learned smoother: 3D levels only");
    const int tiles = (g.m + OT - 1) / OT;
    dim3 grid(tiles * tiles, (g.m + kLearnedZseg - 1) / kLearnedZseg, nrhs);
    hipLaunchKernelGGL((k_learned_step<T>), grid, dim3(LT), 0, st, g, w0, x, f, out, stride, ops, kLearnedZseg,
                       (int)x_zero);
    PASM_CHECK_LAUNCH();
}
template void launch_learned_step<float>(const Grid&, float, const float*, const float*, float*, int, long,
                                         const unsigned long long*, bool, hipStream_t);
template void launch_learned_step<double>(const Grid&, double, const double*, const double*, double*, int, long,
                                          const unsigned long long*, bool, hipStream_t);

// ---------------------------------------------------------------------------
// residual norms, random fields and sample packing (3D levels)
// ---------------------------------------------------------------------------
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_resid_norm3(Grid g, T w0, const T* __restrict__ x, const T* __restrict__ f,
                                                     long stride, double* __restrict__ partial) {
    __shared__ double sh[8];
    const long n = (long)g.m * g.m * g.m;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    const long off = (long)blockIdx.y * stride;
    double q = 0.0, qf = 0.0;
    if (u < n) {
        const int i = (int)(u % g.m) + 1, j = (int)((u / g.m) % g.m) + 1, l = (int)(u / ((long)g.m * g.m)) + 1;
        const long id = off + g.idx(i, j, l);
        const long sy = g.pitch, sz = (long)(g.n + 1) * g.pitch;
        const double Ax = (double)w0 * (6.0 * (double)x[id] - (double)x[id - 1] - (double)x[id + 1] -
                                        (double)x[id - sy] - (double)x[id + sy] - (double)x[id - sz] - (double)x[id + sz]);
        const double r = (double)f[id] - Ax;
        q = r * r;
        qf = (double)f[id] * (double)f[id];
    }
    for (int o = 32; o > 0; o >>= 1) {
        q += __shfl_down(q, o, 64);
        qf += __shfl_down(qf, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = q;
        sh[4 + (threadIdx.x >> 6)] = qf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * b] = sh[0] + sh[1] + sh[2] + sh[3];
        partial[2 * b + 1] = sh[4] + sh[5] + sh[6] + sh[7];
    }
}

// standard normal values on the interior nodes (splitmix64 + Box-Muller)
__device__ inline unsigned long long splitmix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
template <typename T>
__global__ __launch_bounds__(256) void k_fill_normal3(Grid g, T* __restrict__ x, long stride, unsigned long long seed) {
    const long n = (long)g.m * g.m * g.m;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    if (u >= n) return;
    const int i = (int)(u % g.m) + 1, j = (int)((u / g.m) % g.m) + 1, l = (int)(u / ((long)g.m * g.m)) + 1;
    const unsigned long long key = seed * 0x100000001B3ull + (unsigned long long)blockIdx.y * n + u;
    const unsigned long long a = splitmix64(key), b = splitmix64(key ^ 0xD1B54A32D192ED03ull);
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0), u2 = (b >> 11) * (1.0 / 9007199254740992.0);
    x[(long)blockIdx.y * stride + g.idx(i, j, l)] = (T)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

// pool[s] = -(A x)[r] as FP32 compact (the residual for f = 0)
template <typename T>
__global__ __launch_bounds__(256) void k_pack_negA3(Grid g, T w0, const T* __restrict__ x, long stride,
                                                    float* __restrict__ pool) {
    const long n = (long)g.m * g.m * g.m;
    const long u = (long)blockIdx.x * 256 + threadIdx.x;
    if (u >= n) return;
    const int i = (int)(u % g.m) + 1, j = (int)((u / g.m) % g.m) + 1, l = (int)(u / ((long)g.m * g.m)) + 1;
    const long id = (long)blockIdx.y * stride + g.idx(i, j, l);
    const long sy = g.pitch, sz = (long)(g.n + 1) * g.pitch;
    const T Ax = w0 * (T(6) * x[id] - x[id - 1] - x[id + 1] - x[id - sy] - x[id + sy] - x[id - sz] - x[id + sz]);
    pool[(long)blockIdx.y * n + u] = (float)(-Ax);
}

}  // namespace

template <typename T>
int launch_resid_norm3(const Grid& g, T w0, const T* x, const T* f, double* partial, int nrhs, long stride,
                       hipStream_t st) {
    const long n = (long)g.m * g.m * g.m;
    dim3 grid((unsigned)((n + 255) / 256), nrhs);
    hipLaunchKernelGGL((k_resid_norm3<T>), grid, dim3(256), 0, st, g, w0, x, f, stride, partial);
    PASM_CHECK_LAUNCH();
    return (int)grid.x;
}
template int launch_resid_norm3<float>(const Grid&, float, const float*, const float*, double*, int, long, hipStream_t);
template int launch_resid_norm3<double>(const Grid&, double, const double*, const double*, double*, int, long,
                                        hipStream_t);

template <typename T>
void launch_fill_normal3(const Grid& g, T* x, int nrhs, long stride, unsigned long long seed, hipStream_t st) {
    const long n = (long)g.m * g.m * g.m;
    hipLaunchKernelGGL((k_fill_normal3<T>), dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, st, g, x, stride,
                       seed);
    PASM_CHECK_LAUNCH();
}
template void launch_fill_normal3<float>(const Grid&, float*, int, long, unsigned long long, hipStream_t);
template void launch_fill_normal3<double>(const Grid&, double*, int, long, unsigned long long, hipStream_t);

template <typename T>
void launch_pack_negA3(const Grid& g, T w0, const T* x, int nrhs, long stride, float* pool, hipStream_t st) {
    const long n = (long)g.m * g.m * g.m;
    hipLaunchKernelGGL((k_pack_negA3<T>), dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, st, g, w0, x, stride,
                       pool);
    PASM_CHECK_LAUNCH();
}
template void launch_pack_negA3<float>(const Grid&, float, const float*, int, long, float*, hipStream_t);
template void launch_pack_negA3<double>(const Grid&, double, const double*, int, long, float*, hipStream_t);

void LearnedTrainer::init(int m_, int S_, float w0_, std::function<void*(size_t)> alloc) {
    m = m_;
    S = S_;
    w0 = w0_;
    const long vol = (long)m * m * m, pvol = (long)(m + 2) * (m + 2) * (m + 2);
    rho_p = (unsigned short*)alloc(sizeof(unsigned short) * pvol * S);
    h_p = (unsigned short*)alloc(sizeof(unsigned short) * pvol * S * 16);
    g_p = (unsigned short*)alloc(sizeof(unsigned short) * pvol * S);
    gh = (unsigned short*)alloc(sizeof(unsigned short) * vol * S * 16);
    z1 = (float*)alloc(sizeof(float) * vol * S * 16);
    y_p = (float*)alloc(sizeof(float) * pvol * S * 32);
    d_p = (float*)alloc(sizeof(float) * pvol * S);
    res_p = (float*)alloc(sizeof(float) * pvol * S);
    nblk_vox = (int)((vol + 255) / 256);
    nr_part = (float*)alloc(sizeof(float) * nblk_vox * S);
    res_part = (float*)alloc(sizeof(float) * nblk_vox * S);
    coef = (float*)alloc(sizeof(float) * S);
    const long nk = (vol * S + 15) / 16;
    dw_kpw = 16;
    dw_blocks = (int)((nk + 4L * dw_kpw - 1) / (4L * dw_kpw));
    dw_part = (float*)alloc(sizeof(float) * 512 * dw_blocks);
    sums = (double*)alloc(sizeof(double) * (2 * 512 + 2 * nblk_vox * S));
    ops = (unsigned long long*)alloc(sizeof(unsigned long long) * 3 * 128);
}

// Loss and gradient of the samples r[0..S) (FP32, interior m^3 each) with
// the weights W (FP32 [2][16][27]); gradient in grad [2][16][27].
double LearnedTrainer::loss_grad(const float* r, const float* W, double* grad, hipStream_t st) {
    const TGrid tg{m, m + 2, (long)m * m * m, (long)(m + 2) * (m + 2) * (m + 2)};
    // operands: layer 1 (W1 as taps x channels), layer 2 (W2 as channels x
    // taps), hidden gradient (W2 as taps x channels)
    unsigned long long hops[3 * 128];
    learned_pack_taps_by_channel(W, hops);
    learned_pack_channels_by_tap(W + 16 * 27, hops + 128);
    learned_pack_taps_by_channel(W + 16 * 27, hops + 256);
    PASM_HIP(hipMemcpyAsync(ops, hops, sizeof(hops), hipMemcpyHostToDevice, st));
    const dim3 gv(nblk_vox, S);
    const long pvol = tg.pvol * S;
    // zero borders of the padded arrays (their interiors are overwritten)
    hipLaunchKernelGGL(k_lt_zero_u16, dim3(1024), dim3(256), 0, st, rho_p, pvol);
    hipLaunchKernelGGL(k_lt_zero_u16, dim3(1024), dim3(256), 0, st, h_p, pvol * 16);
    hipLaunchKernelGGL(k_lt_zero_u16, dim3(1024), dim3(256), 0, st, g_p, pvol);
    hipLaunchKernelGGL(k_lt_zero_f, dim3(1024), dim3(256), 0, st, y_p, pvol * 32);
    hipLaunchKernelGGL(k_lt_zero_f, dim3(1024), dim3(256), 0, st, d_p, pvol);
    hipLaunchKernelGGL(k_lt_zero_f, dim3(1024), dim3(256), 0, st, res_p, pvol);
    PASM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_lt_rho, gv, dim3(256), 0, st, tg, r, 1.f / (6.f * w0), rho_p, nr_part);
    const long nb16 = (tg.vol * S + 15) / 16;
    const int g16 = (int)((nb16 + 3) / 4);
    hipLaunchKernelGGL((k_lt_tapconv<0>), dim3(g16), dim3(256), 0, st, tg, S, rho_p, ops, 1, z1, h_p);
    hipLaunchKernelGGL(k_lt_y, dim3(g16), dim3(256), 0, st, tg, S, h_p, ops + 128, y_p);
    hipLaunchKernelGGL(k_lt_delta, gv, dim3(256), 0, st, tg, y_p, d_p);
    hipLaunchKernelGGL(k_lt_res, gv, dim3(256), 0, st, tg, r, d_p, w0, res_p, res_part);
    PASM_CHECK_LAUNCH();
    // per-sample norms on the host (S values), then coef = -2 / (S ||r||^2)
    double* hs = sums;
    hipLaunchKernelGGL(k_lt_sum, dim3((nblk_vox * S + 255) / 256), dim3(256), 0, st, nr_part, 1, nblk_vox * S, hs);
    hipLaunchKernelGGL(k_lt_sum, dim3((nblk_vox * S + 255) / 256), dim3(256), 0, st, res_part, 1, nblk_vox * S,
                       hs + nblk_vox * S);
    std::vector<double> pn(2 * (size_t)nblk_vox * S);
    PASM_HIP(hipMemcpyAsync(pn.data(), hs, pn.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    PASM_HIP(hipStreamSynchronize(st));
    std::vector<float> cf(S);
    double loss = 0.0;
    for (int s = 0; s < S; ++s) {
        double nr = 0.0, rr = 0.0;
        for (int b = 0; b < nblk_vox; ++b) {
            nr += pn[(size_t)s * nblk_vox + b];
            rr += pn[(size_t)nblk_vox * S + (size_t)s * nblk_vox + b];
        }
        loss += rr / nr / S;
        cf[s] = (float)(-2.0 / (S * nr));
    }
    PASM_HIP(hipMemcpyAsync(coef, cf.data(), S * sizeof(float), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_lt_g, gv, dim3(256), 0, st, tg, res_p, coef, w0, g_p);
    // hidden gradient: sum_t W2[c][t] g(u - t), masked by z1 > 0
    hipLaunchKernelGGL((k_lt_tapconv<1>), dim3(g16), dim3(256), 0, st, tg, S, g_p, ops + 256, -1, z1, gh);
    // dW2[c][t] = sum_u h(u)[c] g(u - t); dW1[c][t] = sum_u gh(u)[c] rho(u + t)
    hipLaunchKernelGGL((k_lt_dw<true>), dim3(dw_blocks), dim3(256), 0, st, tg, S, h_p, g_p, -1, dw_part, dw_kpw);
    hipLaunchKernelGGL(k_lt_sum, dim3(2), dim3(256), 0, st, dw_part, dw_blocks, 512, sums + 512);
    hipLaunchKernelGGL((k_lt_dw<false>), dim3(dw_blocks), dim3(256), 0, st, tg, S, gh, rho_p, 1, dw_part, dw_kpw);
    hipLaunchKernelGGL(k_lt_sum, dim3(2), dim3(256), 0, st, dw_part, dw_blocks, 512, sums);
    PASM_CHECK_LAUNCH();
    std::vector<double> gd(1024);
    PASM_HIP(hipMemcpyAsync(gd.data(), sums, 1024 * sizeof(double), hipMemcpyDeviceToHost, st));
    PASM_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < 16; ++c)
        for (int t = 0; t < 27; ++t) {
            grad[c * 27 + t] = gd[c * 32 + t];
            grad[16 * 27 + c * 27 + t] = gd[512 + c * 32 + t];
        }
    return loss;
}

}  // namespace pasm

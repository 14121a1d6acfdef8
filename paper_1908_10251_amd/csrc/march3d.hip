// Smoothing phases of the V-cycle on the 3D Kuhn mesh (constant
// coefficients, 128 cells per side) as sweeps that march along z with all S
// steps of a phase in flight.
//
// A workgroup of WAVES wavefronts owns a slab of YL = WAVES * RW rows of every
// z-plane, all 128 columns of them: lane l holds columns 2l + 1 and 2l + 2, so
// its x-neighbours are its own other column or come by a DPP wavefront shift,
// and wavefront w holds RW consecutive rows, so its y-neighbours are in its own
// registers except across the wavefront's first and last row, which
// neighbouring wavefronts exchange through LDS once per plane.  The
// z-neighbours are the thread's own window of the last three planes of every
// stage.  When plane p is loaded, stage t advances plane p - t, so stage S
// emits plane p - S: every node of the slab is read and written once per
// phase.  Rows within t of the slab's edge hold garbage after t steps, so a
// slab stores its YL - 2S inner rows and neighbouring slabs overlap by 2S rows
// (read twice, the second time mostly from the die's L2).
//
// Steps follow x_{t+1} = x_t + a_t (x_t - x_{t-1}) + b_t D^{-1} (f - A x_t)
// with a_0 = 0 and the 7-point stiffness w0 (6 x - sum of the axis
// neighbours) of the constant-coefficient Kuhn mesh.  Modes:
//   0  x_0 read from x;
//   1  x_0 = 0 (x is not read);
//   2  x_0 = x + P e_c: the coarse correction prolongated while loading (a
//      fine node (2I,2J,2L) + o, o in {0,1}^3, takes the mean of the coarse
//      nodes (I,J,L) and (I,J,L) + o).
#include <algorithm>

#include "common.h"

namespace pasm {

namespace {

constexpr int NL = 64;     // lanes per wavefront
constexpr int XCDS = 8;    // accelerator dies; workgroup b runs on die b % 8
constexpr int M3N = 128;   // cells per side the marching sweep covers

// DPP wavefront shifts by one lane; the lane at the edge receives 0.
__device__ inline float lane_from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ inline float lane_from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ inline double lane_from_left(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double lane_from_right(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Raw buffer accesses: a resource over one right-hand side's block (base in
// scalar registers), a 32-bit per-lane byte offset within a plane and the
// plane's byte offset as the uniform scalar offset, so no lane keeps a 64-bit
// address per row.  Every access of the kernels below is inside the block.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRawBufferWord3 = 0x00020000;  // 32-bit data format, raw (stride 0) addressing
// A per-lane offset at or past the resource's size makes the access out of
// range: a load returns 0, a store is discarded.  2^31 stays out of range
// after any plane offset is added (blocks are far below 2 GiB).
constexpr unsigned kDropped = 0x80000000u;
__device__ inline rsrc_t make_rsrc(const void* p, long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kRawBufferWord3);
}
template <typename V>
__device__ inline V bload(rsrc_t r, unsigned vo, unsigned so) {
    if constexpr (sizeof(V) == 4)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    else if constexpr (sizeof(V) == 8)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    else
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
}
// Stores take their whole offset per lane and a constant zero scalar offset.
// A store of more than 64 bits whose data registers are overwritten right
// after it issues has stored stale values in some lanes when the scalar offset
// was a register (a case the compiler treats as free of that hazard and
// inserts no wait for); with a constant scalar offset it inserts the wait.
template <typename V>
__device__ inline void bstore(V v, rsrc_t r, unsigned vo) {
    using u2 = unsigned __attribute__((ext_vector_type(2)));
    using u4 = unsigned __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(V) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, vo, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, vo, 0, 0);
}

template <typename T>
struct March3Shape;
template <>
struct March3Shape<float> {
    static constexpr int WAVES = 8, RW = 4, WPE = 4;  // two workgroups per compute unit
};
template <>
struct March3Shape<double> {
    static constexpr int WAVES = 8, RW = 4, WPE = 2;
};

constexpr int slot3(int v) { return ((v % 3) + 3) % 3; }

template <typename T, int S, int MODE, int WAVES, int RW, int WPE>
__global__ __launch_bounds__(NL* WAVES) __attribute__((amdgpu_waves_per_eu(WPE))) void k_march3(Grid g, T w0, const T* __restrict__ x,
                                                      const T* __restrict__ f, T* __restrict__ out, Grid gc,
                                                      const T* __restrict__ ec, long sf, long sc, SmoothSteps st,
                                                      int slabs, int items, int chunk) {
    using T2 = T __attribute__((ext_vector_type(2)));
    constexpr int YL = WAVES * RW;
    constexpr int YO = YL - 2 * S;             // rows a slab stores
    constexpr int JP = (1 - S) & 1;            // parity of every wavefront's first row (YO, RW even)
    constexpr int CR = ((JP + RW) >> 1) + 1;   // coarse rows under a wavefront's rows
    // FP64: the odd columns' coarse values (column l) are loaded; FP32: they
    // come from the neighbouring lane (registers are the tighter budget there)
    constexpr bool LLOAD = sizeof(T) == 8;
    constexpr int CRL = LLOAD ? ((JP + RW - 1) >> 1) + 1 : 1;  // rows (I, J, L) of the odd columns
    static_assert(RW % 2 == 0 && S >= 1 && S <= 2, "shape");
    __shared__ T2 edge[2][S][WAVES][2][NL];    // [plane parity][stage][wavefront][first/last row][lane]

    // Consecutive pieces of work (the slabs of one right-hand side) go to the
    // same die, so the rows that neighbouring slabs share are found in its L2.
    const int item = (blockIdx.x % XCDS) * chunk + blockIdx.x / XCDS;
    if (item >= items) return;  // uniform per workgroup
    const int r = item / slabs, slab = item % slabs;
    const int lane = threadIdx.x & (NL - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / NL);
    const int n = g.n, m = g.m;
    const long zs = (long)(n + 1) * g.pitch;
    const long zcs = (long)(gc.n + 1) * gc.pitch;
    const T* xr = x + (long)r * sf;
    const T* fr = f + (long)r * sf;
    T* outr = out + (long)r * sf;
    const T* ecr = ec + (long)r * sc;

    // rows of this wavefront; positions outside the grid read the boundary
    // ring (clamped addresses) and are held at zero in every stage.  Byte
    // offsets within a plane are 32-bit, added to per-plane base addresses
    // that are uniform over the workgroup.
    const int jb = 1 + slab * YO - S + w * RW;
    unsigned boff[RW];
    unsigned rowok = 0, outok = 0;
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int j = jb + q;
        boff[q] = (unsigned)(min(max(j, 0), n) * g.pitch + ORIGIN + 2 * lane + 1) * (unsigned)sizeof(T);
        const int y = w * RW + q;
        if (j >= 1 && j <= m) {
            rowok |= 1u << q;
            if (y >= S && y < YL - S) outok |= 1u << q;
        }
    }
    unsigned oboff[RW];  // store offsets; rows a slab does not store are dropped
#pragma unroll
    for (int q = 0; q < RW; ++q) oboff[q] = ((outok >> q) & 1u) ? boff[q] : kDropped;
    const bool c1ok = 2 * lane + 2 <= m;  // column 2l + 1 is always interior for n = 128
    unsigned cboff[CR];
#pragma unroll
    for (int c = 0; c < CR; ++c)
        cboff[c] = (unsigned)(min(max((jb >> 1) + c, 0), gc.n) * gc.pitch + ORIGIN + lane + 1) * (unsigned)sizeof(T);

    const T invD = T(1) / (T(6) * w0);
    T bs[S], as[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        bs[t] = (T)st.b[t] * invD;
        as[t] = (T)st.a[t];
    }

    for (int e = threadIdx.x; e < 2 * S * WAVES * 2 * NL; e += NL * WAVES) (&edge[0][0][0][0][0])[e] = T2(0);
    // edge rows of the wavefronts above and below (the outermost wavefronts
    // read their own: those rows are halo, never stored)
    const int wu = w > 0 ? w - 1 : 0, wd = w < WAVES - 1 ? w + 1 : WAVES - 1;

    T2 X[S][3][RW];  // stage t < S at the plane with slot (plane mod 3)
    T2 F[4][RW];     // f at the plane with slot (plane mod 4); plane p + 1 loads into its slot in place
    T2 PX[RW];
    T C[2][CR];    // coarse column l + 1 of coarse plane L in slot L & 1
    T CL[2][CRL];  // coarse column l of the same planes, rows the odd columns use
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < RW; ++q) X[t][k][q] = T2(0);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < RW; ++q) F[k][q] = T2(0);
#pragma unroll
    for (int c = 0; c < CR; ++c) C[0][c] = C[1][c] = T(0);  // coarse plane 0 is the boundary
#pragma unroll
    for (int c = 0; c < CRL; ++c) CL[0][c] = CL[1][c] = T(0);

    const long blk = sf * (long)sizeof(T), cblk = sc * (long)sizeof(T);
    const rsrc_t xs = make_rsrc(xr, blk), fs = make_rsrc(fr, blk), os = make_rsrc(outr, blk);
    const rsrc_t es = make_rsrc(ecr, cblk);
    const unsigned zsb = (unsigned)(zs * (long)sizeof(T)), zcsb = (unsigned)(zcs * (long)sizeof(T));
    auto issue = [&](int p, T2* fslot) {  // plane p of x and f (clamped onto the boundary plane n)
        const unsigned zo = (unsigned)min(p, n) * zsb;
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            fslot[q] = bload<T2>(fs, boff[q], zo);
            if (MODE != 1) PX[q] = bload<T2>(xs, boff[q], zo);
        }
    };
    auto issue_coarse = [&](int L, T* cslot, T* lslot) {
        const unsigned zo = (unsigned)min(L, gc.n) * zcsb;
#pragma unroll
        for (int c = 0; c < CR; ++c) cslot[c] = bload<T>(es, cboff[c], zo);
        if (LLOAD) {
#pragma unroll
            for (int c = 0; c < CRL; ++c) lslot[c] = bload<T>(es, cboff[c] - (unsigned)sizeof(T), zo);
        }
    };

    issue(1, F[1]);
    if (MODE == 2) issue_coarse(1, C[1], CL[1]);
    // Planes run to m + S, rounded up to whole unrolled bodies: the planes
    // past m + S are all masked and their stores dropped, so the body needs no
    // exit, whose control flow would break the fixed register slots.
    const int pend = m + S;
    for (int p0 = 1; p0 <= pend; p0 += 12) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const int p = p0 + k;  // p0 = 1 (mod 12): slots and parities below are constants
            const bool odd = (k & 1) == 0;
            // coarse plane L = floor(p / 2) = (p0 - 1) / 2 + floor((k + 1) / 2), (p0 - 1) / 2 even
            const int cl = ((k + 1) >> 1) & 1;
            const T* CA = C[cl];      // coarse plane L
            const T* CB = C[cl ^ 1];  // coarse plane L + 1 (odd p)
            const int sp = slot3(1 + k);
            const int fp = (1 + k) & 3;
            const bool pin = p <= m;

            // stage 0 of plane p
            T left[CR];  // coarse plane L, column l
#pragma unroll
            for (int c = 0; c < CR; ++c) left[c] = T(0);
            if (MODE == 2) {
#pragma unroll
                for (int c = 0; c < CR; ++c) left[c] = LLOAD ? (c < CRL ? CL[cl][c] : T(0)) : lane_from_left(CA[c]);
            }
            if (MODE != 1) {
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    T2 v = PX[q];
                    if (MODE == 2) {
                        const int jr = (JP + q) >> 1, b = (JP + q) & 1;
                        // column 2l + 1: coarse (l, J, L) and (l + 1, J + b, L + c)
                        const T hi1 = odd ? CB[jr + b] : CA[jr + b];
                        v.x += T(0.5) * (left[jr] + hi1);
                        // column 2l + 2: coarse (l + 1, J, L) and (l + 1, J + b, L + c)
                        v.y += (b == 0 && !odd) ? CA[jr] : T(0.5) * (CA[jr] + hi1);
                    }
                    const bool ok0 = pin && ((rowok >> q) & 1u);
                    X[0][sp][q] = T2{ok0 ? v.x : T(0), ok0 && c1ok ? v.y : T(0)};
                }
            }

            // plane p + 1 in flight while this plane's stages run (its f slot
            // held plane p - 3, whose last use was in the previous plane)
            issue(p + 1, F[(2 + k) & 3]);
            // even p = 2L: coarse plane L + 1 into the slot of plane L - 1, last used at p - 1
            if (MODE == 2 && !odd) issue_coarse(p / 2 + 1, C[cl ^ 1], CL[cl ^ 1]);
            // this wavefront's edge rows of the previous plane must have
            // reached LDS before the barrier releases their readers; the
            // compiler's own wait is not placed on every unrolled copy
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt and expcnt not waited on
            __syncthreads();

            T2 res[RW];
#pragma unroll
            for (int t = 1; t <= S; ++t) {
                const int qz = p - t;
                const bool qin = qz >= 1 && qz <= m;
                const int sq = slot3(1 + k - t), slo = slot3(k - t), shi = slot3(2 + k - t);
                const int fq = (1 + k - t + 12) & 3;
                const int par = k & 1;  // edge rows written while plane p - 1 was loaded
                T2 up = T2(0), dn = T2(0);
                if (!(MODE == 1 && t == 1)) {
                    up = edge[par][t - 1][wu][1][lane];
                    dn = edge[par][t - 1][wd][0][lane];
                }
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    T2 nv;
                    if (MODE == 1 && t == 1) {
                        nv = bs[0] * F[fq][q];
                    } else {
                        const T2 c = X[t - 1][sq][q];
                        T2 s = (q > 0 ? X[t - 1][sq][q - 1] : up) + (q < RW - 1 ? X[t - 1][sq][q + 1] : dn) +
                               X[t - 1][slo][q] + X[t - 1][shi][q];
                        s.x += lane_from_left(c.y) + c.y;
                        s.y += c.x + lane_from_right(c.x);
                        nv = c + bs[t - 1] * (F[fq][q] - w0 * (T(6) * c - s));
                        if (t >= 2) {
                            const T2 prev = MODE == 1 && t == 2 ? T2(0) : X[t - 2][sq][q];
                            nv += as[t - 1] * (c - prev);
                        }
                    }
                    const bool ok0 = qin && ((rowok >> q) & 1u);
                    nv = T2{ok0 ? nv.x : T(0), ok0 && c1ok ? nv.y : T(0)};
                    if (t < S)
                        X[t][sq][q] = nv;
                    else
                        res[q] = nv;
                }
            }

            // first and last rows for the neighbouring wavefronts, read after
            // the next barrier
            const int pw = (1 + k) & 1;
            if (MODE != 1) {
                edge[pw][0][w][0][lane] = X[0][sp][0];
                edge[pw][0][w][1][lane] = X[0][sp][RW - 1];
            }
#pragma unroll
            for (int t = 1; t < S; ++t) {
                const int sq = slot3(1 + k - t);
                edge[pw][t][w][0][lane] = X[t][sq][0];
                edge[pw][t][w][1][lane] = X[t][sq][RW - 1];
            }

            // stores are unconditional (a branch around them would make the
            // next plane wait for them): rows and planes that are not stored
            // take an offset past the end of the block, which the buffer
            // range check discards
            const int qz = p - S;
            const bool qok = qz >= 1 && qz <= m;
            unsigned zo = qok ? (unsigned)qz * zsb : 0u;
            // opaque to loop strength reduction, which would otherwise keep one
            // per-lane offset register per unrolled plane and row
            asm volatile("" : "+s"(zo));
#pragma unroll
            for (int q = 0; q < RW; ++q) bstore<T2>(res[q], os, (qok ? oboff[q] : kDropped) + zo);
        }
    }
}

template <typename T, int S, int MODE>
void march3_launch(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                   const SmoothSteps& ss, hipStream_t st) {
    constexpr int WAVES = March3Shape<T>::WAVES, RW = March3Shape<T>::RW;
    // x_0 read from memory (mode 0) needs a register window more than the others
    constexpr int WPE = MODE == 0 ? 2 : March3Shape<T>::WPE;
    constexpr int YO = WAVES * RW - 2 * S;
    if ((long)g.plane * (long)sizeof(T) >= (1L << 31) || (long)gc.plane * (long)sizeof(T) >= (1L << 31))
        throw Error(PASM_E_INVALID, "3D marching smoother: right-hand side blocks of 2 GiB or more");
    const int slabs = (g.m + YO - 1) / YO;
    const int items = slabs * nrhs;
    const int chunk = (items + XCDS - 1) / XCDS;
    hipLaunchKernelGGL((k_march3<T, S, MODE, WAVES, RW, WPE>), dim3(chunk * XCDS), dim3(NL * WAVES), 0, st, g, w0, x, f,
                       out, gc, ec, g.plane, gc.plane, ss, slabs, items, chunk);
    PASM_CHECK_LAUNCH();
}

template <typename T, int MODE>
void march3_steps(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                  const SmoothSteps& ss, hipStream_t st) {
    if (ss.s == 1)
        march3_launch<T, 1, MODE>(g, w0, x, f, out, gc, ec, nrhs, ss, st);
    else
        march3_launch<T, 2, MODE>(g, w0, x, f, out, gc, ec, nrhs, ss, st);
}

}  // namespace

bool march3_supported(const Grid& g, bool const_coef, int steps) {
    return g.dim == 3 && const_coef && g.n == M3N && steps >= 1 && steps <= 2;
}

template <typename T>
void launch_march3_smooth(const Grid& g, T w0, const T* x0, const T* f, T* out, int nrhs, const SmoothSteps& ss,
                          bool x_zero, hipStream_t st) {
    if (!march3_supported(g, true, ss.s)) throw Error(PASM_E_INVALID, "3D marching smoother: shape not supported");
    if (x_zero)
        march3_steps<T, 1>(g, w0, x0, f, out, g, x0, nrhs, ss, st);
    else
        march3_steps<T, 0>(g, w0, x0, f, out, g, x0, nrhs, ss, st);
}

template <typename T>
void launch_march3_post(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                        const SmoothSteps& ss, hipStream_t st) {
    if (!march3_supported(g, true, ss.s) || gc.dim != 3 || gc.n * 2 != g.n)
        throw Error(PASM_E_INVALID, "3D marching smoother: shape not supported");
    march3_steps<T, 2>(g, w0, x, f, out, gc, ec, nrhs, ss, st);
}

#define PASM_INST_MARCH3(T)                                                                                        \
    template void launch_march3_smooth<T>(const Grid&, T, const T*, const T*, T*, int, const SmoothSteps&, bool,  \
                                          hipStream_t);                                                           \
    template void launch_march3_post<T>(const Grid&, T, const T*, const T*, T*, const Grid&, const T*, int,        \
                                        const SmoothSteps&, hipStream_t);
PASM_INST_MARCH3(float)
PASM_INST_MARCH3(double)

}  // namespace pasm

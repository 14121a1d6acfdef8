// Conjugate-gradient smoothing: the smoother of the paper's experiments
// (Section 5: one multigrid step with 2 CG steps for pre- and post-smoothing).
//
// nu steps of plain (unpreconditioned) CG on A x = f per right-hand side, on
// one level, from the current x (or from x = 0):
//     r = f - A x, p = r, rr = r.r
//     per step: q = A p, alpha = rr / p.q, x += alpha p, r -= alpha q,
//               rr' = r.r, beta = rr' / rr, p = r + beta p
// A zero denominator (the iterate already exact) gives alpha = 0 / beta = 0.
// Unlike the fixed-polynomial smoothers, every step needs two inner products
// over the whole level per right-hand side: each launch leaves one partial
// sum per workgroup (FP64, a fixed tree inside the workgroup), and a small
// kernel per right-hand side adds them in a fixed order, so results do not
// depend on scheduling.  The direction update p = r + beta p is fused into
// the next q = A p pass (the neighbours' p are formed on the fly from r and
// the old p, so the new p goes to the other of two buffers).
#include "common.h"

namespace pasm {
namespace {

constexpr int CX = 64, CY = 4;  // one workgroup: 64 x 4 nodes of one (z-)plane

// Kernels that apply the operator take RB right-hand sides per thread, so
// that the coefficients of a node's row are read once for all of them; the
// vector updates take UB, so that a workgroup's reduction serves that many.
template <int DIM, int KIND>
constexpr int rhs_block() { return KIND == 0 ? 1 : 4; }
constexpr int UB = 4;

struct NodeIdx {
    long id;    // padded index of the node in its plane / volume
    int r0;     // first right-hand side of the thread's group
    long blk;   // workgroup index within the right-hand side
    bool ok;    // an interior node
};

// blockIdx.z: the right-hand side group (2D), or (plane, group) (3D)
template <int DIM, int RB>
__device__ inline NodeIdx node_of(const Grid& g) {
    NodeIdx n;
    const int i = blockIdx.x * CX + threadIdx.x + 1;
    const int j = blockIdx.y * CY + threadIdx.y + 1;
    int l = 0;
    if (DIM == 2) {
        n.r0 = blockIdx.z * RB;
        n.blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
    } else {
        l = blockIdx.z % g.m + 1;
        n.r0 = (blockIdx.z / g.m) * RB;
        n.blk = ((long)(l - 1) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    }
    n.ok = i <= g.m && j <= g.m;
    n.id = DIM == 2 ? g.idx(i, j) : g.idx(i, j, l);
    return n;
}

// The level operator's row at one node, its coefficients held in registers:
// KIND 0 constant coefficient (w0 times the 5- or 7-point Laplacian), 1 edge
// weights, 2 general 2D 7-point stencil (diagonal, edge weights and the "/"
// diagonal weight), 3 the 3D 15-point operator (diagonal plane, then
// A(i, i + o) for the seven Kuhn edge directions o).  apply() takes v as a
// callable of the padded index (so that v can be formed on the fly).
template <typename T, int DIM, int KIND>
struct OpRow;

template <typename T, int DIM>
struct OpRow<T, DIM, 0> {
    T w0;
    __device__ inline void load(const Grid&, const Coef<T>& c, long) { w0 = c.w0; }
    template <typename V>
    __device__ inline T apply(const Grid& g, long id, V v) const {
        const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
        const T x0 = v(id);
        if (DIM == 2) return w0 * (T(4) * x0 - v(id + 1) - v(id - 1) - v(id + py) - v(id - py));
        return w0 * (T(6) * x0 - v(id + 1) - v(id - 1) - v(id + py) - v(id - py) - v(id + pz) - v(id - pz));
    }
};

template <typename T>
struct OpRow<T, 2, 1> {
    T we, ww, wn, ws;
    __device__ inline void load(const Grid& g, const Coef<T>& c, long id) {
        we = c.wx[id], ww = c.wx[id - 1], wn = c.wy[id], ws = c.wy[id - g.pitch];
    }
    template <typename V>
    __device__ inline T apply(const Grid& g, long id, V v) const {
        const long py = g.pitch;
        const T x0 = v(id);
        return we * (x0 - v(id + 1)) + ww * (x0 - v(id - 1)) + wn * (x0 - v(id + py)) + ws * (x0 - v(id - py));
    }
};

template <typename T>
struct OpRow<T, 2, 2> {
    T d, we, ww, wn, ws, wne, wsw;
    __device__ inline void load(const Grid& g, const Coef<T>& c, long id) {
        const long py = g.pitch;
        d = c.d[id], we = c.wx[id], ww = c.wx[id - 1], wn = c.wy[id], ws = c.wy[id - py];
        wne = c.wne[id], wsw = c.wne[id - py - 1];
    }
    template <typename V>
    __device__ inline T apply(const Grid& g, long id, V v) const {
        const long py = g.pitch;
        return d * v(id) - we * v(id + 1) - ww * v(id - 1) - wn * v(id + py) - ws * v(id - py) -
               wne * v(id + py + 1) - wsw * v(id - py - 1);
    }
};

template <typename T>
struct OpRow<T, 3, 1> {
    T w[6];
    __device__ inline void load(const Grid& g, const Coef<T>& c, long id) {
        const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
        w[0] = c.wx[id], w[1] = c.wx[id - 1], w[2] = c.wy[id], w[3] = c.wy[id - py], w[4] = c.wz[id],
        w[5] = c.wz[id - pz];
    }
    template <typename V>
    __device__ inline T apply(const Grid& g, long id, V v) const {
        const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
        const T x0 = v(id);
        return w[0] * (x0 - v(id + 1)) + w[1] * (x0 - v(id - 1)) + w[2] * (x0 - v(id + py)) +
               w[3] * (x0 - v(id - py)) + w[4] * (x0 - v(id + pz)) + w[5] * (x0 - v(id - pz));
    }
};

template <typename T>
struct OpRow<T, 3, 3> {
    T d, up[7], dn[7];
    __device__ static inline long off(const Grid& g, int t) {
        const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
        const long o7[7] = {1, py, pz, 1 + py, 1 + pz, py + pz, 1 + py + pz};
        return o7[t];
    }
    __device__ inline void load(const Grid& g, const Coef<T>& c, long id) {
        const long P = g.plane;
        d = c.s15[id];
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            up[t] = c.s15[(t + 1) * P + id];
            dn[t] = c.s15[(t + 1) * P + id - off(g, t)];
        }
    }
    template <typename V>
    __device__ inline T apply(const Grid& g, long id, V v) const {
        T acc = d * v(id);
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            const long o = off(g, t);
            acc += up[t] * v(id + o) + dn[t] * v(id - o);
        }
        return acc;
    }
};

// Sums of RB doubles per thread over the workgroup (each in a fixed order);
// the sum of value q goes to out[q * nblk], for q < nvalid.
template <int RB>
__device__ inline void block_partials(double (&v)[RB], double* out, long nblk, int nvalid) {
    __shared__ double sh[RB][CX * CY / 64];
    const int t = threadIdx.y * CX + threadIdx.x;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        double s = v[q];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if ((t & 63) == 0) sh[q][t >> 6] = s;
    }
    __syncthreads();
    if (t < RB && t < nvalid) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < CX * CY / 64; ++w) s += sh[t][w];
        out[(long)t * nblk] = s;
    }
}

// r = f - A x (XZ: x = 0, r = f); partial sums of r.r
template <typename T, int DIM, int KIND, bool XZ>
__global__ __launch_bounds__(CX* CY) void k_cg_start(Grid g, Coef<T> c, const T* __restrict__ x,
                                                     const T* __restrict__ f, T* __restrict__ r,
                                                     double* __restrict__ partial, long stride, long nblk, int nrhs) {
    constexpr int RB = XZ ? UB : rhs_block<DIM, KIND>();
    const NodeIdx n = node_of<DIM, RB>(g);
    const int nv = min(RB, nrhs - n.r0);
    double acc[RB];
    OpRow<T, DIM, KIND> row;
    if (!XZ && n.ok) row.load(g, c, n.id);
    // every right-hand side's value before any store
    T rv[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        rv[q] = T(0);
        if (n.ok && q < nv) {
            const long off = (long)(n.r0 + q) * stride;
            rv[q] = f[off + n.id];
            if (!XZ) {
                const T* xr = x + off;
                rv[q] -= row.apply(g, n.id, [&](long k) { return xr[k]; });
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        acc[q] = 0.0;
        if (n.ok && q < nv) {
            r[(long)(n.r0 + q) * stride + n.id] = rv[q];
            acc[q] = (double)rv[q] * (double)rv[q];
        }
    }
    block_partials<RB>(acc, partial + (long)n.r0 * nblk + n.blk, nblk, nv);
}

// p_new = r + beta p_old (FIRST: p_new = r), q = A p_new; partial sums of p_new.q
template <typename T, int DIM, int KIND, bool FIRST>
__global__ __launch_bounds__(CX* CY) void k_cg_dir(Grid g, Coef<T> c, const T* __restrict__ r,
                                                   const T* __restrict__ pold, const double* __restrict__ beta,
                                                   T* __restrict__ pnew, T* __restrict__ q,
                                                   double* __restrict__ partial, long stride, long nblk, int nrhs) {
    constexpr int RB = rhs_block<DIM, KIND>();
    const NodeIdx n = node_of<DIM, RB>(g);
    const int nv = min(RB, nrhs - n.r0);
    double acc[RB];
    OpRow<T, DIM, KIND> row;
    if (n.ok) row.load(g, c, n.id);
    // every right-hand side's values before any store
    T p0[RB], qv[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        p0[u] = qv[u] = T(0);
        if (n.ok && u < nv) {
            const long off = (long)(n.r0 + u) * stride;
            const T* rr = r + off;
            const T* po = pold + off;
            const T b = FIRST ? T(0) : (T)beta[n.r0 + u];
            auto pv = [&](long k) { return FIRST ? rr[k] : rr[k] + b * po[k]; };
            p0[u] = pv(n.id);
            qv[u] = row.apply(g, n.id, pv);
        }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        acc[u] = 0.0;
        if (n.ok && u < nv) {
            const long off = (long)(n.r0 + u) * stride;
            pnew[off + n.id] = p0[u];
            q[off + n.id] = qv[u];
            acc[u] = (double)p0[u] * (double)qv[u];
        }
    }
    block_partials<RB>(acc, partial + (long)n.r0 * nblk + n.blk, nblk, nv);
}

// The direction pass for 3D 15-point operators marching along z: a
// workgroup owns ZX x ZY nodes of a chunk of ZC planes for RB right-hand
// sides, and keeps the last three planes of the new direction
// p = r + beta p_old (one-node halo) for all of them in an LDS ring, formed
// while the plane enters; q = A p comes from the ring, each node's 15
// coefficients loaded once for the RB right-hand sides.  The arithmetic is
// k_cg_dir's; the partial sums are per workgroup of this grid.
constexpr int ZX = 32, ZY = 16, ZC = 16;
constexpr int ZHX = ZX + 2, ZHY = ZY + 2, ZN = ZHX * ZHY, ZPL = (ZN + CX * CY - 1) / (CX * CY),
              ZOWN = ZX * ZY / (CX * CY);
template <typename T, bool FIRST, int RB>
__global__ __launch_bounds__(CX* CY) void k_cg_dir_z(Grid g, Coef<T> c, const T* __restrict__ r,
                                                     const T* __restrict__ pold, const double* __restrict__ beta,
                                                     T* __restrict__ pnew, T* __restrict__ q,
                                                     double* __restrict__ partial, long stride, long nblk, int nrhs,
                                                     int zchunks) {
    constexpr int NT = CX * CY;
    __shared__ T ring[RB][3][ZN];
    const int tid = threadIdx.y * CX + threadIdx.x;
    const int zc = blockIdx.z % zchunks, grp = blockIdx.z / zchunks;
    const int r0 = grp * RB, nv = min(RB, nrhs - r0);
    const int i0 = blockIdx.x * ZX + 1, j0 = blockIdx.y * ZY + 1;
    const int k0 = zc * ZC + 1, k1 = min(k0 + ZC, g.m + 1);
    const long blk = ((long)zc * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const long pz = (long)g.pitch * (g.n + 1);
    // ring positions of this thread (clamped onto the grid; outside the
    // interior the direction is zero)
    long ho[ZPL];
    bool hin[ZPL];
#pragma unroll
    for (int e = 0; e < ZPL; ++e) {
        const int t = tid + NT * e;
        const int i = i0 - 1 + t % ZHX, j = j0 - 1 + t / ZHX;
        hin[e] = t < ZN && i >= 1 && j >= 1 && i <= g.m && j <= g.m;
        ho[e] = (long)min(j, g.n) * g.pitch + ORIGIN + min(i, g.n);
    }
    T b[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) b[u] = (!FIRST && u < nv) ? (T)beta[r0 + u] : T(0);
    // the direction at plane k of the ring positions, for every right-hand side
    auto form = [&](int k, T (&v)[RB][ZPL]) {
        const bool kin = k >= 1 && k <= g.m;
        const long base = (long)min(max(k, 0), g.n) * pz;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const long off = (long)(r0 + min(u, nv - 1)) * stride + base;
#pragma unroll
            for (int e = 0; e < ZPL; ++e) {
                const T rv = r[off + ho[e]];
                const T pv = FIRST ? rv : rv + b[u] * pold[off + ho[e]];
                v[u][e] = (kin && hin[e]) ? pv : T(0);
            }
        }
    };
    auto store = [&](int slot, const T (&v)[RB][ZPL]) {
#pragma unroll
        for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int e = 0; e < ZPL; ++e)
                if (tid + NT * e < ZN) ring[u][slot][tid + NT * e] = v[u][e];
    };
    double acc[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) acc[u] = 0.0;
    T va[RB][ZPL], vb[RB][ZPL];
    form(k0 - 1, va);
    form(k0, vb);
    store((k0 - 1) % 3, va);
    store(k0 % 3, vb);
    form(k0 + 1, va);
    // ring offsets of the seven Kuhn edge directions (x, y within the plane;
    // z by the ring slot)
    constexpr int o_in[7] = {1, ZHX, 0, 1 + ZHX, 1, ZHX, 1 + ZHX};
    constexpr int o_dz[7] = {0, 0, 1, 0, 1, 1, 1};
    for (int k = k0; k < k1; ++k) {
        store((k + 1) % 3, va);
        if (k + 1 < k1) form(k + 2, va);  // one plane ahead
        __syncthreads();
        const int s0 = k % 3, sp = (k + 1) % 3, sm = (k + 2) % 3;
#pragma unroll
        for (int e = 0; e < ZOWN; ++e) {
            const int t = tid + NT * e;
            const int a = t % ZX, bb = t / ZX;
            const int i = i0 + a, j = j0 + bb;
            if (i > g.m || j > g.m) continue;
            const long gid = (long)k * pz + (long)j * g.pitch + ORIGIN + i;
            OpRow<T, 3, 3> row;
            row.load(g, c, gid);
            const int hc = (bb + 1) * ZHX + (a + 1);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                if (u >= nv) break;
                const T* R0 = ring[u][s0];
                const T* RP = ring[u][sp];
                const T* RM = ring[u][sm];
                const T p0 = R0[hc];
                T qv = row.d * p0;
#pragma unroll
                for (int tt = 0; tt < 7; ++tt) {
                    const T* Ru = o_dz[tt] ? RP : R0;
                    const T* Rd = o_dz[tt] ? RM : R0;
                    qv += row.up[tt] * Ru[hc + o_in[tt]] + row.dn[tt] * Rd[hc - o_in[tt]];
                }
                const long id = (long)(r0 + u) * stride + gid;
                pnew[id] = p0;
                q[id] = qv;
                acc[u] += (double)p0 * (double)qv;
            }
        }
        __syncthreads();
    }
    block_partials<RB>(acc, partial + (long)r0 * nblk + blk, nblk, nv);
}

// x += alpha p (XZ: x = alpha p); with RR also r -= alpha q and partial sums of r.r
template <typename T, int DIM, bool RR, bool XZ>
__global__ __launch_bounds__(CX* CY) void k_cg_update(Grid g, T* __restrict__ x, T* __restrict__ r,
                                                      const T* __restrict__ p, const T* __restrict__ q,
                                                      const double* __restrict__ alpha, double* __restrict__ partial,
                                                      long stride, long nblk, int nrhs) {
    const NodeIdx n = node_of<DIM, UB>(g);
    const int nv = min(UB, nrhs - n.r0);
    double acc[UB];
    // every load of the thread's right-hand sides before any store
    T av[UB], pv[UB], qv[UB], rv[UB], xv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        av[u] = pv[u] = qv[u] = rv[u] = xv[u] = T(0);
        if (n.ok && u < nv) {
            const long k = (long)(n.r0 + u) * stride + n.id;
            av[u] = (T)alpha[n.r0 + u];
            pv[u] = p[k];
            if (RR) qv[u] = q[k], rv[u] = r[k];
            if (!XZ) xv[u] = x[k];
        }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        acc[u] = 0.0;
        if (n.ok && u < nv) {
            const long k = (long)(n.r0 + u) * stride + n.id;
            x[k] = XZ ? av[u] * pv[u] : xv[u] + av[u] * pv[u];
            if (RR) {
                const T rn = rv[u] - av[u] * qv[u];
                r[k] = rn;
                acc[u] = (double)rn * (double)rn;
            }
        }
    }
    if (RR) block_partials<UB>(acc, partial + (long)n.r0 * nblk + n.blk, nblk, nv);
}

// Per right-hand side: s = sum of its nblk partials (fixed order), then
// MODE 0: rr = s;  1: alpha = rr / s (0 if s = 0);  2: beta = s / rr (0 if rr = 0), rr = s.
template <int MODE>
__global__ __launch_bounds__(256) void k_cg_reduce(const double* __restrict__ partial, long nblk,
                                                   double* __restrict__ rr, double* __restrict__ out) {
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const double* pr = partial + (long)r * nblk;
    double s = 0.0;
    for (long b = threadIdx.x; b < nblk; b += 256) s += pr[b];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        if (MODE == 0) {
            rr[r] = t;
        } else if (MODE == 1) {
            out[r] = t != 0.0 ? rr[r] / t : 0.0;
        } else {
            out[r] = rr[r] != 0.0 ? t / rr[r] : 0.0;
            rr[r] = t;
        }
    }
}

template <typename T, int DIM, int KIND>
void cg_run(const Grid& g, const Coef<T>& c, T* x, const T* f, int nrhs, int steps, bool x_zero, const CgWork& w,
            hipStream_t st) {
    constexpr int RB = rhs_block<DIM, KIND>();
    const dim3 blk(CX, CY);
    const int ngrp = (nrhs + RB - 1) / RB;
    const int ngu = (nrhs + UB - 1) / UB;
    const dim3 grid((g.m + CX - 1) / CX, (g.m + CY - 1) / CY, DIM == 2 ? ngu : g.m * ngu);
    const dim3 grid_op(grid.x, grid.y, DIM == 2 ? ngrp : g.m * ngrp);
    const long nblk = (long)grid.x * grid.y * (DIM == 2 ? 1 : g.m);
    const long sd = g.plane;
    T* r = static_cast<T*>(w.r);
    T* pa = static_cast<T*>(w.pa);
    T* pb = static_cast<T*>(w.pb);
    T* q = static_cast<T*>(w.q);
    if (x_zero)
        hipLaunchKernelGGL((k_cg_start<T, DIM, KIND, true>), grid, blk, 0, st, g, c, x, f, r, w.partial, sd, nblk,
                           nrhs);
    else
        hipLaunchKernelGGL((k_cg_start<T, DIM, KIND, false>), grid_op, blk, 0, st, g, c, x, f, r, w.partial, sd,
                           nblk, nrhs);
    hipLaunchKernelGGL(k_cg_reduce<0>, dim3(nrhs), dim3(256), 0, st, w.partial, nblk, w.rr, (double*)nullptr);
    // 15-point operators: the direction pass marching along z
    constexpr bool ZM = DIM == 3 && KIND == 3;
    const int nzc = (g.m + ZC - 1) / ZC;
    const dim3 grid_z((g.m + ZX - 1) / ZX, (g.m + ZY - 1) / ZY, nzc * ngrp);
    const long nblk_z = (long)grid_z.x * grid_z.y * nzc;
    for (int s = 0; s < steps; ++s) {
        if constexpr (ZM) {
            if (s == 0)
                hipLaunchKernelGGL((k_cg_dir_z<T, true, RB>), grid_z, blk, 0, st, g, c, r, pb, w.beta, pa, q,
                                   w.partial, sd, nblk_z, nrhs, nzc);
            else
                hipLaunchKernelGGL((k_cg_dir_z<T, false, RB>), grid_z, blk, 0, st, g, c, r, pb, w.beta, pa, q,
                                   w.partial, sd, nblk_z, nrhs, nzc);
        } else {
            if (s == 0)
                hipLaunchKernelGGL((k_cg_dir<T, DIM, KIND, true>), grid_op, blk, 0, st, g, c, r, pb, w.beta, pa, q,
                                   w.partial, sd, nblk, nrhs);
            else
                hipLaunchKernelGGL((k_cg_dir<T, DIM, KIND, false>), grid_op, blk, 0, st, g, c, r, pb, w.beta, pa, q,
                                   w.partial, sd, nblk, nrhs);
        }
        hipLaunchKernelGGL(k_cg_reduce<1>, dim3(nrhs), dim3(256), 0, st, w.partial, ZM ? nblk_z : nblk, w.rr,
                           w.alpha);
        const bool last = s == steps - 1, xz = x_zero && s == 0;
        if (last) {
            if (xz)
                hipLaunchKernelGGL((k_cg_update<T, DIM, false, true>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk, nrhs);
            else
                hipLaunchKernelGGL((k_cg_update<T, DIM, false, false>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk, nrhs);
        } else {
            if (xz)
                hipLaunchKernelGGL((k_cg_update<T, DIM, true, true>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk, nrhs);
            else
                hipLaunchKernelGGL((k_cg_update<T, DIM, true, false>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk, nrhs);
            hipLaunchKernelGGL(k_cg_reduce<2>, dim3(nrhs), dim3(256), 0, st, w.partial, nblk, w.rr, w.beta);
        }
        std::swap(pa, pb);  // the new direction is the old one of the next step
    }
    PASM_CHECK_LAUNCH();
}

}  // namespace

long cg_partials(const Grid& g) {
    const long gx = (g.m + CX - 1) / CX, gy = (g.m + CY - 1) / CY;
    return gx * gy * (g.dim == 2 ? 1 : g.m);
}

template <typename T>
void cg_smooth(const Grid& g, const Coef<T>& c, T* x, const T* f, int nrhs, int steps, bool x_zero, const CgWork& w,
               hipStream_t st) {
    if (steps <= 0) return;
    if (c.kpm > 1 || c.ms != 0) throw Error(PASM_E_INVALID, "CG smoothing: single problems only");
    const int kind = coef_kind(c);
    if (g.dim == 2) {
        if (kind == 0) cg_run<T, 2, 0>(g, c, x, f, nrhs, steps, x_zero, w, st);
        else if (kind == 1) cg_run<T, 2, 1>(g, c, x, f, nrhs, steps, x_zero, w, st);
        else cg_run<T, 2, 2>(g, c, x, f, nrhs, steps, x_zero, w, st);
    } else {
        if (kind == 0) cg_run<T, 3, 0>(g, c, x, f, nrhs, steps, x_zero, w, st);
        else if (kind == 1) cg_run<T, 3, 1>(g, c, x, f, nrhs, steps, x_zero, w, st);
        else if (kind == 3) cg_run<T, 3, 3>(g, c, x, f, nrhs, steps, x_zero, w, st);
        else throw Error(PASM_E_INVALID, "CG smoothing: unknown 3D operator");
    }
}

template void cg_smooth<double>(const Grid&, const Coef<double>&, double*, const double*, int, int, bool,
                                const CgWork&, hipStream_t);
template void cg_smooth<float>(const Grid&, const Coef<float>&, float*, const float*, int, int, bool, const CgWork&,
                               hipStream_t);

}  // namespace pasm

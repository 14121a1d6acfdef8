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

struct NodeIdx {
    long id;    // padded index of the node in its plane / volume
    int r;      // right-hand side
    long blk;   // workgroup index within the right-hand side
    bool ok;    // an interior node
};

template <int DIM>
__device__ inline NodeIdx node_of(const Grid& g) {
    NodeIdx n;
    const int i = blockIdx.x * CX + threadIdx.x + 1;
    const int j = blockIdx.y * CY + threadIdx.y + 1;
    int l = 0;
    if (DIM == 2) {
        n.r = blockIdx.z;
        n.blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
    } else {
        l = blockIdx.z % g.m + 1;
        n.r = blockIdx.z / g.m;
        n.blk = ((long)(l - 1) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    }
    n.ok = i <= g.m && j <= g.m;
    n.id = DIM == 2 ? g.idx(i, j) : g.idx(i, j, l);
    return n;
}

// (A v)(id) for the level operator, v given as a callable of the padded
// index (so that v can be formed on the fly).  KIND: 0 constant coefficient
// (w0 times the 5- or 7-point Laplacian), 1 edge weights, 2 general 2D
// 7-point stencil (diagonal, edge weights and the "/" diagonal weight).
template <typename T, int DIM, int KIND, typename V>
__device__ inline T apply_op(const Grid& g, const Coef<T>& c, long id, V v) {
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    const T x0 = v(id);
    if (DIM == 2) {
        if (KIND == 0) return c.w0 * (T(4) * x0 - v(id + 1) - v(id - 1) - v(id + py) - v(id - py));
        const T we = c.wx[id], ww = c.wx[id - 1], wn = c.wy[id], ws = c.wy[id - py];
        if (KIND == 1)
            return we * (x0 - v(id + 1)) + ww * (x0 - v(id - 1)) + wn * (x0 - v(id + py)) + ws * (x0 - v(id - py));
        return c.d[id] * x0 - we * v(id + 1) - ww * v(id - 1) - wn * v(id + py) - ws * v(id - py) -
               c.wne[id] * v(id + py + 1) - c.wne[id - py - 1] * v(id - py - 1);
    } else {
        if (KIND == 0)
            return c.w0 * (T(6) * x0 - v(id + 1) - v(id - 1) - v(id + py) - v(id - py) - v(id + pz) - v(id - pz));
        if (KIND == 3) {
            // the 15-point operator: diagonal plane, then A(i, i + o) for the
            // seven Kuhn edge directions o
            const long P = g.plane;
            const long o7[7] = {1, py, pz, 1 + py, 1 + pz, py + pz, 1 + py + pz};
            T acc = c.s15[id] * x0;
#pragma unroll
            for (int t = 0; t < 7; ++t)
                acc += c.s15[(t + 1) * P + id] * v(id + o7[t]) + c.s15[(t + 1) * P + id - o7[t]] * v(id - o7[t]);
            return acc;
        }
        const T w1 = c.wx[id], w2 = c.wx[id - 1], w3 = c.wy[id], w4 = c.wy[id - py], w5 = c.wz[id],
                w6 = c.wz[id - pz];
        return w1 * (x0 - v(id + 1)) + w2 * (x0 - v(id - 1)) + w3 * (x0 - v(id + py)) + w4 * (x0 - v(id - py)) +
               w5 * (x0 - v(id + pz)) + w6 * (x0 - v(id - pz));
    }
}

// Sum of one double per thread over the workgroup (fixed order), stored by
// thread 0 at out.
__device__ inline void block_partial(double v, double* out) {
    __shared__ double sh[CX * CY / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int t = threadIdx.y * CX + threadIdx.x;
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < CX * CY / 64; ++w) s += sh[w];
        *out = s;
    }
}

// r = f - A x (XZ: x = 0, r = f); partial sums of r.r
template <typename T, int DIM, int KIND, bool XZ>
__global__ __launch_bounds__(CX* CY) void k_cg_start(Grid g, Coef<T> c, const T* __restrict__ x,
                                                     const T* __restrict__ f, T* __restrict__ r,
                                                     double* __restrict__ partial, long stride, long nblk) {
    const NodeIdx n = node_of<DIM>(g);
    const long off = (long)n.r * stride;
    double acc = 0.0;
    if (n.ok) {
        T rv = f[off + n.id];
        if (!XZ) {
            const T* xr = x + off;
            rv -= apply_op<T, DIM, KIND>(g, c, n.id, [&](long q) { return xr[q]; });
        }
        r[off + n.id] = rv;
        acc = (double)rv * (double)rv;
    }
    block_partial(acc, partial + (long)n.r * nblk + n.blk);
}

// p_new = r + beta p_old (FIRST: p_new = r), q = A p_new; partial sums of p_new.q
template <typename T, int DIM, int KIND, bool FIRST>
__global__ __launch_bounds__(CX* CY) void k_cg_dir(Grid g, Coef<T> c, const T* __restrict__ r,
                                                   const T* __restrict__ pold, const double* __restrict__ beta,
                                                   T* __restrict__ pnew, T* __restrict__ q,
                                                   double* __restrict__ partial, long stride, long nblk) {
    const NodeIdx n = node_of<DIM>(g);
    const long off = (long)n.r * stride;
    double acc = 0.0;
    if (n.ok) {
        const T* rr = r + off;
        const T* po = pold + off;
        const T b = FIRST ? T(0) : (T)beta[n.r];
        auto pv = [&](long k) { return FIRST ? rr[k] : rr[k] + b * po[k]; };
        const T p0 = pv(n.id);
        const T qv = apply_op<T, DIM, KIND>(g, c, n.id, pv);
        pnew[off + n.id] = p0;
        q[off + n.id] = qv;
        acc = (double)p0 * (double)qv;
    }
    block_partial(acc, partial + (long)n.r * nblk + n.blk);
}

// x += alpha p (XZ: x = alpha p); with RR also r -= alpha q and partial sums of r.r
template <typename T, int DIM, bool RR, bool XZ>
__global__ __launch_bounds__(CX* CY) void k_cg_update(Grid g, T* __restrict__ x, T* __restrict__ r,
                                                      const T* __restrict__ p, const T* __restrict__ q,
                                                      const double* __restrict__ alpha, double* __restrict__ partial,
                                                      long stride, long nblk) {
    const NodeIdx n = node_of<DIM>(g);
    const long off = (long)n.r * stride;
    double acc = 0.0;
    if (n.ok) {
        const T a = (T)alpha[n.r];
        const long k = off + n.id;
        x[k] = XZ ? a * p[k] : x[k] + a * p[k];
        if (RR) {
            const T rv = r[k] - a * q[k];
            r[k] = rv;
            acc = (double)rv * (double)rv;
        }
    }
    if (RR) block_partial(acc, partial + (long)n.r * nblk + n.blk);
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
    const dim3 blk(CX, CY);
    const dim3 grid((g.m + CX - 1) / CX, (g.m + CY - 1) / CY, DIM == 2 ? nrhs : g.m * nrhs);
    const long nblk = (long)grid.x * grid.y * (DIM == 2 ? 1 : g.m);
    const long sd = g.plane;
    T* r = static_cast<T*>(w.r);
    T* pa = static_cast<T*>(w.pa);
    T* pb = static_cast<T*>(w.pb);
    T* q = static_cast<T*>(w.q);
    if (x_zero)
        hipLaunchKernelGGL((k_cg_start<T, DIM, KIND, true>), grid, blk, 0, st, g, c, x, f, r, w.partial, sd, nblk);
    else
        hipLaunchKernelGGL((k_cg_start<T, DIM, KIND, false>), grid, blk, 0, st, g, c, x, f, r, w.partial, sd, nblk);
    hipLaunchKernelGGL(k_cg_reduce<0>, dim3(nrhs), dim3(256), 0, st, w.partial, nblk, w.rr, (double*)nullptr);
    for (int s = 0; s < steps; ++s) {
        if (s == 0)
            hipLaunchKernelGGL((k_cg_dir<T, DIM, KIND, true>), grid, blk, 0, st, g, c, r, pb, w.beta, pa, q, w.partial,
                               sd, nblk);
        else
            hipLaunchKernelGGL((k_cg_dir<T, DIM, KIND, false>), grid, blk, 0, st, g, c, r, pb, w.beta, pa, q,
                               w.partial, sd, nblk);
        hipLaunchKernelGGL(k_cg_reduce<1>, dim3(nrhs), dim3(256), 0, st, w.partial, nblk, w.rr, w.alpha);
        const bool last = s == steps - 1, xz = x_zero && s == 0;
        if (last) {
            if (xz)
                hipLaunchKernelGGL((k_cg_update<T, DIM, false, true>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk);
            else
                hipLaunchKernelGGL((k_cg_update<T, DIM, false, false>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk);
        } else {
            if (xz)
                hipLaunchKernelGGL((k_cg_update<T, DIM, true, true>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk);
            else
                hipLaunchKernelGGL((k_cg_update<T, DIM, true, false>), grid, blk, 0, st, g, x, r, pa, q, w.alpha,
                                   w.partial, sd, nblk);
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

// Matrix-free P1 operators and transfers on the Kuhn tetrahedral mesh (six
// tetrahedra per cube sharing the main diagonal), for all right-hand sides.
//
// With constant kappa the stiffness is h * (6 at the centre, -1 at the six axis
// neighbours): every non-axis edge coupling of a Kuhn tetrahedron cancels when
// the 24 tetrahedra around a node are summed.  The mass matrix, |T|(1+delta)/20
// per tetrahedron, gives h^3 * (2/5 at the centre, 1/20 on the six axis
// neighbours, 1/30 on the six face diagonals +-(1,1,0), +-(1,0,1), +-(0,1,1),
// 1/20 on the two body diagonals +-(1,1,1)).  These follow from the element
// integrals of Section 2 on this mesh.
// Prolongation: a fine node (2I,2J,2L) + o, o in {0,1}^3 \ 0, is the midpoint
// of the coarse edge from (I,J,L) to (I,J,L) + o (every such o is an edge
// direction of the Kuhn mesh), so it takes the mean of those two coarse nodes.
//
// Launch shape: 64 x 4 threads over (x, y); grid.z enumerates (z-plane, rhs).
#include "common.h"

namespace pasm {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

inline dim3 grid3(int m, int nrhs) { return dim3((m + BX - 1) / BX, (m + BY - 1) / BY, m * nrhs); }

struct Pos {
    int i, j, l, r;
    bool ok;
};
__device__ inline Pos pos3(int m) {
    Pos p;
    p.i = blockIdx.x * BX + threadIdx.x + 1;
    p.j = blockIdx.y * BY + threadIdx.y + 1;
    p.l = blockIdx.z % m + 1;
    p.r = blockIdx.z / m;
    p.ok = p.i <= m && p.j <= m;
    return p;
}

template <typename T, bool CONST>
__device__ inline void stiff3(const Grid& g, const Coef<T>& c, const T* __restrict__ x, long id, T& Ax, T& D) {
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    const T x0 = x[id];
    const T s = x[id + 1] + x[id - 1] + x[id + py] + x[id - py] + x[id + pz] + x[id - pz];
    if (CONST) {
        D = T(6) * c.w0;
        Ax = c.w0 * (T(6) * x0 - s);
    } else {
        const T w1 = c.wx[id], w2 = c.wx[id - 1], w3 = c.wy[id], w4 = c.wy[id - py], w5 = c.wz[id],
                w6 = c.wz[id - pz];
        D = w1 + w2 + w3 + w4 + w5 + w6;
        Ax = D * x0 - w1 * x[id + 1] - w2 * x[id - 1] - w3 * x[id + py] - w4 * x[id - py] -
             w5 * x[id + pz] - w6 * x[id - pz];
    }
}

template <typename T, bool CONST>
__device__ inline T diag3(const Grid& g, const Coef<T>& c, long id) {
    if (CONST) return T(6) * c.w0;
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    return c.wx[id] + c.wx[id - 1] + c.wy[id] + c.wy[id - py] + c.wz[id] + c.wz[id - pz];
}

template <typename T, bool CONST>
__global__ __launch_bounds__(BX* BY) void k_smooth3(Grid g, Coef<T> c, const T* __restrict__ xc, const T* xp,
                                                    const T* __restrict__ f, T* xn, long stride, T a, T b,
                                                    int zmode) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long off = (long)p.r * stride;
    const long id = g.idx(p.i, p.j, p.l);
    const T fv = f[off + id];
    if (zmode & 1) {
        xn[off + id] = b * fv / diag3<T, CONST>(g, c, id);
        return;
    }
    T Ax, D;
    stiff3<T, CONST>(g, c, xc + off, id, Ax, D);
    const T x0 = xc[off + id];
    T v = x0 + b * (fv - Ax) / D;
    if (a != T(0)) v += a * (x0 - ((zmode & 2) ? T(0) : xp[off + id]));
    xn[off + id] = v;
}

template <typename T, bool CONST>
__global__ __launch_bounds__(BX* BY) void k_apply_A3(Grid g, Coef<T> c, const T* __restrict__ x,
                                                     T* __restrict__ y, long stride) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long off = (long)p.r * stride;
    const long id = g.idx(p.i, p.j, p.l);
    T Ax, D;
    stiff3<T, CONST>(g, c, x + off, id, Ax, D);
    y[off + id] = Ax;
}

// The 14 fine neighbours (+-o for the 7 nonzero o in {0,1}^3) of a fine node.
__device__ inline long nb_off(const Grid& g, int t) {
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    const int o = (t >> 1) + 1;  // 1..7
    const long d = (o & 1 ? 1 : 0) + (o & 2 ? py : 0) + (o & 4 ? pz : 0);
    return (t & 1) ? -d : d;
}

template <typename T, bool CONST>
__global__ __launch_bounds__(BX* BY) void k_resid_restrict3(Grid gf, Coef<T> c, const T* __restrict__ x,
                                                            const T* __restrict__ f, Grid gc,
                                                            T* __restrict__ rc, long sf, long sc) {
    const Pos p = pos3(gc.m);
    if (!p.ok) return;
    const T* xr = x + (long)p.r * sf;
    const T* fr = f + (long)p.r * sf;
    const long id0 = gf.idx(2 * p.i, 2 * p.j, 2 * p.l);
    auto res = [&](long id) -> T {
        T Ax, D;
        stiff3<T, CONST>(gf, c, xr, id, Ax, D);
        return fr[id] - Ax;
    };
    T s = T(0);
#pragma unroll
    for (int t = 0; t < 14; ++t) s += res(id0 + nb_off(gf, t));
    rc[(long)p.r * sc + gc.idx(p.i, p.j, p.l)] = res(id0) + T(0.5) * s;
}

template <typename T>
__global__ __launch_bounds__(BX* BY) void k_restrict3(Grid gf, const T* __restrict__ xf, Grid gc,
                                                      T* __restrict__ xc, long sf, long sc) {
    const Pos p = pos3(gc.m);
    if (!p.ok) return;
    const T* xr = xf + (long)p.r * sf;
    const long id0 = gf.idx(2 * p.i, 2 * p.j, 2 * p.l);
    T s = T(0);
#pragma unroll
    for (int t = 0; t < 14; ++t) s += xr[id0 + nb_off(gf, t)];
    xc[(long)p.r * sc + gc.idx(p.i, p.j, p.l)] = xr[id0] + T(0.5) * s;
}

// Restriction through an LDS tile: a workgroup owns 8 x 8 x 4 coarse nodes,
// stages x on the 19 x 19 x 11 fine nodes around them once, forms the fine
// values v on the 17 x 17 x 9 nodes their restriction reaches, and restricts
// from LDS (centre 1, the 14 Kuhn-edge neighbours 1/2).
//   MODE 0: v = f - A x (the residual restriction of a V-cycle);
//   MODE 1 (double): v = A u and w = M u, both restricted, and the sums u.Au,
//           u.Mu over the workgroup's own fine nodes (the first 16 x 16 x 8 of
//           the 17 x 17 x 9; coarse nodes up to nc over the grid, so every
//           fine interior node is counted once), one pair per workgroup.
constexpr int RCX = 8, RCY = 8, RCZ = 4;                                 // coarse nodes per workgroup
constexpr int RFX = 2 * RCX + 1, RFY = 2 * RCY + 1, RFZ = 2 * RCZ + 1;   // fine nodes with values
constexpr int RUX = RFX + 2, RUY = RFY + 2, RUZ = RFZ + 2;               // fine nodes of x (halo 1)
// ADD (MODE 1): x is the V-cycles' iterate before its last correction; the
// tile holds x + ecor (the FP32 correction, added in FP64) and the own nodes
// of the corrected field are written to xout (which must not alias x).
// Threads per workgroup: the border mode's FP64 tiles take 73 KB of LDS, two
// workgroups per compute unit, so it runs 512 threads each to keep as many
// wavefronts resident as the residual mode.
template <int MODE>
constexpr int tile3_threads() { return MODE == 1 ? 512 : 256; }
template <typename T, int MODE, bool CONST, bool ADD = false>
__global__ __launch_bounds__(tile3_threads<MODE>()) void k_tile_restrict3(Grid gf, Coef<T> c, const T* __restrict__ x,
                                                        const T* __restrict__ f, Grid gc, T* __restrict__ oc,
                                                        T* __restrict__ oc2, double* __restrict__ partial, long sf,
                                                        long sc, int zblocks, const float* __restrict__ ecor,
                                                        T* __restrict__ xout) {
    static_assert(!ADD || MODE == 1, "the correction is added in the border mode only");
    constexpr int TB = tile3_threads<MODE>();
    constexpr int NU = RUX * RUY * RUZ, NV = RFX * RFY * RFZ, NPT = (NU + TB - 1) / TB;
    __shared__ T us[NU];
    __shared__ T vs[NV];
    __shared__ T ws[MODE == 1 ? NV : 1];
    __shared__ double sh[2 * TB / 64];
    const int tid = threadIdx.x;
    const int zb = blockIdx.z % zblocks, r = blockIdx.z / zblocks;
    const int I0 = blockIdx.x * RCX + 1, J0 = blockIdx.y * RCY + 1, K0 = zb * RCZ + 1;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1, fk0 = 2 * K0 - 1;  // first fine node with a value
    const T* xr = x + (long)r * sf;
    const long py = gf.pitch, pz = (long)gf.pitch * (gf.n + 1);
    {
        T v[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int t = tid + TB * e;
            const int a = t % RUX, b = (t / RUX) % RUY, cz = t / (RUX * RUY);
            const int i = min(fi0 - 1 + a, gf.n), j = min(fj0 - 1 + b, gf.n), k = min(fk0 - 1 + cz, gf.n);
            v[e] = xr[gf.idx(i, j, k)];
            if constexpr (ADD) v[e] += (T)ecor[(long)r * sf + gf.idx(i, j, k)];
            if (t >= NU || fi0 - 1 + a > gf.n || fj0 - 1 + b > gf.n || fk0 - 1 + cz > gf.n) v[e] = T(0);
        }
#pragma unroll
        for (int e = 0; e < NPT; ++e)
            if (tid + TB * e < NU) us[tid + TB * e] = v[e];
    }
    __syncthreads();
    const T* fr = MODE == 0 ? f + (long)r * sf : nullptr;
    double ua = 0.0, um = 0.0;
    const double h3 = gf.h * gf.h * gf.h;
    for (int t = tid; t < NV; t += TB) {
        const int a = t % RFX, b = (t / RFX) % RFY, cz = t / (RFX * RFY);
        const int i = fi0 + a, j = fj0 + b, k = fk0 + cz;
        T val = T(0), wal = T(0);
        if (i <= gf.m && j <= gf.m && k <= gf.m) {
            const int q = ((cz + 1) * RUY + (b + 1)) * RUX + (a + 1);
            constexpr int QY = RUX, QZ = RUX * RUY;
            const T x0 = us[q];
            const T xe = us[q + 1], xw = us[q - 1], xn = us[q + QY], xs = us[q - QY], xu = us[q + QZ], xd = us[q - QZ];
            T Ax;
            if (CONST) {
                Ax = c.w0 * (T(6) * x0 - (xe + xw + xn + xs + xu + xd));
            } else {
                const long id = gf.idx(i, j, k);
                const T w1 = c.wx[id], w2 = c.wx[id - 1], w3 = c.wy[id], w4 = c.wy[id - py], w5 = c.wz[id],
                        w6 = c.wz[id - pz];
                Ax = (w1 + w2 + w3 + w4 + w5 + w6) * x0 - w1 * xe - w2 * xw - w3 * xn - w4 * xs - w5 * xu - w6 * xd;
            }
            if (MODE == 0) {
                val = fr[gf.idx(i, j, k)] - Ax;
            } else {
                const T ax = xe + xw + xn + xs + xu + xd;
                const T fd = us[q + 1 + QY] + us[q - 1 - QY] + us[q + 1 + QZ] + us[q - 1 - QZ] + us[q + QY + QZ] +
                             us[q - QY - QZ];
                const T bd = us[q + 1 + QY + QZ] + us[q - 1 - QY - QZ];
                val = Ax;
                wal = (T)h3 * (T(0.4) * x0 + (ax + bd) * T(1.0 / 20.0) + fd * T(1.0 / 30.0));
                if (a < 2 * RCX && b < 2 * RCY && cz < 2 * RCZ) {  // own node
                    ua += (double)(x0 * val);
                    um += (double)(x0 * wal);
                    if constexpr (ADD) xout[(long)r * sf + gf.idx(i, j, k)] = x0;
                }
            }
        }
        vs[t] = val;
        if (MODE == 1) ws[t] = wal;
    }
    __syncthreads();
    {
        const int cx = tid % RCX, cy = (tid / RCX) % RCY, cz = tid / (RCX * RCY);
        const int I = I0 + cx, J = J0 + cy, K = K0 + cz;
        if (cz < RCZ && I <= gc.m && J <= gc.m && K <= gc.m) {
            const int q = ((2 * cz + 1) * RFY + (2 * cy + 1)) * RFX + (2 * cx + 1);
            T sv = T(0), sw = T(0);
#pragma unroll
            for (int t = 0; t < 14; ++t) {
                const int o = (t >> 1) + 1;
                const int d = ((o & 1) ? 1 : 0) + ((o & 2) ? RFX : 0) + ((o & 4) ? RFX * RFY : 0);
                const int qq = (t & 1) ? q - d : q + d;
                sv += vs[qq];
                if (MODE == 1) sw += ws[qq];
            }
            const long cid = (long)r * sc + gc.idx(I, J, K);
            oc[cid] = vs[q] + T(0.5) * sv;
            if (MODE == 1) oc2[cid] = ws[q] + T(0.5) * sw;
        }
    }
    if (MODE == 1) {
        for (int o = 32; o > 0; o >>= 1) {
            ua += __shfl_down(ua, o, 64);
            um += __shfl_down(um, o, 64);
        }
        if ((tid & 63) == 0) {
            sh[2 * (tid >> 6)] = ua;
            sh[2 * (tid >> 6) + 1] = um;
        }
        __syncthreads();
        if (tid == 0) {
            const long per = (long)gridDim.x * gridDim.y * zblocks;  // workgroups per right-hand side
            const long b = (long)r * per + ((long)zb * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            double sa = 0.0, sm = 0.0;
#pragma unroll
            for (int w = 0; w < TB / 64; ++w) {
                sa += sh[2 * w];
                sm += sh[2 * w + 1];
            }
            partial[2 * b] = sa;
            partial[2 * b + 1] = sm;
        }
    }
}

// Residual restriction marching along z (3D, constant coefficients): a
// workgroup owns ZTX x ZTY coarse nodes in x, y and a chunk of ZKC coarse
// planes, and walks the fine planes of the chunk upwards.  It keeps the last
// three fine planes of x (with a one-node halo) and of the residual in LDS
// rings, so every x plane is read once per chunk (plus its x-y halo and the
// chunk's two extra planes) instead of the 1.9x of a staged cube.  Per fine
// plane p: x of plane p + 1 enters the ring (loaded one plane ahead into
// registers), the residual r = f - A x of plane p is formed, and when p is
// odd the coarse plane (p - 1) / 2 is restricted from the residual planes
// p - 2, p - 1, p (centre 1, the 14 Kuhn-edge neighbours 1/2), with the
// arithmetic, in the same order, of k_tile_restrict3's residual mode.
constexpr int ZTX = 16, ZTY = 16, ZKC = 8;                   // coarse nodes per workgroup
constexpr int ZRX = 2 * ZTX + 1, ZRY = 2 * ZTY + 1;           // fine residual nodes of a plane
constexpr int ZUX = ZRX + 2, ZUY = ZRY + 2;                   // fine x nodes of a plane (halo 1)
constexpr int ZNU = ZUX * ZUY, ZNR = ZRX * ZRY;
constexpr int ZPU = (ZNU + 255) / 256, ZPR = (ZNR + 255) / 256;
template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict3z(Grid gf, T w0, const T* __restrict__ x,
                                                          const T* __restrict__ f, Grid gc, T* __restrict__ rc,
                                                          long sf, long sc, int zchunks) {
    __shared__ T xs[3][ZNU];
    __shared__ T rs[3][ZNR];
    const int tid = threadIdx.x;
    const int zc = blockIdx.z % zchunks, r = blockIdx.z / zchunks;
    const int I0 = blockIdx.x * ZTX + 1, J0 = blockIdx.y * ZTY + 1;
    const int K0 = zc * ZKC + 1, K1 = min(K0 + ZKC, gc.m + 1);  // coarse planes [K0, K1)
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;                  // first fine residual node
    const T* xr = x + (long)r * sf;
    const T* fr = f + (long)r * sf;
    // per-thread positions of the x plane (clamped onto the grid: the
    // boundary ring holds zeros, positions past it are zeroed) and of the
    // residual plane
    long xo[ZPU];
    bool xin[ZPU];
#pragma unroll
    for (int e = 0; e < ZPU; ++e) {
        const int t = tid + 256 * e;
        const int i = fi0 - 1 + t % ZUX, j = fj0 - 1 + t / ZUX;
        xin[e] = t < ZNU && i <= gf.n && j <= gf.n;
        xo[e] = (long)min(j, gf.n) * gf.pitch + ORIGIN + min(i, gf.n);
    }
    long ro[ZPR];
    bool rin[ZPR];
    int rq[ZPR];
#pragma unroll
    for (int e = 0; e < ZPR; ++e) {
        const int t = tid + 256 * e;
        const int a = t % ZRX, b = t / ZRX;
        const int i = fi0 + a, j = fj0 + b;
        rin[e] = t < ZNR && i <= gf.m && j <= gf.m;
        ro[e] = (long)min(j, gf.n) * gf.pitch + ORIGIN + min(i, gf.n);
        rq[e] = (b + 1) * ZUX + (a + 1);  // the node in the x plane
    }
    const long pz = (long)gf.pitch * (gf.n + 1);
    auto load_x = [&](int k, T (&v)[ZPU]) {
        const long base = (long)min(max(k, 0), gf.n) * pz;
#pragma unroll
        for (int e = 0; e < ZPU; ++e) v[e] = xr[base + xo[e]];
#pragma unroll
        for (int e = 0; e < ZPU; ++e)
            if (!xin[e] || k < 0 || k > gf.n) v[e] = T(0);
    };
    auto load_f = [&](int k, T (&v)[ZPR]) {
        const long base = (long)min(max(k, 1), gf.m) * pz;
#pragma unroll
        for (int e = 0; e < ZPR; ++e) v[e] = fr[base + ro[e]];
    };
    auto store_x = [&](int slot, const T (&v)[ZPU]) {
#pragma unroll
        for (int e = 0; e < ZPU; ++e)
            if (tid + 256 * e < ZNU) xs[slot][tid + 256 * e] = v[e];
    };
    const int p0 = 2 * K0 - 1, p1 = 2 * K1 - 1;  // residual planes [p0, p1]
    T xa[ZPU], xb[ZPU], fv[ZPR], fn[ZPR];
    load_x(p0 - 1, xa);
    load_x(p0, xb);
    store_x((p0 - 1 + 3) % 3, xa);
    store_x(p0 % 3, xb);
    load_x(p0 + 1, xa);   // enters at the first plane
    load_f(p0, fv);
    for (int p = p0; p <= p1; ++p) {
        store_x((p + 1) % 3, xa);
        if (p + 2 <= p1 + 1) load_x(p + 2, xa);  // one plane ahead
        if (p + 1 <= p1) load_f(p + 1, fn);
        __syncthreads();
        // residual of plane p
        {
            const T* xm = xs[(p + 2) % 3];  // plane p - 1
            const T* x0 = xs[p % 3];
            const T* xp = xs[(p + 1) % 3];
            T* rp = rs[p % 3];
            const bool pin = p >= 1 && p <= gf.m;
#pragma unroll
            for (int e = 0; e < ZPR; ++e) {
                const int t = tid + 256 * e;
                if (t >= ZNR) break;
                const int q = rq[e];
                const T c = x0[q];
                const T Ax = w0 * (T(6) * c - (x0[q + 1] + x0[q - 1] + x0[q + ZUX] + x0[q - ZUX] + xp[q] + xm[q]));
                rp[t] = (pin && rin[e]) ? fv[e] - Ax : T(0);
            }
        }
        __syncthreads();
        if (p & 1 && p >= p0 + 2) {
            // coarse plane K = (p - 1) / 2 from residual planes p - 2, p - 1, p
            const int K = (p - 1) >> 1;
            const int cx = tid % ZTX, cy = tid / ZTX;
            const int I = I0 + cx, J = J0 + cy;
            if (I <= gc.m && J <= gc.m) {
                const T* rl[3] = {rs[(p + 1) % 3], rs[(p + 2) % 3], rs[p % 3]};  // planes p-2, p-1, p
                const int q = (2 * cy + 1) * ZRX + (2 * cx + 1);
                T sv = T(0);
#pragma unroll
                for (int t = 0; t < 14; ++t) {
                    const int o = (t >> 1) + 1;
                    const int dx = (o & 1) ? 1 : 0, dy = (o & 2) ? ZRX : 0, dz = (o & 4) ? 1 : 0;
                    const int dq = dx + dy;
                    sv += (t & 1) ? rl[1 - dz][q - dq] : rl[1 + dz][q + dq];
                }
                rc[(long)r * sc + gc.idx(I, J, K)] = rl[1][q] + T(0.5) * sv;
            }
        }
#pragma unroll
        for (int e = 0; e < ZPR; ++e) fv[e] = fn[e];
    }
}

// The borders of a correction step marching along z (3D, constant
// coefficients, FP64): A u and M u, their restrictions P^T A u, P^T M u to
// the next coarser grid, and the sums u.Au, u.Mu over each fine node once.
// A workgroup owns ZTX x ZTY coarse nodes (up to nc, whose fine nodes it owns
// for the sums) and ZKC coarse planes, keeps three fine planes of u (one-node
// halo) in an LDS ring and one plane of A u and M u; after each fine plane
// every thread adds that plane's share to the restrictions of its coarse
// node (centre plane 2K: the node and its six in-plane Kuhn neighbours; plane
// 2K - 1 and 2K + 1: the four neighbours along the edge directions with
// z component -1 and +1), and writes coarse plane K once plane 2K + 1 is in.
// ADD: the ring holds u + e (the last FP32 correction, added in FP64) and
// the own nodes of the corrected field are written to un.
template <bool ADD>
__global__ __launch_bounds__(256) void k_border3z(Grid gf, double w0, const double* __restrict__ u,
                                                  const float* __restrict__ e, double* __restrict__ un, Grid gc,
                                                  double* __restrict__ bc, double* __restrict__ cc,
                                                  double* __restrict__ partial, long sf, long sc, int zchunks) {
    __shared__ double xs[3][ZNU];
    __shared__ double va[ZNR], vm[ZNR];
    __shared__ double sh[8];
    const int tid = threadIdx.x;
    const int zc = blockIdx.z % zchunks, r = blockIdx.z / zchunks;
    const int I0 = blockIdx.x * ZTX + 1, J0 = blockIdx.y * ZTY + 1;
    const int K0 = zc * ZKC + 1, K1 = min(K0 + ZKC, gc.n + 1);  // coarse planes [K0, K1), up to nc
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;
    const double* xr = u + (long)r * sf;
    const float* er = ADD ? e + (long)r * sf : nullptr;
    long xo[ZPU];
    bool xin[ZPU];
#pragma unroll
    for (int q = 0; q < ZPU; ++q) {
        const int t = tid + 256 * q;
        const int i = fi0 - 1 + t % ZUX, j = fj0 - 1 + t / ZUX;
        xin[q] = t < ZNU && i <= gf.n && j <= gf.n;
        xo[q] = (long)min(j, gf.n) * gf.pitch + ORIGIN + min(i, gf.n);
    }
    const long pz = (long)gf.pitch * (gf.n + 1);
    auto load_x = [&](int k, double (&v)[ZPU]) {
        const long base = (long)min(max(k, 0), gf.n) * pz;
#pragma unroll
        for (int q = 0; q < ZPU; ++q) {
            v[q] = xr[base + xo[q]];
            if (ADD) v[q] += (double)er[base + xo[q]];
        }
#pragma unroll
        for (int q = 0; q < ZPU; ++q)
            if (!xin[q] || k < 0 || k > gf.n) v[q] = 0.0;
    };
    auto store_x = [&](int slot, const double (&v)[ZPU]) {
#pragma unroll
        for (int q = 0; q < ZPU; ++q)
            if (tid + 256 * q < ZNU) xs[slot][tid + 256 * q] = v[q];
    };
    const double h3 = gf.h * gf.h * gf.h;
    // this thread's coarse node and its running restrictions for the coarse
    // planes K (index 0) and K + 1 (index 1) around the current fine plane
    const int cx = tid % ZTX, cy = tid / ZTX;
    const int I = I0 + cx, J = J0 + cy;
    const int qc = (2 * cy + 1) * ZRX + (2 * cx + 1);
    double ba[2] = {0.0, 0.0}, bm[2] = {0.0, 0.0};
    double ua = 0.0, um = 0.0;
    const int p0 = 2 * K0 - 1, p1 = 2 * K1 - 1;
    const int own_hi = 2 * K1 - 2;  // own fine planes [p0, own_hi]
    double xa[ZPU], xb[ZPU];
    load_x(p0 - 1, xa);
    load_x(p0, xb);
    store_x((p0 - 1 + 3) % 3, xa);
    store_x(p0 % 3, xb);
    load_x(p0 + 1, xa);
    for (int p = p0; p <= p1; ++p) {
        store_x((p + 1) % 3, xa);
        if (p + 2 <= p1 + 1) load_x(p + 2, xa);
        __syncthreads();
        {
            const double* xm = xs[(p + 2) % 3];
            const double* x0 = xs[p % 3];
            const double* xp = xs[(p + 1) % 3];
            const bool pin = p >= 1 && p <= gf.m;
            for (int t = tid; t < ZNR; t += 256) {
                const int a = t % ZRX, b = t / ZRX;
                const int i = fi0 + a, j = fj0 + b;
                double Ax = 0.0, Mx = 0.0;
                if (pin && i <= gf.m && j <= gf.m) {
                    const int q = (b + 1) * ZUX + (a + 1);
                    const double c = x0[q];
                    const double xe = x0[q + 1], xw = x0[q - 1], xn = x0[q + ZUX], xsv = x0[q - ZUX], xu = xp[q],
                                 xd = xm[q];
                    Ax = w0 * (6.0 * c - (xe + xw + xn + xsv + xu + xd));
                    const double ax = xe + xw + xn + xsv + xu + xd;
                    const double fd = x0[q + 1 + ZUX] + x0[q - 1 - ZUX] + xp[q + 1] + xm[q - 1] + xp[q + ZUX] +
                                      xm[q - ZUX];
                    const double bd = xp[q + 1 + ZUX] + xm[q - 1 - ZUX];
                    Mx = h3 * (0.4 * c + (ax + bd) * (1.0 / 20.0) + fd * (1.0 / 30.0));
                    if (a < 2 * ZTX && b < 2 * ZTY && p <= own_hi) {  // own node
                        ua += c * Ax;
                        um += c * Mx;
                        if (ADD) un[(long)r * sf + (long)p * pz + (long)j * gf.pitch + ORIGIN + i] = c;
                    }
                }
                va[t] = Ax;
                vm[t] = Mx;
            }
        }
        __syncthreads();
        {
            // this plane's share of the restrictions
            const int dy = ZRX;
            if ((p & 1) == 0) {
                // centre plane of K = p / 2 (index 0)
                ba[0] += va[qc] + 0.5 * (va[qc + 1] + va[qc - 1] + va[qc + dy] + va[qc - dy] + va[qc + 1 + dy] +
                                         va[qc - 1 - dy]);
                bm[0] += vm[qc] + 0.5 * (vm[qc + 1] + vm[qc - 1] + vm[qc + dy] + vm[qc - dy] + vm[qc + 1 + dy] +
                                         vm[qc - 1 - dy]);
            } else {
                // upper plane of K = (p - 1) / 2 (index 0), lower plane of K + 1 (index 1)
                ba[0] += 0.5 * (va[qc] + va[qc + 1] + va[qc + dy] + va[qc + 1 + dy]);
                bm[0] += 0.5 * (vm[qc] + vm[qc + 1] + vm[qc + dy] + vm[qc + 1 + dy]);
                ba[1] += 0.5 * (va[qc] + va[qc - 1] + va[qc - dy] + va[qc - 1 - dy]);
                bm[1] += 0.5 * (vm[qc] + vm[qc - 1] + vm[qc - dy] + vm[qc - 1 - dy]);
                const int K = (p - 1) >> 1;
                if (K >= K0 && I <= gc.m && J <= gc.m && K <= gc.m) {
                    const long cid = (long)r * sc + gc.idx(I, J, K);
                    bc[cid] = ba[0];
                    cc[cid] = bm[0];
                }
                ba[0] = ba[1], bm[0] = bm[1];
                ba[1] = 0.0, bm[1] = 0.0;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        ua += __shfl_down(ua, o, 64);
        um += __shfl_down(um, o, 64);
    }
    if ((tid & 63) == 0) {
        sh[2 * (tid >> 6)] = ua;
        sh[2 * (tid >> 6) + 1] = um;
    }
    __syncthreads();
    if (tid == 0) {
        const long per = (long)gridDim.x * gridDim.y * zchunks;  // workgroups per right-hand side
        const long b = (long)r * per + ((long)zc * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[2 * b] = sh[0] + sh[2] + sh[4] + sh[6];
        partial[2 * b + 1] = sh[1] + sh[3] + sh[5] + sh[7];
    }
}

// The FP64 residual of a mixed-precision step marching along z (3D,
// constant coefficients), with f = lam M u formed from u: r = lam M u - A x
// rounded to FP32, x = u (first cycle) or x = u + e (ADD: the first cycle's
// correction added in FP64, x written to un).  A workgroup owns 64 x 16 fine
// nodes of a chunk of ZRC fine planes and keeps three planes of u (and e)
// with a one-node halo in LDS rings; the arithmetic is that of
// k_resid_cast3 / k_add_resid3 with the mass term.
// PRO: u itself is formed in the ring, u = P q + beta u~ (q the coarse-space
// field on the next coarser grid, u~ the old field in the input, a zero beta
// dropping it), and written to un: the prolongation of a correction step and
// the next step's first residual in one pass.
constexpr int ZFX = 64, ZFY = 16, ZRC = 32;
constexpr int ZQX = ZFX + 2, ZQY = ZFY + 2, ZNQ = ZQX * ZQY, ZPQ = (ZNQ + 255) / 256, ZPO = ZFX * ZFY / 256;
template <bool ADD, bool PRO = false>
__global__ __launch_bounds__(256) void k_resid3z(Grid g, double w0, const double* __restrict__ u,
                                                 const float* __restrict__ e, const double* __restrict__ lam,
                                                 double* __restrict__ un, float* __restrict__ r, long sf,
                                                 int zchunks, Grid gc, const double* __restrict__ xc, long sc,
                                                 const double* __restrict__ beta) {
    static_assert(!(ADD && PRO), "the prolonging pass starts a step");
    __shared__ double us[3][ZNQ];
    __shared__ float es[ADD ? 3 : 1][ADD ? ZNQ : 1];
    const int tid = threadIdx.x;
    const int zc = blockIdx.z % zchunks, z = blockIdx.z / zchunks;
    const int i0 = blockIdx.x * ZFX + 1, j0 = blockIdx.y * ZFY + 1;
    const int k0 = zc * ZRC + 1, k1 = min(k0 + ZRC, g.m + 1);  // fine planes [k0, k1)
    const double* ur = u + (long)z * sf;
    const float* er = ADD ? e + (long)z * sf : nullptr;
    const double lz = lam[z];
    long qo[ZPQ];
    bool qin[ZPQ];
    int qi[ZPQ], qj[ZPQ];
#pragma unroll
    for (int q = 0; q < ZPQ; ++q) {
        const int t = tid + 256 * q;
        const int i = i0 - 1 + t % ZQX, j = j0 - 1 + t / ZQX;
        qin[q] = t < ZNQ && i <= g.n && j <= g.n;
        qi[q] = min(i, g.n);
        qj[q] = min(j, g.n);
        qo[q] = (long)qj[q] * g.pitch + ORIGIN + qi[q];
    }
    const long pz = (long)g.pitch * (g.n + 1);
    const double* cr = PRO ? xc + (long)z * sc : nullptr;
    const double bz = PRO ? beta[z] : 0.0;
    const long cpz = (long)gc.pitch * (gc.n + 1);
    auto load = [&](int k, double (&vu)[ZPQ], float (&ve)[ZPQ]) {
        const int kc = min(max(k, 0), g.n);
        const long base = (long)kc * pz;
#pragma unroll
        for (int q = 0; q < ZPQ; ++q) {
            vu[q] = ur[base + qo[q]];
            if (ADD) ve[q] = er[base + qo[q]];
        }
        if constexpr (PRO) {
            // the nodal interpolation: the coarse node, or the mean of the
            // two ends of the coarse Kuhn edge the fine node halves
#pragma unroll
            for (int q = 0; q < ZPQ; ++q) {
                const int i = qi[q], j = qj[q];
                const long cid = gc.idx(i >> 1, j >> 1, kc >> 1);
                double v = cr[cid];
                if ((i | j | kc) & 1)
                    v = 0.5 * (v + cr[cid + (i & 1) + (long)(j & 1) * gc.pitch + (long)(kc & 1) * cpz]);
                if (bz != 0.0) v += bz * vu[q];
                vu[q] = v;
            }
        }
#pragma unroll
        for (int q = 0; q < ZPQ; ++q)
            if (!qin[q] || k > g.n || (PRO && (qi[q] < 1 || qj[q] < 1 || qi[q] > g.m || qj[q] > g.m || kc < 1 ||
                                               kc > g.m)))
                vu[q] = 0.0, ve[q] = 0.0f;
    };
    auto store = [&](int slot, const double (&vu)[ZPQ], const float (&ve)[ZPQ]) {
#pragma unroll
        for (int q = 0; q < ZPQ; ++q)
            if (tid + 256 * q < ZNQ) {
                us[slot][tid + 256 * q] = vu[q];
                if (ADD) es[slot][tid + 256 * q] = ve[q];
            }
    };
    const double h3 = g.h * g.h * g.h;
    double au[ZPQ], bu[ZPQ];
    float ae[ZPQ], be[ZPQ];
    load(k0 - 1, au, ae);
    load(k0, bu, be);
    store((k0 - 1) % 3, au, ae);
    store(k0 % 3, bu, be);
    load(k0 + 1, au, ae);
    for (int p = k0; p < k1; ++p) {
        store((p + 1) % 3, au, ae);
        if (p + 1 < k1) load(p + 2, au, ae);  // one plane ahead
        __syncthreads();
        const double* um = us[(p + 2) % 3];
        const double* u0 = us[p % 3];
        const double* up = us[(p + 1) % 3];
        const float* em = es[ADD ? (p + 2) % 3 : 0];
        const float* e0 = es[ADD ? p % 3 : 0];
        const float* ep = es[ADD ? (p + 1) % 3 : 0];
#pragma unroll
        for (int q = 0; q < ZPO; ++q) {
            const int t = tid + 256 * q;
            const int a = t % ZFX, b = t / ZFX;
            const int i = i0 + a, j = j0 + b;
            if (i > g.m || j > g.m) continue;
            const int c = (b + 1) * ZQX + (a + 1);
            // lam M u, the neighbours in the order of the mass kernels
            const double ax = u0[c + 1] + u0[c - 1] + u0[c + ZQX] + u0[c - ZQX] + up[c] + um[c];
            const double fd = u0[c + 1 + ZQX] + u0[c - 1 - ZQX] + up[c + 1] + um[c - 1] + up[c + ZQX] + um[c - ZQX];
            const double bd = up[c + 1 + ZQX] + um[c - 1 - ZQX];
            const double fv = lz * (h3 * (0.4 * u0[c] + (ax + bd) * (1.0 / 20.0) + fd * (1.0 / 30.0)));
            double x0 = u0[c], xe = u0[c + 1], xw = u0[c - 1], xn = u0[c + ZQX], xs = u0[c - ZQX], xu = up[c],
                   xd = um[c];
            if (ADD) {
                x0 += (double)e0[c], xe += (double)e0[c + 1], xw += (double)e0[c - 1], xn += (double)e0[c + ZQX];
                xs += (double)e0[c - ZQX], xu += (double)ep[c], xd += (double)em[c];
            }
            const double Ax = w0 * (6.0 * x0 - (xe + xw + xn + xs + xu + xd));
            const long id = (long)z * sf + (long)p * pz + (long)j * g.pitch + ORIGIN + i;
            if (ADD || PRO) un[id] = x0;
            r[id] = (float)(fv - Ax);
        }
        __syncthreads();
    }
}

// Prolongation and combination with the mass right-hand side of the next
// step (3D): xn = P xc + beta[r] xo on every fine node, and f = lam[r] M xn on
// the workgroup's 32 x 8 x 4 nodes (xn on their one-node halo is formed again
// from xo and xc).  xn must not alias xo.
constexpr int QMX = 32, QMY = 8, QMZ = 4;
__global__ __launch_bounds__(256) void k_prolong_mass3(Grid gc, const double* __restrict__ xc, Grid gf,
                                                       const double* __restrict__ xo, double* __restrict__ xn,
                                                       double* __restrict__ f, long sc, long sf,
                                                       const double* __restrict__ beta,
                                                       const double* __restrict__ lam, int zblocks) {
    constexpr int UX = QMX + 2, UY = QMY + 2, UZ = QMZ + 2, NU = UX * UY * UZ, NPT = (NU + 255) / 256;
    __shared__ double us[NU];
    const int tid = threadIdx.x;
    const int zb = blockIdx.z % zblocks, r = blockIdx.z / zblocks;
    const int i0 = blockIdx.x * QMX + 1, j0 = blockIdx.y * QMY + 1, k0 = zb * QMZ + 1;
    const double* cr = xc + (long)r * sc;
    const double* xr = xo + (long)r * sf;
    const double bz = beta[r], lz = lam[r];
    const long cpz = (long)gc.pitch * (gc.n + 1);
    {
        double c0[NPT], c1[NPT], xv[NPT];
        bool ok[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int t = tid + 256 * e;
            const int i = i0 - 1 + t % UX, j = j0 - 1 + (t / UX) % UY, k = k0 - 1 + t / (UX * UY);
            ok[e] = t < NU && i >= 1 && i <= gf.m && j >= 1 && j <= gf.m && k >= 1 && k <= gf.m;
            const int ic = ok[e] ? i : 1, jc = ok[e] ? j : 1, kc = ok[e] ? k : 1;
            const long cid = gc.idx(ic >> 1, jc >> 1, kc >> 1);
            c0[e] = cr[cid];
            c1[e] = cr[cid + (ic & 1) + (long)(jc & 1) * gc.pitch + (long)(kc & 1) * cpz];
            xv[e] = xr[gf.idx(ic, jc, kc)];
        }
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int t = tid + 256 * e;
            const int i = i0 - 1 + t % UX, j = j0 - 1 + (t / UX) % UY, k = k0 - 1 + t / (UX * UY);
            double v = c0[e];
            if ((i | j | k) & 1) v = 0.5 * (v + c1[e]);
            if (bz != 0.0) v += bz * xv[e];  // a zero weight drops the old field (whatever it holds)
            if (t < NU) us[t] = ok[e] ? v : 0.0;
        }
    }
    __syncthreads();
    const double h3 = gf.h * gf.h * gf.h;
    constexpr int QY = UX, QZ = UX * UY;
    for (int t = tid; t < QMX * QMY * QMZ; t += 256) {
        const int a = t % QMX, b = (t / QMX) % QMY, cz = t / (QMX * QMY);
        const int i = i0 + a, j = j0 + b, k = k0 + cz;
        if (i > gf.m || j > gf.m || k > gf.m) continue;
        const int q = ((cz + 1) * UY + (b + 1)) * UX + (a + 1);
        const double x0 = us[q];
        const double ax = us[q + 1] + us[q - 1] + us[q + QY] + us[q - QY] + us[q + QZ] + us[q - QZ];
        const double fd = us[q + 1 + QY] + us[q - 1 - QY] + us[q + 1 + QZ] + us[q - 1 - QZ] + us[q + QY + QZ] +
                          us[q - QY - QZ];
        const double bd = us[q + 1 + QY + QZ] + us[q - 1 - QY - QZ];
        const long id = (long)r * sf + gf.idx(i, j, k);
        xn[id] = x0;
        if (f) f[id] = lz * (h3 * (0.4 * x0 + (ax + bd) * (1.0 / 20.0) + fd * (1.0 / 30.0)));
    }
}

template <typename T>
__global__ __launch_bounds__(BX* BY) void k_prolong3(Grid gc, const T* __restrict__ xc, Grid gf,
                                                     T* __restrict__ xf, long sc, long sf, int mode,
                                                     const double* __restrict__ beta) {
    const Pos p = pos3(gf.m);
    if (!p.ok) return;
    const T* cr = xc + (long)p.r * sc;
    const int a = p.i & 1, b = p.j & 1, e = p.l & 1;
    const long cid = gc.idx(p.i >> 1, p.j >> 1, p.l >> 1);
    T v = cr[cid];
    if (a | b | e) v = T(0.5) * (v + cr[cid + a + (long)b * gc.pitch + (long)e * gc.pitch * (gc.n + 1)]);
    const long id = (long)p.r * sf + gf.idx(p.i, p.j, p.l);
    if (mode == 1) v += xf[id];
    else if (mode == 2 && beta[p.r] != 0.0) v += T(beta[p.r]) * xf[id];  // a zero weight drops the old field
    xf[id] = v;
}

__device__ inline double mass3(const Grid& g, const double* __restrict__ u, long id) {
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    const double ax = u[id + 1] + u[id - 1] + u[id + py] + u[id - py] + u[id + pz] + u[id - pz];
    const double fd = u[id + 1 + py] + u[id - 1 - py] + u[id + 1 + pz] + u[id - 1 - pz] + u[id + py + pz] +
                      u[id - py - pz];
    const double bd = u[id + 1 + py + pz] + u[id - 1 - py - pz];
    const double h3 = g.h * g.h * g.h;
    return h3 * (0.4 * u[id] + (ax + bd) * (1.0 / 20.0) + fd * (1.0 / 30.0));
}

__global__ __launch_bounds__(BX* BY) void k_mass_rhs3(Grid g, const double* __restrict__ u,
                                                      const double* __restrict__ lam, double* __restrict__ f,
                                                      long stride) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long off = (long)p.r * stride;
    const long id = g.idx(p.i, p.j, p.l);
    const double l = lam ? lam[p.r] : 1.0;
    f[off + id] = l * mass3(g, u + off, id);
}

// MASS: f is not read but formed as lam M u from u itself (u is the start of
// the correction step, f = lam M u), with the arithmetic of k_prolong_mass3.
template <bool CONST, bool MASS = false>
__global__ __launch_bounds__(BX* BY) void k_resid_cast3(Grid g, Coef<double> c, const double* __restrict__ u,
                                                        const double* __restrict__ f, float* __restrict__ r,
                                                        long stride, const double* __restrict__ lam) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long off = (long)p.r * stride;
    const long id = g.idx(p.i, p.j, p.l);
    double Ax, D;
    stiff3<double, CONST>(g, c, u + off, id, Ax, D);
    const double fv = MASS ? lam[p.r] * mass3(g, u + off, id) : f[off + id];
    r[off + id] = (float)(fv - Ax);
}

// Defect correction between two cycles in one pass: un = u + e on every
// interior node and r = f - A un (FP64, rounded to FP32) for the next cycle;
// un at the neighbours is formed again from u and e.  un must not alias u.
// MASS: f is not read but formed as lam M u from u itself (u is then the
// start of the correction step: the step's first cycle).
template <bool CONST, bool MASS = false>
__global__ __launch_bounds__(BX* BY) void k_add_resid3(Grid g, Coef<double> c, const double* __restrict__ u,
                                                       const float* __restrict__ e, const double* __restrict__ f,
                                                       double* __restrict__ un, float* __restrict__ r, long stride,
                                                       const double* __restrict__ lam) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long off = (long)p.r * stride;
    const long id = g.idx(p.i, p.j, p.l);
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    const double* ur = u + off;
    const float* er = e + off;
    // every load before the stores
    const double fv = MASS ? lam[p.r] * mass3(g, ur, id) : f[off + id];
    auto v = [&](long q) { return ur[q] + (double)er[q]; };
    const double x0 = v(id), xe = v(id + 1), xw = v(id - 1), xn = v(id + py), xs = v(id - py), xu = v(id + pz),
                 xd = v(id - pz);
    double Ax;
    if (CONST) {
        Ax = c.w0 * (6.0 * x0 - (xe + xw + xn + xs + xu + xd));
    } else {
        const double w1 = c.wx[id], w2 = c.wx[id - 1], w3 = c.wy[id], w4 = c.wy[id - py], w5 = c.wz[id],
                     w6 = c.wz[id - pz];
        Ax = (w1 + w2 + w3 + w4 + w5 + w6) * x0 - w1 * xe - w2 * xw - w3 * xn - w4 * xs - w5 * xu - w6 * xd;
    }
    un[off + id] = x0;
    r[off + id] = (float)(fv - Ax);
}

template <bool CONST>
__global__ __launch_bounds__(BX* BY) void k_border3(Grid g, Coef<double> c, const double* __restrict__ u,
                                                    double* __restrict__ au, double* __restrict__ mu,
                                                    double* __restrict__ partial, long stride) {
    __shared__ double sh[8];
    const Pos p = pos3(g.m);
    const long off = (long)p.r * stride;
    double ua = 0.0, um = 0.0;
    if (p.ok) {
        const long id = g.idx(p.i, p.j, p.l);
        double Ax, D;
        stiff3<double, CONST>(g, c, u + off, id, Ax, D);
        const double Mx = mass3(g, u + off, id);
        au[off + id] = Ax;
        mu[off + id] = Mx;
        ua = u[off + id] * Ax;
        um = u[off + id] * Mx;
    }
    const int lane = threadIdx.x + threadIdx.y * BX;
    for (int o = 32; o > 0; o >>= 1) {
        ua += __shfl_down(ua, o, 64);
        um += __shfl_down(um, o, 64);
    }
    if ((lane & 63) == 0) {
        sh[2 * threadIdx.y] = ua;
        sh[2 * threadIdx.y + 1] = um;
    }
    __syncthreads();
    if (lane == 0) {
        const long per = (long)gridDim.x * gridDim.y * g.m;  // blocks per rhs
        const long b = (long)p.r * per + ((long)(p.l - 1) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[2 * b] = sh[0] + sh[2] + sh[4] + sh[6];
        partial[2 * b + 1] = sh[1] + sh[3] + sh[5] + sh[7];
    }
}

template <typename T>
__global__ void k_pack3(Grid g, const T* __restrict__ padded, long sp, double* __restrict__ compact, long ld) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long ci = ((long)(p.l - 1) * g.m + (p.j - 1)) * g.m + (p.i - 1);
    compact[(long)p.r * ld + ci] = (double)padded[(long)p.r * sp + g.idx(p.i, p.j, p.l)];
}

template <typename T>
__global__ void k_unpack3(Grid g, const double* __restrict__ compact, long ld, T* __restrict__ padded, long sp) {
    const Pos p = pos3(g.m);
    if (!p.ok) return;
    const long ci = ((long)(p.l - 1) * g.m + (p.j - 1)) * g.m + (p.i - 1);
    padded[(long)p.r * sp + g.idx(p.i, p.j, p.l)] = (T)compact[(long)p.r * ld + ci];
}

}  // namespace

template <typename T>
void launch_smooth3(const Grid& g, const Coef<T>& c, const T* xc, const T* xp, const T* f, T* xn, int nrhs,
                    long stride, Cheb s, int zmode, hipStream_t st) {
    if (c.s15) return launch_smooth3g<T>(g, c.s15, xc, xp, f, xn, nrhs, stride, s, zmode, st);
    if (c.wx)
        hipLaunchKernelGGL((k_smooth3<T, false>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, xc, xp, f, xn,
                           stride, (T)s.a, (T)s.b, zmode);
    else
        hipLaunchKernelGGL((k_smooth3<T, true>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, xc, xp, f, xn,
                           stride, (T)s.a, (T)s.b, zmode);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_apply_A3(const Grid& g, const Coef<T>& c, const T* x, T* y, int nrhs, long stride, hipStream_t st) {
    if (c.s15) return launch_apply3g<T>(g, c.s15, x, y, nrhs, stride, st);
    if (c.wx)
        hipLaunchKernelGGL((k_apply_A3<T, false>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, x, y, stride);
    else
        hipLaunchKernelGGL((k_apply_A3<T, true>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, x, y, stride);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_resid_restrict3(const Grid& gf, const Coef<T>& c, const T* x, const T* f, const Grid& gc, T* rc,
                            int nrhs, long sf, long sc, hipStream_t st) {
    if (c.s15) return launch_resid_restrict3g<T>(gf, c.s15, x, f, gc, rc, nrhs, sf, sc, st);
    if (gc.n * 2 == gf.n && !c.wx && gc.m >= 1) {
        // constant coefficients: marching along z
        const int zc = (gc.m + ZKC - 1) / ZKC;
        dim3 grid((gc.m + ZTX - 1) / ZTX, (gc.m + ZTY - 1) / ZTY, zc * nrhs);
        hipLaunchKernelGGL((k_resid_restrict3z<T>), grid, dim3(256), 0, st, gf, c.w0, x, f, gc, rc, sf, sc, zc);
        PASM_CHECK_LAUNCH();
        return;
    }
    if (gc.n * 2 == gf.n) {  // the tiled form (ratio 2, which every hierarchy here has)
        const int zb = (gc.m + RCZ - 1) / RCZ;
        dim3 grid((gc.m + RCX - 1) / RCX, (gc.m + RCY - 1) / RCY, zb * nrhs);
        if (c.wx)
            hipLaunchKernelGGL((k_tile_restrict3<T, 0, false>), grid, dim3(256), 0, st, gf, c, x, f, gc, rc,
                               (T*)nullptr, nullptr, sf, sc, zb, nullptr, (T*)nullptr);
        else
            hipLaunchKernelGGL((k_tile_restrict3<T, 0, true>), grid, dim3(256), 0, st, gf, c, x, f, gc, rc,
                               (T*)nullptr, nullptr, sf, sc, zb, nullptr, (T*)nullptr);
        PASM_CHECK_LAUNCH();
        return;
    }
    if (c.wx)
        hipLaunchKernelGGL((k_resid_restrict3<T, false>), grid3(gc.m, nrhs), dim3(BX, BY), 0, st, gf, c, x, f,
                           gc, rc, sf, sc);
    else
        hipLaunchKernelGGL((k_resid_restrict3<T, true>), grid3(gc.m, nrhs), dim3(BX, BY), 0, st, gf, c, x, f,
                           gc, rc, sf, sc);
    PASM_CHECK_LAUNCH();
}

int launch_border_restrict3(const Grid& g, const Coef<double>& c, const double* u, const Grid& gc, double* bc,
                            double* cc, double* partial, int nrhs, long stride, long sc, hipStream_t st,
                            const float* e, double* un) {
    if (g.dim != 3 || gc.n * 2 != g.n) throw Error(PASM_E_INVALID, "fused border restriction: 3D, ratio 2");
    if (c.s15) throw Error(PASM_E_INVALID, "fused border restriction: no general 3D operator");
    if ((e == nullptr) != (un == nullptr) || (un && (un == u || c.wx)))
        throw Error(PASM_E_INVALID, "correction with borders (3D): constant coefficients, separate output");
    if (!c.wx) {
        // constant coefficients: marching along z; coarse nodes up to nc own
        // fine nodes for the sums
        const int zc = (gc.n + ZKC - 1) / ZKC;
        dim3 grid((gc.n + ZTX - 1) / ZTX, (gc.n + ZTY - 1) / ZTY, zc * nrhs);
        if (e)
            hipLaunchKernelGGL(k_border3z<true>, grid, dim3(256), 0, st, g, c.w0, u, e, un, gc, bc, cc, partial,
                               stride, sc, zc);
        else
            hipLaunchKernelGGL(k_border3z<false>, grid, dim3(256), 0, st, g, c.w0, u, e, un, gc, bc, cc, partial,
                               stride, sc, zc);
        PASM_CHECK_LAUNCH();
        return (int)(grid.x * grid.y * zc);
    }
    // coarse nodes up to nc (not only the interior ones) own fine nodes for the sums
    const int zb = (gc.n + RCZ - 1) / RCZ;
    dim3 grid((gc.n + RCX - 1) / RCX, (gc.n + RCY - 1) / RCY, zb * nrhs);
    if (e)
        hipLaunchKernelGGL((k_tile_restrict3<double, 1, true, true>), grid, dim3(tile3_threads<1>()), 0, st, g, c, u,
                           (const double*)nullptr, gc, bc, cc, partial, stride, sc, zb, e, un);
    else if (c.wx)
        hipLaunchKernelGGL((k_tile_restrict3<double, 1, false>), grid, dim3(tile3_threads<1>()), 0, st, g, c, u,
                           (const double*)nullptr,
                           gc, bc, cc, partial, stride, sc, zb, nullptr, (double*)nullptr);
    else
        hipLaunchKernelGGL((k_tile_restrict3<double, 1, true>), grid, dim3(tile3_threads<1>()), 0, st, g, c, u,
                           (const double*)nullptr,
                           gc, bc, cc, partial, stride, sc, zb, nullptr, (double*)nullptr);
    PASM_CHECK_LAUNCH();
    return (int)(grid.x * grid.y * zb);
}

template <typename T>
void launch_prolong3(const Grid& gc, const T* xc, const Grid& gf, T* xf, int nrhs, long sc, long sf, int mode,
                     const double* beta, hipStream_t st) {
    hipLaunchKernelGGL((k_prolong3<T>), grid3(gf.m, nrhs), dim3(BX, BY), 0, st, gc, xc, gf, xf, sc, sf, mode,
                       beta);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_restrict3(const Grid& gf, const T* xf, const Grid& gc, T* xc, int nrhs, long sf, long sc,
                      hipStream_t st) {
    hipLaunchKernelGGL((k_restrict3<T>), grid3(gc.m, nrhs), dim3(BX, BY), 0, st, gf, xf, gc, xc, sf, sc);
    PASM_CHECK_LAUNCH();
}

void launch_prolong_mass3(const Grid& gc, const double* xc, const Grid& gf, const double* xo, double* xn,
                          double* f, int nrhs, long sc, long sf, const double* beta, const double* lam,
                          hipStream_t st) {
    const int zb = (gf.m + QMZ - 1) / QMZ;
    dim3 grid((gf.m + QMX - 1) / QMX, (gf.m + QMY - 1) / QMY, zb * nrhs);
    hipLaunchKernelGGL(k_prolong_mass3, grid, dim3(256), 0, st, gc, xc, gf, xo, xn, f, sc, sf, beta, lam, zb);
    PASM_CHECK_LAUNCH();
}

void launch_prolong_resid3(const Grid& gc, const double* xc, const Grid& gf, const Coef<double>& c, const double* xo,
                           double* xn, float* r, int nrhs, long sc, long sf, const double* beta, const double* lam,
                           hipStream_t st) {
    if (gf.dim != 3 || gc.n * 2 != gf.n || c.wx || c.s15 || xn == xo)
        throw Error(PASM_E_INVALID, "prolongation with the first residual (3D): constant coefficients, ratio 2");
    const int zc = (gf.m + ZRC - 1) / ZRC;
    dim3 grid((gf.m + ZFX - 1) / ZFX, (gf.m + ZFY - 1) / ZFY, zc * nrhs);
    hipLaunchKernelGGL((k_resid3z<false, true>), grid, dim3(256), 0, st, gf, c.w0, xo, (const float*)nullptr, lam,
                       xn, r, sf, zc, gc, xc, sc, beta);
    PASM_CHECK_LAUNCH();
}

void launch_mass_rhs3(const Grid& g, const double* u, const double* lam, double* f, int nrhs, long stride,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_mass_rhs3, grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, u, lam, f, stride);
    PASM_CHECK_LAUNCH();
}

void launch_resid_cast3(const Grid& g, const Coef<double>& c, const double* u, const double* f, float* r,
                        int nrhs, long stride, hipStream_t st, const double* lam) {
    if (lam && c.wx) throw Error(PASM_E_INVALID, "residual with lam M u (3D): constant or 15-point operators");
    if (c.s15) return launch_resid_cast3g(g, c.s15, u, f, r, nrhs, stride, st, lam);
    if (lam) {
        const int zc = (g.m + ZRC - 1) / ZRC;
        dim3 grid((g.m + ZFX - 1) / ZFX, (g.m + ZFY - 1) / ZFY, zc * nrhs);
        hipLaunchKernelGGL((k_resid3z<false>), grid, dim3(256), 0, st, g, c.w0, u, (const float*)nullptr, lam,
                           (double*)nullptr, r, stride, zc, g, (const double*)nullptr, 0L, (const double*)nullptr);
    }
    else if (c.wx)
        hipLaunchKernelGGL((k_resid_cast3<false>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, u, f, r, stride,
                           nullptr);
    else
        hipLaunchKernelGGL((k_resid_cast3<true>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, u, f, r, stride,
                           nullptr);
    PASM_CHECK_LAUNCH();
}

void launch_add_resid3(const Grid& g, const Coef<double>& c, const double* u, const float* e, const double* f,
                       double* un, float* r, int nrhs, long stride, hipStream_t st, const double* lam) {
    if (g.dim != 3 || un == u) throw Error(PASM_E_INVALID, "add and residual: 3D, separate output");
    if (lam && c.wx) throw Error(PASM_E_INVALID, "add and residual with lam M u (3D): constant or 15-point operators");
    if (c.s15) return launch_add_resid3g(g, c.s15, u, e, f, un, r, nrhs, stride, st, lam);
    if (lam) {
        const int zc = (g.m + ZRC - 1) / ZRC;
        dim3 grid((g.m + ZFX - 1) / ZFX, (g.m + ZFY - 1) / ZFY, zc * nrhs);
        hipLaunchKernelGGL((k_resid3z<true>), grid, dim3(256), 0, st, g, c.w0, u, e, lam, un, r, stride, zc, g,
                           (const double*)nullptr, 0L, (const double*)nullptr);
    }
    else if (c.wx)
        hipLaunchKernelGGL((k_add_resid3<false>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, u, e, f, un, r, stride,
                           nullptr);
    else
        hipLaunchKernelGGL((k_add_resid3<true>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, c, u, e, f, un, r, stride,
                           nullptr);
    PASM_CHECK_LAUNCH();
}

int launch_border3(const Grid& g, const Coef<double>& c, const double* u, double* au, double* mu,
                   double* partial, int nrhs, long stride, hipStream_t st) {
    if (c.s15) return launch_border3g(g, c.s15, u, au, mu, partial, nrhs, stride, st);
    dim3 grid = grid3(g.m, nrhs);
    if (c.wx)
        hipLaunchKernelGGL(k_border3<false>, grid, dim3(BX, BY), 0, st, g, c, u, au, mu, partial, stride);
    else
        hipLaunchKernelGGL(k_border3<true>, grid, dim3(BX, BY), 0, st, g, c, u, au, mu, partial, stride);
    PASM_CHECK_LAUNCH();
    return (int)(grid.x * grid.y * g.m);
}

template <typename T>
void launch_pack3(const Grid& g, const T* padded, long sp, double* compact, long ld, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL((k_pack3<T>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, padded, sp, compact, ld);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_unpack3(const Grid& g, const double* compact, long ld, T* padded, long sp, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL((k_unpack3<T>), grid3(g.m, nrhs), dim3(BX, BY), 0, st, g, compact, ld, padded, sp);
    PASM_CHECK_LAUNCH();
}

#define PASM_INST3(T)                                                                                    \
    template void launch_smooth3<T>(const Grid&, const Coef<T>&, const T*, const T*, const T*, T*, int,   \
                                    long, Cheb, int, hipStream_t);                                       \
    template void launch_apply_A3<T>(const Grid&, const Coef<T>&, const T*, T*, int, long, hipStream_t);  \
    template void launch_resid_restrict3<T>(const Grid&, const Coef<T>&, const T*, const T*, const Grid&, \
                                            T*, int, long, long, hipStream_t);                            \
    template void launch_prolong3<T>(const Grid&, const T*, const Grid&, T*, int, long, long, int,        \
                                     const double*, hipStream_t);                                         \
    template void launch_restrict3<T>(const Grid&, const T*, const Grid&, T*, int, long, long, hipStream_t); \
    template void launch_pack3<T>(const Grid&, const T*, long, double*, long, int, hipStream_t);          \
    template void launch_unpack3<T>(const Grid&, const double*, long, T*, long, int, hipStream_t);
PASM_INST3(double)
PASM_INST3(float)
#undef PASM_INST3

}  // namespace pasm

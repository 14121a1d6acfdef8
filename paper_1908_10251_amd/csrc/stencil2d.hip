// Matrix-free P1 operators and grid transfers on the uniform "/" triangle mesh
// (2D Kuhn split), for all k right-hand sides of a batch.
//
// Stiffness: for kappa constant per element, each triangle couples the two
// ends of each leg with -kappa_T/2 and the hypotenuse ends with 0, so the
// stiffness is a 5-point stencil whose edge weights are read per node
// (Section 2, the discrete eigenproblem; weak form a(u,v)).
// Mass: |T|(1+delta_ij)/12 summed over the 6 triangles around a node gives
// h^2 (1/2 at the centre, 1/12 at E, W, N, S, NE, SW).
// Prolongation (nested spaces of Section 3): a fine node at (2I+a, 2J+b) takes
// the mean of the coarse nodes (I, J) and (I+a, J+b) (a coarse P1 function is
// linear along the coarse edge in direction (a, b)); restriction is its
// transpose.
//
// Launch shape: 64 x 4 threads, one wavefront per 64 consecutive nodes of a
// row (coalesced, 128-byte aligned rows), grid.z = right-hand side.
#include <algorithm>

#include "common.h"

namespace pasm {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

inline dim3 grid_for(int mx, int my, int nrhs) {
    return dim3((mx + BX - 1) / BX, (my + BY - 1) / BY, nrhs);
}

// KIND: 0 constant coefficients, 1 edge weights, 2 general 7-point (see Coef).
template <typename T, int KIND>
struct Stiff2 {
    // Returns A x at node id and the diagonal D.
    __device__ static inline void apply(const Grid& g, const Coef<T>& c, const T* __restrict__ x,
                                        long id, T& Ax, T& D) {
        const int p = g.pitch;
        const T x0 = x[id];
        const T xe = x[id + 1], xw = x[id - 1], xn = x[id + p], xs = x[id - p];
        if (KIND == 0) {
            D = T(4) * c.w0;
            Ax = c.w0 * (T(4) * x0 - xe - xw - xn - xs);
        } else if (KIND == 1) {
            const T we = c.wx[id], ww = c.wx[id - 1], wn = c.wy[id], ws = c.wy[id - p];
            D = we + ww + wn + ws;
            Ax = D * x0 - we * xe - ww * xw - wn * xn - ws * xs;
        } else {
            const T we = c.wx[id], ww = c.wx[id - 1], wn = c.wy[id], ws = c.wy[id - p];
            const T wa = c.wne[id], wb = c.wne[id - p - 1];
            D = c.d[id];
            Ax = D * x0 - we * xe - ww * xw - wn * xn - ws * xs - wa * x[id + p + 1] - wb * x[id - p - 1];
        }
    }
    __device__ static inline T diag(const Grid& g, const Coef<T>& c, long id) {
        if (KIND == 0) return T(4) * c.w0;
        if (KIND == 1) return c.wx[id] + c.wx[id - 1] + c.wy[id] + c.wy[id - g.pitch];
        return c.d[id];
    }
};

// The coefficients of the member that right-hand side z belongs to, and that
// member's factor on the smoother's b coefficients.
template <typename T>
__device__ inline Coef<T> member_coef(const Coef<T>& c, int z, T& bscale) {
    Coef<T> r = c;
    const int mem = z / c.kpm;
    const long o = (long)mem * c.ms;
    if (r.wx) r.wx += o;
    if (r.wy) r.wy += o;
    if (r.wz) r.wz += o;
    if (r.d) r.d += o;
    if (r.wne) r.wne += o;
    bscale = c.bsc ? c.bsc[mem] : T(1);
    return r;
}

// One smoothing step, x_{k+1} = x_k + a (x_k - x_{k-1}) + b D^{-1} (f - A x_k).
// xp may alias xn: each thread reads xp at its own node before writing xn there.
template <typename T, int KIND>
__global__ __launch_bounds__(BX* BY) void k_smooth(Grid g, Coef<T> cg, const T* __restrict__ xc,
                                                   const T* xp, const T* __restrict__ f, T* xn,
                                                   long stride, T a, T b, int zmode) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    T bs;
    const Coef<T> c = member_coef(cg, blockIdx.z, bs);
    b *= bs;
    const long off = (long)blockIdx.z * stride;
    const long id = g.idx(i, j);
    const T fv = f[off + id];
    if (zmode & 1) {
        const T D = Stiff2<T, KIND>::diag(g, c, id);
        xn[off + id] = b * fv / D;
        return;
    }
    T Ax, D;
    Stiff2<T, KIND>::apply(g, c, xc + off, id, Ax, D);
    const T x0 = xc[off + id];
    T v = x0 + b * (fv - Ax) / D;
    if (a != T(0)) v += a * (x0 - ((zmode & 2) ? T(0) : xp[off + id]));
    xn[off + id] = v;
}

// All S steps of one smoothing phase in one pass over HBM (temporal
// blocking).  A 64 x 4 workgroup owns a tile of 64 LDS columns by 4*ROWS LDS
// rows: the (64 - 2S) x (4*ROWS - 2S) output nodes plus an S-node halo.
// Thread (tx, ty) owns LDS column tx and rows ty, ty+4, ...; it keeps f,
// x_{t-1} and x_t of its own nodes in registers, and the current iterate of
// the tile lives in LDS (double buffered) for the neighbours.  Every step
// updates all nodes except the outer ring of the tile: after S steps the
// nodes at distance >= S from the tile edge hold x_S exactly (their
// dependence cone stays inside the loaded region); values nearer the edge are
// discarded.  Nodes on or outside the domain boundary stay zero.  A phase
// always starts fresh (a_0 = 0), so only x_0 is read, and not at all when
// x_0 = 0.
template <typename T, int KIND, int S, int ROWS>
__global__ __launch_bounds__(256) void k_smooth_fused(Grid g, Coef<T> cg, const T* __restrict__ x0,
                                                      const T* __restrict__ f, T* __restrict__ out, long stride,
                                                      SmoothSteps st, int x_zero, int share, int rb) {
    constexpr int W = 64, HH = 4 * ROWS, TX = W - 2 * S, TY = HH - 2 * S;
    constexpr bool CONST = KIND == 0;
    constexpr bool GEN = KIND == 2;
    __shared__ T sa[W * HH], sb[W * HH];
    __shared__ T swx[CONST ? 1 : W * HH], swy[CONST ? 1 : W * HH];
    __shared__ T sd[GEN ? W * HH : 1], swne[GEN ? W * HH : 1];
    // this workgroup's right-hand sides [r0, r1): consecutive ones sharing
    // one coefficient array, which is staged in LDS once for all of them
    const int zb = (share + rb - 1) / rb;
    const int grp = blockIdx.z / zb;
    const int r0 = grp * share + (blockIdx.z % zb) * rb;
    const int r1 = min(r0 + rb, (grp + 1) * share);
    T bsc;
    const Coef<T> c = member_coef(cg, r0, bsc);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = blockIdx.x * TX + 1 - S + tx;  // global column of this thread
    const int jb = blockIdx.y * TY + 1 - S;      // global row of LDS row 0
    bool upd[ROWS], inn[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int ly = ty + 4 * r, j = jb + ly;
        const bool inner = i >= 1 && i <= g.m && j >= 1 && j <= g.m;
        inn[r] = inner;
        upd[r] = inner && tx > 0 && tx < W - 1 && ly > 0 && ly < HH - 1;
        if (!CONST) {
            const bool stored = i >= 0 && i <= g.n && j >= 0 && j <= g.n;
            swx[ly * W + tx] = (stored && i < g.n) ? c.wx[g.idx(i, j)] : T(0);
            swy[ly * W + tx] = (stored && j < g.n) ? c.wy[g.idx(i, j)] : T(0);
            if (GEN) {
                swne[ly * W + tx] = (stored && i < g.n && j < g.n) ? c.wne[g.idx(i, j)] : T(0);
                sd[ly * W + tx] = inner ? c.d[g.idx(i, j)] : T(1);
            }
        }
    }
    const T invD0 = T(1) / (T(4) * c.w0);
    // reciprocal diagonal of the own nodes, once for all right-hand sides
    T idg[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) idg[r] = invD0;
    __syncthreads();  // coefficient tiles complete before they are read
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int p = (ty + 4 * r) * W + tx;
        if (!CONST && upd[r]) {
            const T D = GEN ? sd[p] : (swx[p] + swx[p - 1] + swy[p] + swy[p - W]);
            idg[r] = T(1) / D;
        }
    }
    // x and f of the next right-hand side are loaded while this one is
    // smoothed: unconditional loads from clamped positions (the values off
    // the interior are replaced by zeros when they are used)
    int rid[ROWS];  // offsets within one right-hand side's block (< 2^31)
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
        rid[r] = (int)g.idx(min(max(i, 1), g.m), min(max(jb + ty + 4 * r, 1), g.m));
    const T* xsrc = x_zero ? f : x0;
    T nf[ROWS], nx[ROWS];
    auto fetch = [&](int rhs) {
        const long off = (long)rhs * stride;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            nf[r] = f[off + rid[r]];
            nx[r] = xsrc[off + rid[r]];
        }
    };
    fetch(r0);
    for (int rhs = r0; rhs < r1; ++rhs) {
        const long off = (long)rhs * stride;
        T fr[ROWS], xc[ROWS], xp[ROWS];
        __syncthreads();  // the previous right-hand side is done with sa / sb
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int ly = ty + 4 * r;
            const T fv = inn[r] ? nf[r] : T(0);
            const T xv = (inn[r] && !x_zero) ? nx[r] : T(0);
            fr[r] = fv;
            xc[r] = xv;
            xp[r] = xv;
            sa[ly * W + tx] = xv;
        }
        if (rhs + 1 < r1) fetch(rhs + 1);
        __syncthreads();
        T* cur = sa;
        T* nxt = sb;
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const T a = (T)st.a[t], b = (T)st.b[t] * bsc;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int p = (ty + 4 * r) * W + tx;
                T v = xc[r];
                if (upd[r]) {
                    const T xe = cur[p + 1], xw = cur[p - 1], xn = cur[p + W], xs = cur[p - W];
                    if (CONST) {
                        const T Ax = c.w0 * (T(4) * v - xe - xw - xn - xs);
                        v = v + b * (fr[r] - Ax) * invD0;
                    } else if (!GEN) {
                        const T we = swx[p], ww = swx[p - 1], wn = swy[p], ws = swy[p - W];
                        const T D = we + ww + wn + ws;
                        const T Ax = D * v - we * xe - ww * xw - wn * xn - ws * xs;
                        v = v + b * (fr[r] - Ax) * idg[r];
                    } else {
                        const T we = swx[p], ww = swx[p - 1], wn = swy[p], ws = swy[p - W];
                        const T wa = swne[p], wb = swne[p - W - 1];
                        const T D = sd[p];
                        const T Ax = D * v - we * xe - ww * xw - wn * xn - ws * xs - wa * cur[p + W + 1] -
                                     wb * cur[p - W - 1];
                        v = v + b * (fr[r] - Ax) * idg[r];
                    }
                    if (a != T(0)) v += a * (xc[r] - xp[r]);
                }
                xp[r] = xc[r];
                xc[r] = v;
                nxt[p] = v;
            }
            __syncthreads();
            T* tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
        if (tx >= S && tx < W - S) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int ly = ty + 4 * r, j = jb + ly;
                if (ly < S || ly >= HH - S) continue;
                if (i < 1 || i > g.m || j < 1 || j > g.m) continue;
                out[off + g.idx(i, j)] = xc[r];
            }
        }
    }
}

template <typename T, int KIND>
__global__ __launch_bounds__(BX* BY) void k_apply_A(Grid g, Coef<T> cg, const T* __restrict__ x,
                                                    T* __restrict__ y, long stride) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    T bs;
    const Coef<T> c = member_coef(cg, blockIdx.z, bs);
    const long off = (long)blockIdx.z * stride;
    const long id = g.idx(i, j);
    T Ax, D;
    Stiff2<T, KIND>::apply(g, c, x + off, id, Ax, D);
    y[off + id] = Ax;
}

// r_c = P^T (f - A x): each coarse interior node gathers the residual at the 7
// fine nodes whose interpolation stencil contains it.
template <typename T, int KIND>
__global__ __launch_bounds__(BX* BY) void k_resid_restrict(Grid gf, Coef<T> cg, const T* __restrict__ x,
                                                           const T* __restrict__ f, Grid gc,
                                                           T* __restrict__ rc, long sf, long sc) {
    const int I = blockIdx.x * BX + threadIdx.x + 1;
    const int J = blockIdx.y * BY + threadIdx.y + 1;
    if (I > gc.m || J > gc.m) return;
    T bs;
    const Coef<T> c = member_coef(cg, blockIdx.z, bs);
    const T* xr = x + (long)blockIdx.z * sf;
    const T* fr = f + (long)blockIdx.z * sf;
    const int i = 2 * I, j = 2 * J;
    auto res = [&](int ii, int jj) -> T {
        const long id = gf.idx(ii, jj);
        T Ax, D;
        Stiff2<T, KIND>::apply(gf, c, xr, id, Ax, D);
        return fr[id] - Ax;
    };
    T v = res(i, j);
    T s = res(i + 1, j) + res(i - 1, j) + res(i, j + 1) + res(i, j - 1) + res(i + 1, j + 1) +
          res(i - 1, j - 1);
    rc[(long)blockIdx.z * sc + gc.idx(I, J)] = v + T(0.5) * s;
}

template <typename T>
__global__ __launch_bounds__(BX* BY) void k_restrict(Grid gf, const T* __restrict__ xf, Grid gc,
                                                     T* __restrict__ xc, long sf, long sc) {
    const int I = blockIdx.x * BX + threadIdx.x + 1;
    const int J = blockIdx.y * BY + threadIdx.y + 1;
    if (I > gc.m || J > gc.m) return;
    const T* xr = xf + (long)blockIdx.z * sf;
    const long id = gf.idx(2 * I, 2 * J);
    const int p = gf.pitch;
    T s = xr[id + 1] + xr[id - 1] + xr[id + p] + xr[id - p] + xr[id + p + 1] + xr[id - p - 1];
    T v;
    if constexpr (sizeof(T) == 8)
        v = __builtin_fma(0.5, s, xr[id]);  // as the chained restriction forms it
    else
        v = xr[id] + T(0.5) * s;
    xc[(long)blockIdx.z * sc + gc.idx(I, J)] = v;
}

// Three restrictions in a row (FP64, 2D): a workgroup stages a tile of the
// finest of the four levels in LDS, forms the two intermediate levels there
// and writes RC_T x RC_T nodes of the coarsest.  Every node is formed as
// k_restrict forms it (the six neighbours in the same order, one fused
// multiply-add), nodes off a level's interior are zero, so the result equals
// three k_restrict launches bit for bit, with one pass over the fine field.
constexpr int RC_T = 8;
__global__ __launch_bounds__(256) void k_restrict_chain3(Grid g3, const double* __restrict__ x3, Grid g2, Grid g1,
                                                         Grid g0, double* __restrict__ x0, long s3, long s0) {
    constexpr int N3 = 8 * RC_T + 7, N2 = 4 * RC_T + 3, N1 = 2 * RC_T + 1;
    __shared__ double a3[N3][N3 + 1];
    __shared__ double a2[N2][N2 + 1];
    __shared__ double a1[N1][N1 + 1];
    const int I0 = blockIdx.x * RC_T + 1, J0 = blockIdx.y * RC_T + 1;
    // first node of each level's tile: coarse node I needs 2I - 1 .. 2I + 1
    // one level finer, so the tiles start at 2 o - 1 of the level below
    const int o1i = 2 * I0 - 1, o1j = 2 * J0 - 1;
    const int o2i = 2 * o1i - 1, o2j = 2 * o1j - 1;
    const int o3i = 2 * o2i - 1, o3j = 2 * o2j - 1;
    const double* xr = x3 + (long)blockIdx.z * s3;
    {
        // every load of the thread in flight at once, then the LDS stores
        constexpr int E = (N3 * N3 + 255) / 256;
        double v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e, a = t % N3, b = t / N3, i = o3i + a, j = o3j + b;
            v[e] = (t < N3 * N3 && i >= 0 && i <= g3.n && j >= 0 && j <= g3.n) ? xr[g3.idx(i, j)] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            if (t < N3 * N3) a3[t / N3][t % N3] = v[e];
        }
    }
    __syncthreads();
    // node (i, j) of the coarser level from local (2a + 1, 2b + 1) of the finer
    auto rstr = [](const double* A, int ld, int c, int r) {
        const double s = A[r * ld + c + 1] + A[r * ld + c - 1] + A[(r + 1) * ld + c] + A[(r - 1) * ld + c] +
                         A[(r + 1) * ld + c + 1] + A[(r - 1) * ld + c - 1];
        return __builtin_fma(0.5, s, A[r * ld + c]);
    };
    for (int t = threadIdx.x; t < N2 * N2; t += 256) {
        const int a = t % N2, b = t / N2, i = o2i + a, j = o2j + b;
        a2[b][a] = (i >= 1 && i <= g2.m && j >= 1 && j <= g2.m) ? rstr(&a3[0][0], N3 + 1, 2 * a + 1, 2 * b + 1) : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < N1 * N1; t += 256) {
        const int a = t % N1, b = t / N1, i = o1i + a, j = o1j + b;
        a1[b][a] = (i >= 1 && i <= g1.m && j >= 1 && j <= g1.m) ? rstr(&a2[0][0], N2 + 1, 2 * a + 1, 2 * b + 1) : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < RC_T * RC_T) {
        const int a = threadIdx.x % RC_T, b = threadIdx.x / RC_T, I = I0 + a, J = J0 + b;
        if (I <= g0.m && J <= g0.m)
            x0[(long)blockIdx.z * s0 + g0.idx(I, J)] = rstr(&a1[0][0], N1 + 1, 2 * a + 1, 2 * b + 1);
    }
}

// mode 0: x_f = P x_c; 1: x_f += P x_c; 2: x_f = P x_c + beta[r] x_f
template <typename T>
__global__ __launch_bounds__(BX* BY) void k_prolong(Grid gc, const T* __restrict__ xc, Grid gf,
                                                    T* __restrict__ xf, long sc, long sf, int mode,
                                                    const double* __restrict__ beta) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > gf.m || j > gf.m) return;
    const T* cr = xc + (long)blockIdx.z * sc;
    const int I = i >> 1, J = j >> 1, a = i & 1, b = j & 1;
    const long cid = gc.idx(I, J);
    T v = cr[cid];
    if (a | b) v = T(0.5) * (v + cr[cid + a + (long)b * gc.pitch]);
    const long id = (long)blockIdx.z * sf + gf.idx(i, j);
    if (mode == 1) v += xf[id];
    else if (mode == 2 && beta[blockIdx.z] != 0.0) v += T(beta[blockIdx.z]) * xf[id];  // a zero weight drops the old field
    xf[id] = v;
}

__device__ inline double mass2(const Grid& g, const double* __restrict__ u, long id) {
    const int p = g.pitch;
    const double s = u[id + 1] + u[id - 1] + u[id + p] + u[id - p] + u[id + p + 1] + u[id - p - 1];
    return g.h * g.h * (0.5 * u[id] + s * (1.0 / 12.0));
}

__global__ __launch_bounds__(BX* BY) void k_mass_rhs(Grid g, const double* __restrict__ u,
                                                     const double* __restrict__ lam,
                                                     double* __restrict__ f, long stride) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    const long off = (long)blockIdx.z * stride;
    const long id = g.idx(i, j);
    const double l = lam ? lam[blockIdx.z] : 1.0;
    f[off + id] = l * mass2(g, u + off, id);
}

// RB right-hand sides per workgroup (edge weights of a single problem: the
// weights are loaded once for all of them; RB = 1 for batches, whose members
// have planes of their own).  MASS: f is not read but formed as lam M u
// from u itself (u is the start of the correction step, f = lam M u).
template <int KIND, typename TO, int RB = 1, bool MASS = false>
__global__ __launch_bounds__(BX* BY) void k_resid_cast(Grid g, Coef<double> cg, const double* __restrict__ u,
                                                       const double* __restrict__ f,
                                                       TO* __restrict__ r, long stride, long rstride, int nrhs,
                                                       const double* __restrict__ lam) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    const long id = g.idx(i, j);
    if (RB > 1 && KIND == 1) {
        const double we = cg.wx[id], ww = cg.wx[id - 1], wn = cg.wy[id], ws = cg.wy[id - g.pitch];
        const double D = we + ww + wn + ws;
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int z = blockIdx.z * RB + q;
            if (z >= nrhs) break;
            const double* ur = u + (long)z * stride;
            const int p = g.pitch;
            const double u0 = ur[id], uE = ur[id + 1], uW = ur[id - 1], uN = ur[id + p], uS = ur[id - p];
            const double Ax = D * u0 - we * uE - ww * uW - wn * uN - ws * uS;
            double fv;
            if (MASS) {
                // lam M u with the neighbours in the order of k_prolong_mass
                const double sn = uE + uW + uN + uS + ur[id + p + 1] + ur[id - p - 1];
                fv = lam[z] * (g.h * g.h * __builtin_fma(sn, 1.0 / 12.0, 0.5 * u0));
            } else {
                fv = f[(long)z * stride + id];
            }
            r[(long)z * rstride + id] = (TO)(fv - Ax);
        }
        return;
    }
    static_assert(!MASS || (RB > 1 && KIND == 1), "mass right-hand side: edge weights, several right-hand sides");
    double bs;
    const Coef<double> c = member_coef(cg, blockIdx.z, bs);
    const long off = (long)blockIdx.z * stride;
    double Ax, D;
    Stiff2<double, KIND>::apply(g, c, u + off, id, Ax, D);
    r[(long)blockIdx.z * rstride + id] = (TO)(f[off + id] - Ax);
}

// Defect correction between two cycles in one pass (2D; KIND 0 constant
// coefficients, 1 edge weights): un = u + e on every interior node and
// r = f - A un (FP64, rounded to FP32) for the next cycle; un at the
// neighbours is formed again from u and e.  un must not alias u.
// MASS: f is not read but formed as lam M u from u itself (u is then the
// start of the correction step: the step's first cycle).  !WUN: un is not
// stored (the caller keeps u and e and adds them again later).
template <int KIND, int RB = 1, bool MASS = false, bool WUN = true>
__global__ __launch_bounds__(BX* BY) void k_add_resid(Grid g, Coef<double> c, const double* __restrict__ u,
                                                      const float* __restrict__ e, const double* __restrict__ f,
                                                      double* __restrict__ un, float* __restrict__ r, long stride,
                                                      int nrhs, const double* __restrict__ lam) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    const long gid = g.idx(i, j);
    double we = 0.0, ww = 0.0, wn = 0.0, ws = 0.0;
    if (KIND == 1) {
        // loaded once for the workgroup's RB right-hand sides
        we = c.wx[gid], ww = c.wx[gid - 1], wn = c.wy[gid], ws = c.wy[gid - g.pitch];
    }
    const int p = g.pitch;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int z = blockIdx.z * RB + q;
        if (z >= nrhs) break;
        const long id = (long)z * stride + gid;
        // every load of the right-hand side before its stores
        const double u0 = u[id], uE = u[id + 1], uW = u[id - 1], uN = u[id + p], uS = u[id - p];
        const double x0 = u0 + (double)e[id], xE = uE + (double)e[id + 1], xW = uW + (double)e[id - 1],
                     xN = uN + (double)e[id + p], xS = uS + (double)e[id - p];
        double Ax;
        if (KIND == 0) {
            Ax = c.w0 * (4.0 * x0 - (xE + xW + xN + xS));
        } else {
            Ax = (we + ww + wn + ws) * x0 - we * xE - ww * xW - wn * xN - ws * xS;
        }
        double fv;
        if (MASS) {
            // lam M u with the neighbours in the order of k_prolong_mass
            const double sn = uE + uW + uN + uS + u[id + p + 1] + u[id - p - 1];
            fv = lam[z] * (g.h * g.h * __builtin_fma(sn, 1.0 / 12.0, 0.5 * u0));
        } else {
            fv = f[id];
        }
        if (WUN) un[id] = x0;
        r[id] = (float)(fv - Ax);
    }
}

// The same for batches (right-hand side z of member z / kpm, the member's
// coefficient planes) with edge weights (KIND 1) or the general operator
// (KIND 2), f = lam M u formed from u: un = u + e, r = lam M u - A un
// (ADD), or r = lam M u - A u.  RB consecutive right-hand sides of one
// member per thread (RB divides kpm) share the coefficient loads.
template <int KIND, int RB, bool ADD>
__global__ __launch_bounds__(BX* BY) void k_resid_mass_m(Grid g, Coef<double> cg, const double* __restrict__ u,
                                                         const float* __restrict__ e, double* __restrict__ un,
                                                         float* __restrict__ r, long stride,
                                                         const double* __restrict__ lam) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    const int z0 = blockIdx.z * RB;
    double bs;
    const Coef<double> c = member_coef(cg, z0, bs);
    const int p = g.pitch;
    const long gid = g.idx(i, j);
    const double we = c.wx[gid], ww = c.wx[gid - 1], wn = c.wy[gid], ws = c.wy[gid - p];
    double wa = 0.0, wb = 0.0, d = we + ww + wn + ws;
    if (KIND == 2) {
        wa = c.wne[gid];
        wb = c.wne[gid - p - 1];
        d = c.d[gid];
    }
    const double h2 = g.h * g.h;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int z = z0 + q;
        const long id = (long)z * stride + gid;
        // every load of the right-hand side before its stores
        const double u0 = u[id], uE = u[id + 1], uW = u[id - 1], uN = u[id + p], uS = u[id - p];
        const double uNE = u[id + p + 1], uSW = u[id - p - 1];
        double x0 = u0, xE = uE, xW = uW, xN = uN, xS = uS, xNE = uNE, xSW = uSW;
        if (ADD) {
            x0 += (double)e[id], xE += (double)e[id + 1], xW += (double)e[id - 1], xN += (double)e[id + p];
            xS += (double)e[id - p];
            if (KIND == 2) xNE += (double)e[id + p + 1], xSW += (double)e[id - p - 1];
        }
        double Ax = d * x0 - we * xE - ww * xW - wn * xN - ws * xS;
        if (KIND == 2) Ax -= wa * xNE + wb * xSW;
        const double fv = lam[z] * (h2 * (0.5 * u0 + (uE + uW + uN + uS + uNE + uSW) * (1.0 / 12.0)));
        if (ADD) un[id] = x0;
        r[id] = (float)(fv - Ax);
    }
}

template <typename TE>
__global__ void k_add_correction(const TE* __restrict__ e, double* __restrict__ u, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        u[t] += (double)e[t];
}

// Deterministic block sum of two values; result valid in thread 0.
__device__ inline void block_sum2(double& a, double& b, double* sh) {
    const int lane = threadIdx.x + threadIdx.y * BX;  // BX == 64: one wavefront per row of the block
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    const int w = lane >> 6;
    if ((lane & 63) == 0) {
        sh[2 * w] = a;
        sh[2 * w + 1] = b;
    }
    __syncthreads();
    if (lane == 0) {
        a = sh[0] + sh[2] + sh[4] + sh[6];
        b = sh[1] + sh[3] + sh[5] + sh[7];
    }
}

template <int KIND>
__global__ __launch_bounds__(BX* BY) void k_border(Grid g, Coef<double> cg, const double* __restrict__ u,
                                                   double* __restrict__ au, double* __restrict__ mu,
                                                   double* __restrict__ partial, long stride) {
    __shared__ double sh[8];
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    const long off = (long)blockIdx.z * stride;
    double bs;
    const Coef<double> c = member_coef(cg, blockIdx.z, bs);
    double ua = 0.0, um = 0.0;
    if (i <= g.m && j <= g.m) {
        const long id = g.idx(i, j);
        double Ax, D;
        Stiff2<double, KIND>::apply(g, c, u + off, id, Ax, D);
        const double Mx = mass2(g, u + off, id);
        au[off + id] = Ax;
        mu[off + id] = Mx;
        ua = u[off + id] * Ax;
        um = u[off + id] * Mx;
    }
    block_sum2(ua, um, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const long nblk = (long)gridDim.x * gridDim.y;
        const long b = (long)blockIdx.z * nblk + blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * b] = ua;
        partial[2 * b + 1] = um;
    }
}

// Borders fused with the first restriction: each thread owns coarse node
// (I, J) of the next coarser grid (I, J = 1 .. nc, the last row/column only
// for the sums), computes A u and M u at the seven fine nodes whose
// interpolation reaches (I, J), writes b_c = P^T A u and c_c = P^T M u there,
// and adds u.Au, u.Mu over the four fine nodes (2I - a, 2J - b), a, b in
// {0, 1}, that it owns, so every fine node is counted once.
template <int KIND>
__global__ __launch_bounds__(BX* BY) void k_border_restrict(Grid g, Coef<double> cg, const double* __restrict__ u,
                                                            Grid gc, double* __restrict__ bc,
                                                            double* __restrict__ cc, double* __restrict__ partial,
                                                            long stride, long sc) {
    __shared__ double sh[8];
    const int I = blockIdx.x * BX + threadIdx.x + 1;
    const int J = blockIdx.y * BY + threadIdx.y + 1;
    double bs;
    const Coef<double> c = member_coef(cg, blockIdx.z, bs);
    const double* ur = u + (long)blockIdx.z * stride;
    double ua = 0.0, um = 0.0;
    if (I <= gc.n && J <= gc.n) {
        constexpr int off[7][2] = {{0, 0}, {-1, 0}, {0, -1}, {-1, -1}, {1, 0}, {0, 1}, {1, 1}};
        double rb = 0.0, rc = 0.0;
#pragma unroll
        for (int o = 0; o < 7; ++o) {
            const int i = 2 * I + off[o][0], j = 2 * J + off[o][1];
            if (i < 1 || j < 1 || i > g.m || j > g.m) continue;
            const long id = g.idx(i, j);
            double Ax, D;
            Stiff2<double, KIND>::apply(g, c, ur, id, Ax, D);
            const double Mx = mass2(g, ur, id);
            const double w = o == 0 ? 1.0 : 0.5;
            rb += w * Ax;
            rc += w * Mx;
            if (o < 4) {  // owned: offsets (0,0), (-1,0), (0,-1), (-1,-1)
                ua += ur[id] * Ax;
                um += ur[id] * Mx;
            }
        }
        if (I <= gc.m && J <= gc.m) {
            const long cid = (long)blockIdx.z * sc + gc.idx(I, J);
            bc[cid] = rb;
            cc[cid] = rc;
        }
    }
    block_sum2(ua, um, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const long nblk = (long)gridDim.x * gridDim.y;
        const long b = (long)blockIdx.z * nblk + blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * b] = ua;
        partial[2 * b + 1] = um;
    }
}

// The same through LDS: a workgroup owns 32 x 8 coarse nodes, stages u on
// the 67 x 19 fine nodes around them once (coalesced rows), forms A u and M u
// on the 65 x 17 fine nodes their restriction reaches, and then restricts
// from LDS.  It owns the fine nodes of the first 64 x 16 of those for the
// sums (coarse I, J = 1 .. nc over the grid, as above).
constexpr int BRX = 32, BRY = 8;                  // coarse nodes per workgroup
constexpr int BFX = 2 * BRX + 1, BFY = 2 * BRY + 1;  // fine nodes with A u, M u
constexpr int BUX = BFX + 2, BUY = BFY + 2;          // fine nodes of u (halo 1)
// ADD: u is the V-cycles' iterate before its last correction; the tile
// holds u + ecor (the FP32 correction, added in FP64) and the owned nodes of
// the corrected field are written to un (which must not alias u).
// ZF (single problems with edge weights): a 1D grid whose consecutive
// pieces of work are the right-hand sides of one tile, on one die (workgroup
// w runs on die w % 8), so the tile's weights are read from HBM once;
// otherwise tile (x, y) and right-hand side z from the 3D grid.
struct BorderWork {
    int ntx, nty, nrhs;  // tiles per direction and right-hand sides (ZF)
};
template <int KIND, bool ADD = false, bool ZF = false>
__global__ __launch_bounds__(256) void k_border_restrict_t(Grid g, Coef<double> cg, const double* __restrict__ u,
                                                          Grid gc, double* __restrict__ bc,
                                                          double* __restrict__ cc, double* __restrict__ partial,
                                                          long stride, long sc, const float* __restrict__ ecor,
                                                          double* __restrict__ un, BorderWork bw) {
    int bx, by, bz, nbx, nby;
    if (ZF) {
        const int total = bw.ntx * bw.nty * bw.nrhs;
        const int per = gridDim.x / 8;
        const int work = (blockIdx.x % 8) * per + blockIdx.x / 8;
        if (work >= total) return;  // uniform per workgroup
        bz = work % bw.nrhs;
        bx = (work / bw.nrhs) % bw.ntx;
        by = work / (bw.nrhs * bw.ntx);
        nbx = bw.ntx;
        nby = bw.nty;
    } else {
        bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
        nbx = gridDim.x, nby = gridDim.y;
    }
    __shared__ double us[BUY][BUX];
    __shared__ double as[BFY][BFX];
    __shared__ double ms[BFY][BFX];
    __shared__ double sh[8];
    const int tid = threadIdx.x;
    const int I0 = bx * BRX + 1, J0 = by * BRY + 1;  // first coarse node
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;                    // first fine node with A u
    double bs;
    const Coef<double> c = member_coef(cg, bz, bs);
    const double* ur = u + (long)bz * stride;
    const float* er = ADD ? ecor + (long)bz * stride : nullptr;
    // edge weights (single problems): the four weights of each node this
    // thread forms A u at, loaded with the tile so that no load waits after
    // the barrier
    constexpr int NC = (BFX * BFY + 255) / 256;
    constexpr bool PW = KIND == 1 && ZF;
    double pw[PW ? NC : 1][4];
    if constexpr (PW) {
        const int p = g.pitch;
#pragma unroll
        for (int e = 0; e < NC; ++e) {
            const int t = tid + 256 * e;
            const int a = t % BFX, b = t / BFX;
            const int i = fi0 + a, j = fj0 + b;
            const bool in = t < BFX * BFY && i <= g.m && j <= g.m;
            const long id = g.idx(in ? i : fi0, in ? j : fj0);
            pw[e][0] = c.wx[id], pw[e][1] = c.wx[id - 1], pw[e][2] = c.wy[id], pw[e][3] = c.wy[id - p];
        }
    }
    {
        // all of a thread's loads are issued before any of them is used
        constexpr int NPT = (BUX * BUY + 255) / 256;
        double v[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int t = tid + 256 * e;
            const int a = t % BUX, b = t / BUX;
            const int i = fi0 - 1 + a, j = fj0 - 1 + b;
            const bool in = t < BUX * BUY && i <= g.n && j <= g.n;
            v[e] = in ? ur[g.idx(i, j)] : 0.0;
            if (ADD) v[e] += in ? (double)er[g.idx(i, j)] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int t = tid + 256 * e;
            if (t < BUX * BUY) us[t / BUX][t % BUX] = v[e];
        }
    }
    __syncthreads();
    const double h2 = g.h * g.h;
    double ua = 0.0, um = 0.0;
#pragma unroll
    for (int e = 0; e < NC; ++e) {
        const int t = tid + 256 * e;
        if (t >= BFX * BFY) break;
        const int a = t % BFX, b = t / BFX;
        const int i = fi0 + a, j = fj0 + b;
        double Ax = 0.0, Mx = 0.0;
        if (i <= g.m && j <= g.m) {
            const double x0 = us[b + 1][a + 1];
            const double xe = us[b + 1][a + 2], xw = us[b + 1][a], xn = us[b + 2][a + 1], xs = us[b][a + 1];
            const double xne = us[b + 2][a + 2], xsw = us[b][a];
            if (KIND == 0) {
                Ax = c.w0 * (4.0 * x0 - xe - xw - xn - xs);
            } else if (PW) {
                const double we = pw[e][0], ww = pw[e][1], wn = pw[e][2], ws = pw[e][3];
                Ax = (we + ww + wn + ws) * x0 - we * xe - ww * xw - wn * xn - ws * xs;
            } else {
                const long id = g.idx(i, j);
                const int p = g.pitch;
                const double we = c.wx[id], ww = c.wx[id - 1], wn = c.wy[id], ws = c.wy[id - p];
                if (KIND == 1) {
                    Ax = (we + ww + wn + ws) * x0 - we * xe - ww * xw - wn * xn - ws * xs;
                } else {
                    Ax = c.d[id] * x0 - we * xe - ww * xw - wn * xn - ws * xs - c.wne[id] * xne -
                         c.wne[id - p - 1] * xsw;
                }
            }
            Mx = h2 * (0.5 * x0 + (xe + xw + xn + xs + xne + xsw) * (1.0 / 12.0));
            if (a < 2 * BRX && b < 2 * BRY) {  // owned
                ua += x0 * Ax;
                um += x0 * Mx;
                if (ADD) un[(long)bz * stride + g.idx(i, j)] = x0;
            }
        }
        as[b][a] = Ax;
        ms[b][a] = Mx;
    }
    __syncthreads();
    {
        const int cx = tid % BRX, cy = tid / BRX;
        const int I = I0 + cx, J = J0 + cy;
        if (I <= gc.m && J <= gc.m) {
            const int a = 2 * cx + 1, b = 2 * cy + 1;
            const double rb = as[b][a] + 0.5 * (as[b][a - 1] + as[b - 1][a] + as[b - 1][a - 1] + as[b][a + 1] +
                                                as[b + 1][a] + as[b + 1][a + 1]);
            const double rc = ms[b][a] + 0.5 * (ms[b][a - 1] + ms[b - 1][a] + ms[b - 1][a - 1] + ms[b][a + 1] +
                                                ms[b + 1][a] + ms[b + 1][a + 1]);
            const long cid = (long)bz * sc + gc.idx(I, J);
            bc[cid] = rb;
            cc[cid] = rc;
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
        const long nblk = (long)nbx * nby;
        const long blk = (long)bz * nblk + (long)by * nbx + bx;
        partial[2 * blk] = sh[0] + sh[2] + sh[4] + sh[6];
        partial[2 * blk + 1] = sh[1] + sh[3] + sh[5] + sh[7];
    }
}

// Prolongation and combination with the mass right-hand side of the next
// step in one pass: xn = P xc + beta[r] xo on every fine node, and
// f = lam[r] M xn on the workgroup's 64 x 16 nodes (xn on their one-node
// halo is formed again from xo and xc).  xn must not alias xo.  The coarse
// field may lie any power-of-two ratio R = 2^lr below: the spaces are nested,
// so the prolongation through all levels in between is the P1 interpolant on
// the coarse "/" triangles.  For a fine node in coarse cell (I, J) at
// offsets (a, b) < R, on the lower triangle (a >= b)
//   xn = ((R - a) x(I,J) + (a - b) x(I+1,J) + b x(I+1,J+1)) / R,
// on the upper one the same with the roles of a, b and of (I+1,J), (I,J+1)
// exchanged (R = 2 gives the midpoints of the coarse edges).
// RES (edge weights wx, wy of the fine level): instead of f, the next
// step's first residual r = lam M xn - A xn, rounded to FP32, with the
// arithmetic of the residual kernel (k_resid_cast with the mass term), so
// that it equals what that kernel would form from xn.
constexpr int PMX = 64, PMY = 16;
// A workgroup covers one tile for RB right-hand sides in turn (RES: the
// weights of its nodes are loaded once for all of them).
template <bool RES = false, int RB = 1>
__global__ __launch_bounds__(256) void k_prolong_mass(Grid gc, const double* __restrict__ xc, Grid gf,
                                                      const double* __restrict__ xo, double* __restrict__ xn,
                                                      double* __restrict__ f, long sc, long sf,
                                                      const double* __restrict__ beta,
                                                      const double* __restrict__ lam, int lr,
                                                      const double* __restrict__ wx, const double* __restrict__ wy,
                                                      float* __restrict__ r32, int nrhs) {
    constexpr int UX = PMX + 2, UY = PMY + 2, NPT = (UX * UY + 255) / 256, NO = PMX * PMY / 256;
    __shared__ double us[UY][UX];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * PMX + 1, j0 = blockIdx.y * PMY + 1;
    const int R = 1 << lr;
    const double invR = 1.0 / R;
    // the coarse nodes under the tile and its halo (at most 35 x 11 for R >= 2)
    constexpr int CSX = PMX / 2 + 3, CSY = PMY / 2 + 3;
    __shared__ double cs[CSY][CSX];
    const int I0 = (i0 - 1) >> lr, J0 = (j0 - 1) >> lr;
    const int CX = min(((i0 + PMX) >> lr) - I0 + 2, CSX), CY = min(((j0 + PMY) >> lr) - J0 + 2, CSY);
    bool ok[NPT];
    int ic_[NPT], jc_[NPT];
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
        const int t = tid + 256 * e;
        const int i = i0 - 1 + t % UX, j = j0 - 1 + t / UX;
        ok[e] = t < UX * UY && i >= 1 && i <= gf.m && j >= 1 && j <= gf.m;
        ic_[e] = ok[e] ? i : i0;
        jc_[e] = ok[e] ? j : j0;
    }
    // the thread's output nodes t = tid + 256 e and (RES) their four weights
    double w4[RES ? NO : 1][4];
    if constexpr (RES) {
        const int p = gf.pitch;
#pragma unroll
        for (int e = 0; e < NO; ++e) {
            const int t = tid + 256 * e;
            const int i = min(i0 + t % PMX, gf.m), j = min(j0 + t / PMX, gf.m);
            const long gid = gf.idx(i, j);
            w4[e][0] = wx[gid], w4[e][1] = wx[gid - 1], w4[e][2] = wy[gid], w4[e][3] = wy[gid - p];
        }
    }
    const double h2 = gf.h * gf.h;
    for (int q = 0; q < RB; ++q) {
        const int z = blockIdx.z * RB + q;
        if (z >= nrhs) break;  // uniform per workgroup
        if (q > 0) __syncthreads();  // the previous right-hand side's tile is consumed
        const double* cr = xc + (long)z * sc;
        const double* xr = xo + (long)z * sf;
        const double bz = beta[z], lz = lam[z];
        double xv[NPT];
#pragma unroll
        for (int e = 0; e < NPT; ++e) xv[e] = xr[gf.idx(ic_[e], jc_[e])];
        for (int t = tid; t < CX * CY; t += 256) {
            const int a = t % CX, b = t / CX;
            cs[b][a] = cr[gc.idx(min(I0 + a, gc.n), min(J0 + b, gc.n))];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int t = tid + 256 * e;
            const int a = ic_[e] & (R - 1), b = jc_[e] & (R - 1);
            const int ir = (ic_[e] >> lr) - I0, jr = (jc_[e] >> lr) - J0;  // within the staged block
            const bool lower = a >= b;
            const int wa = lower ? a : b, wb = lower ? b : a;  // the larger and the smaller offset
            const double c0 = cs[jr][ir], c1 = lower ? cs[jr][ir + 1] : cs[jr + 1][ir], c2 = cs[jr + 1][ir + 1];
            // explicit fused multiply-adds: the marching pre-smoothing that
            // forms the same field on the fly rounds identically
            double v =
                __builtin_fma((double)wb, c2, __builtin_fma((double)(wa - wb), c1, (double)(R - wa) * c0)) * invR;
            if (bz != 0.0) v = __builtin_fma(bz, xv[e], v);  // a zero weight drops the old field (whatever it holds)
            if (t < UX * UY) us[t / UX][t % UX] = ok[e] ? v : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < NO; ++e) {
            const int t = tid + 256 * e;
            const int a = t % PMX, b = t / PMX;
            const int i = i0 + a, j = j0 + b;
            if (i > gf.m || j > gf.m) continue;
            const double x0 = us[b + 1][a + 1];
            const double sn = us[b + 1][a + 2] + us[b + 1][a] + us[b + 2][a + 1] + us[b][a + 1] + us[b + 2][a + 2] +
                              us[b][a];
            const long gid = gf.idx(i, j), id = (long)z * sf + gid;
            xn[id] = x0;
            const double fv = lz * (h2 * __builtin_fma(sn, 1.0 / 12.0, 0.5 * x0));
            if constexpr (RES) {
                const double we = w4[e][0], ww = w4[e][1], wn = w4[e][2], ws = w4[e][3];
                const double D = we + ww + wn + ws;
                const double Ax = D * x0 - we * us[b + 1][a + 2] - ww * us[b + 1][a] - wn * us[b + 2][a + 1] -
                                  ws * us[b][a + 1];
                r32[id] = (float)(fv - Ax);
            } else {
                if (f) f[id] = fv;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_reduce_pairs(const double* __restrict__ partial, int nblk,
                                                      double* __restrict__ out) {
    __shared__ double sh[8];
    const double* pr = partial + 2L * nblk * blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < nblk; t += 256) {
        a += pr[2 * t];
        b += pr[2 * t + 1];
    }
    // reuse the 64 x 4 reduction with a flat block of 256
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[2 * w] = a;
        sh[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = sh[0] + sh[2] + sh[4] + sh[6];
        out[2 * blockIdx.x + 1] = sh[1] + sh[3] + sh[5] + sh[7];
    }
}

template <typename T>
__global__ void k_pack(Grid g, const T* __restrict__ padded, long sp, double* __restrict__ compact, long ld) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    compact[(long)blockIdx.z * ld + (long)(j - 1) * g.m + (i - 1)] =
        (double)padded[(long)blockIdx.z * sp + g.idx(i, j)];
}

template <typename T>
__global__ void k_unpack(Grid g, const double* __restrict__ compact, long ld, T* __restrict__ padded, long sp) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    if (i > g.m || j > g.m) return;
    padded[(long)blockIdx.z * sp + g.idx(i, j)] =
        (T)compact[(long)blockIdx.z * ld + (long)(j - 1) * g.m + (i - 1)];
}

__global__ void k_fill_zero(uint32_t* p, size_t n) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        p[t] = 0u;
}

inline int flat_blocks(long n) {
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers (2D only here; the 3D kernels live in stencil3d.hip)
// ---------------------------------------------------------------------------
template <typename T>
void launch_smooth3(const Grid& g, const Coef<T>& c, const T* xc, const T* xp, const T* f, T* xn,
                    int nrhs, long stride, Cheb s, int zmode, hipStream_t st);
template <typename T>
void launch_resid_restrict3(const Grid& gf, const Coef<T>& c, const T* x, const T* f, const Grid& gc,
                            T* rc, int nrhs, long sf, long sc, hipStream_t st);
template <typename T>
void launch_prolong3(const Grid& gc, const T* xc, const Grid& gf, T* xf, int nrhs, long sc, long sf,
                     int mode, const double* beta, hipStream_t st);
template <typename T>
void launch_restrict3(const Grid& gf, const T* xf, const Grid& gc, T* xc, int nrhs, long sf, long sc,
                      hipStream_t st);
template <typename T>
void launch_apply_A3(const Grid& g, const Coef<T>& c, const T* x, T* y, int nrhs, long stride, hipStream_t st);
void launch_mass_rhs3(const Grid& g, const double* u, const double* lam, double* f, int nrhs, long stride,
                      hipStream_t st);
int launch_border3(const Grid& g, const Coef<double>& c, const double* u, double* au, double* mu,
                   double* partial, int nrhs, long stride, hipStream_t st);
template <typename T>
void launch_pack3(const Grid& g, const T* padded, long sp, double* compact, long ld, int nrhs, hipStream_t st);
template <typename T>
void launch_unpack3(const Grid& g, const double* compact, long ld, T* padded, long sp, int nrhs, hipStream_t st);

template <typename T>
void launch_smooth(const Grid& g, const Coef<T>& c, const T* xc, const T* xp, const T* f, T* xn,
                   int nrhs, long stride, Cheb s, int zmode, hipStream_t st) {
    if (g.dim == 3) return launch_smooth3<T>(g, c, xc, xp, f, xn, nrhs, stride, s, zmode, st);
    dim3 grid = grid_for(g.m, g.m, nrhs), blk(BX, BY);
    switch (coef_kind(c)) {
        case 0: hipLaunchKernelGGL((k_smooth<T, 0>), grid, blk, 0, st, g, c, xc, xp, f, xn, stride, (T)s.a, (T)s.b, zmode); break;
        case 1: hipLaunchKernelGGL((k_smooth<T, 1>), grid, blk, 0, st, g, c, xc, xp, f, xn, stride, (T)s.a, (T)s.b, zmode); break;
        default: hipLaunchKernelGGL((k_smooth<T, 2>), grid, blk, 0, st, g, c, xc, xp, f, xn, stride, (T)s.a, (T)s.b, zmode); break;
    }
    PASM_CHECK_LAUNCH();
}

// LDS of a fused launch: the double-buffered iterate plus 0 / 2 / 4
// coefficient tiles (constant / edge / general).
constexpr size_t fused_lds(int kind, size_t elem, int rows) {
    return (2 + (kind == 0 ? 0 : kind == 1 ? 2 : 4)) * (size_t)64 * 4 * rows * elem;
}
constexpr size_t kLdsLimit = 65536;
// right-hand sides a fused workgroup smooths with one staged coefficient tile
constexpr int kFusedRhsPerBlock = 8;

size_t fused_lds_bytes(int kind, size_t elem, int rows) { return fused_lds(kind, elem, rows); }

template <typename T, int KIND, int S, int ROWS>
void fused_launch(const Grid& g, const Coef<T>& c, const T* x0, const T* f, T* out, int nrhs, long stride,
                  const SmoothSteps& ss, bool x_zero, hipStream_t st) {
    if constexpr (fused_lds(KIND, sizeof(T), ROWS) <= kLdsLimit && 4 * ROWS - 2 * S > 0) {
        constexpr int TX = 64 - 2 * S, TY = 4 * ROWS - 2 * S;
        // right-hand sides that share coefficients: all of them for one
        // problem, a member's for a batch; constant coefficients need no sharing
        int share = (KIND == 0) ? 1 : (c.ms == 0 ? nrhs : c.kpm);
        if (share < 1 || nrhs % share != 0) share = 1;
        // group right-hand sides only as far as the grid keeps ~2048 workgroups
        const long tiles = (long)((g.m + TX - 1) / TX) * ((g.m + TY - 1) / TY);
        const int rb = (int)std::max<long>(1, std::min<long>({(long)share, (long)kFusedRhsPerBlock,
                                                              tiles * nrhs / 2048}));
        const int zb = (share + rb - 1) / rb;
        dim3 grid((g.m + TX - 1) / TX, (g.m + TY - 1) / TY, (nrhs / share) * zb);
        hipLaunchKernelGGL((k_smooth_fused<T, KIND, S, ROWS>), grid, dim3(64, 4), 0, st, g, c, x0, f, out, stride,
                           ss, (int)x_zero, share, rb);
        PASM_CHECK_LAUNCH();
    } else {
        throw Error(PASM_E_INVALID, "fused smoothing tile too large for LDS or too short for the steps");
    }
}

template <typename T, int S, int ROWS>
void fused_kind(const Grid& g, const Coef<T>& c, const T* x0, const T* f, T* out, int nrhs, long stride,
                const SmoothSteps& ss, bool x_zero, hipStream_t st) {
    switch (coef_kind(c)) {
        case 0: fused_launch<T, 0, S, ROWS>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st); break;
        case 1: fused_launch<T, 1, S, ROWS>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st); break;
        default: fused_launch<T, 2, S, ROWS>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st); break;
    }
}

template <typename T, int S>
void fused_dispatch(const Grid& g, const Coef<T>& c, const T* x0, const T* f, T* out, int nrhs, long stride,
                    const SmoothSteps& ss, bool x_zero, hipStream_t st, int rows) {
    switch (rows) {
        case 2: fused_kind<T, S, 2>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st); break;
        case 4: fused_kind<T, S, 4>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st); break;
        default: fused_kind<T, S, 8>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st); break;
    }
}

bool fused_supported(const Grid& g, int steps) { return g.dim == 2 && steps >= 1 && steps <= 4; }

template <typename T>
bool launch_smooth_fused(const Grid& g, const Coef<T>& c, const T* x0, const T* f, T* out, int nrhs, long stride,
                         const SmoothSteps& ss, bool x_zero, hipStream_t st, int rows) {
    if (!fused_supported(g, ss.s)) return false;
    if (rows != 2 && rows != 4 && rows != 8) return false;
    if (4 * rows - 2 * ss.s <= 0) return false;
    if (fused_lds(coef_kind(c), sizeof(T), rows) > kLdsLimit) return false;
    switch (ss.s) {
        case 1: fused_dispatch<T, 1>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st, rows); return true;
        case 2: fused_dispatch<T, 2>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st, rows); return true;
        case 3: fused_dispatch<T, 3>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st, rows); return true;
        case 4:
            if (rows == 2) return false;  // a 4-step phase needs more than 8 LDS rows
            fused_dispatch<T, 4>(g, c, x0, f, out, nrhs, stride, ss, x_zero, st, rows);
            return true;
        default: return false;
    }
}

template <typename T>
void launch_apply_A(const Grid& g, const Coef<T>& c, const T* x, T* y, int nrhs, long stride,
                    hipStream_t st) {
    if (g.dim == 3) return launch_apply_A3<T>(g, c, x, y, nrhs, stride, st);
    dim3 grid = grid_for(g.m, g.m, nrhs), blk(BX, BY);
    switch (coef_kind(c)) {
        case 0: hipLaunchKernelGGL((k_apply_A<T, 0>), grid, blk, 0, st, g, c, x, y, stride); break;
        case 1: hipLaunchKernelGGL((k_apply_A<T, 1>), grid, blk, 0, st, g, c, x, y, stride); break;
        default: hipLaunchKernelGGL((k_apply_A<T, 2>), grid, blk, 0, st, g, c, x, y, stride); break;
    }
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_resid_restrict(const Grid& gf, const Coef<T>& c, const T* x, const T* f, const Grid& gc,
                           T* rc, int nrhs, long sf, long sc, hipStream_t st) {
    if (gf.dim == 3) return launch_resid_restrict3<T>(gf, c, x, f, gc, rc, nrhs, sf, sc, st);
    dim3 grid = grid_for(gc.m, gc.m, nrhs), blk(BX, BY);
    switch (coef_kind(c)) {
        case 0: hipLaunchKernelGGL((k_resid_restrict<T, 0>), grid, blk, 0, st, gf, c, x, f, gc, rc, sf, sc); break;
        case 1: hipLaunchKernelGGL((k_resid_restrict<T, 1>), grid, blk, 0, st, gf, c, x, f, gc, rc, sf, sc); break;
        default: hipLaunchKernelGGL((k_resid_restrict<T, 2>), grid, blk, 0, st, gf, c, x, f, gc, rc, sf, sc); break;
    }
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_prolong(const Grid& gc, const T* xc, const Grid& gf, T* xf, int nrhs, long sc, long sf,
                    bool add, const double* beta, hipStream_t st) {
    const int mode = beta ? 2 : (add ? 1 : 0);
    if (gf.dim == 3) return launch_prolong3<T>(gc, xc, gf, xf, nrhs, sc, sf, mode, beta, st);
    dim3 grid = grid_for(gf.m, gf.m, nrhs), blk(BX, BY);
    hipLaunchKernelGGL((k_prolong<T>), grid, blk, 0, st, gc, xc, gf, xf, sc, sf, mode, beta);
    PASM_CHECK_LAUNCH();
}

void launch_prolong_mass(const Grid& gc, const double* xc, const Grid& gf, const double* xo, double* xn,
                         double* f, int nrhs, long sc, long sf, const double* beta, const double* lam,
                         hipStream_t st, const double* wx, const double* wy, float* r32) {
    if (xn == xo) throw Error(PASM_E_INVALID, "prolong with mass: separate output");
    if (r32 && (gf.dim != 2 || !wx || !wy || f))
        throw Error(PASM_E_INVALID, "prolong with the first residual: 2D edge weights, no f");
    if (gf.dim == 3) {
        if (gc.n * 2 != gf.n) throw Error(PASM_E_INVALID, "prolong with mass (3D): ratio 2");
        return launch_prolong_mass3(gc, xc, gf, xo, xn, f, nrhs, sc, sf, beta, lam, st);
    }
    int lr = 0;
    while ((gc.n << lr) < gf.n) ++lr;
    if (lr < 1 || (gc.n << lr) != gf.n) throw Error(PASM_E_INVALID, "prolong with mass: power-of-two ratio");
    dim3 grid((gf.m + PMX - 1) / PMX, (gf.m + PMY - 1) / PMY, nrhs);
    if (r32) {
        constexpr int RB = 5;
        grid.z = (nrhs + RB - 1) / RB;
        hipLaunchKernelGGL((k_prolong_mass<true, RB>), grid, dim3(256), 0, st, gc, xc, gf, xo, xn, f, sc, sf, beta,
                           lam, lr, wx, wy, r32, nrhs);
    } else {
        hipLaunchKernelGGL((k_prolong_mass<false, 1>), grid, dim3(256), 0, st, gc, xc, gf, xo, xn, f, sc, sf, beta,
                           lam, lr, wx, wy, r32, nrhs);
    }
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_restrict(const Grid& gf, const T* xf, const Grid& gc, T* xc, int nrhs, long sf, long sc,
                     hipStream_t st) {
    if (gf.dim == 3) return launch_restrict3<T>(gf, xf, gc, xc, nrhs, sf, sc, st);
    dim3 grid = grid_for(gc.m, gc.m, nrhs), blk(BX, BY);
    hipLaunchKernelGGL((k_restrict<T>), grid, blk, 0, st, gf, xf, gc, xc, sf, sc);
    PASM_CHECK_LAUNCH();
}

void launch_restrict_chain3(const Grid& g3, const double* x3, const Grid& g2, const Grid& g1, const Grid& g0,
                            double* x0, int nrhs, long s3, long s0, hipStream_t st) {
    if (g3.dim != 2 || g2.n * 2 != g3.n || g1.n * 2 != g2.n || g0.n * 2 != g1.n)
        throw Error(PASM_E_INVALID, "chained restriction: 2D levels of ratio 2");
    dim3 grid((g0.m + RC_T - 1) / RC_T, (g0.m + RC_T - 1) / RC_T, nrhs);
    hipLaunchKernelGGL(k_restrict_chain3, grid, dim3(256), 0, st, g3, x3, g2, g1, g0, x0, s3, s0);
    PASM_CHECK_LAUNCH();
}

void launch_mass_rhs(const Grid& g, const double* u, const double* lam, double* f, int nrhs, long stride,
                     hipStream_t st) {
    if (g.dim == 3) return launch_mass_rhs3(g, u, lam, f, nrhs, stride, st);
    dim3 grid = grid_for(g.m, g.m, nrhs), blk(BX, BY);
    hipLaunchKernelGGL(k_mass_rhs, grid, blk, 0, st, g, u, lam, f, stride);
    PASM_CHECK_LAUNCH();
}

void launch_apply_M(const Grid& g, const double* x, double* y, int nrhs, long stride, hipStream_t st) {
    launch_mass_rhs(g, x, nullptr, y, nrhs, stride, st);
}

void launch_resid_cast(const Grid& g, const Coef<double>& c, const double* u, const double* f, float* r,
                       int nrhs, long stride, hipStream_t st, const double* lam) {
    if (lam && g.dim == 3) return launch_resid_cast3(g, c, u, f, r, nrhs, stride, st, lam);
    if (lam) {
        if (!mass_rhs_fusable(g, c)) throw Error(PASM_E_INVALID, "residual with lam M u: 2D edge weights only");
        constexpr int RB = 4;
        const dim3 gr = grid_for(g.m, g.m, (nrhs + RB - 1) / RB), blk(BX, BY);
        hipLaunchKernelGGL((k_resid_cast<1, float, RB, true>), gr, blk, 0, st, g, c, u, f, r, stride, stride, nrhs,
                           lam);
        PASM_CHECK_LAUNCH();
        return;
    }
    if (g.dim == 3) return launch_resid_cast3(g, c, u, f, r, nrhs, stride, st);
    launch_resid_to<float>(g, c, u, f, r, nrhs, stride, st);
}

bool mass_rhs_fusable(const Grid& g, const Coef<double>& c) {
    if (c.kpm > 1 || c.ms != 0) return false;
    return (g.dim == 2 && coef_kind(c) == 1) || (g.dim == 3 && (coef_kind(c) == 0 || c.s15));
}

template <typename TO>
void launch_resid_to(const Grid& g, const Coef<double>& c, const double* u, const double* f, TO* r, int nrhs,
                     long stride, hipStream_t st) {
    if (g.dim == 3) throw Error(PASM_E_INVALID, "residual kernel: 2D only");
    dim3 grid = grid_for(g.m, g.m, nrhs), blk(BX, BY);
    const bool single = c.kpm <= 1 && c.ms == 0;
    switch (coef_kind(c)) {
        case 0: hipLaunchKernelGGL((k_resid_cast<0, TO>), grid, blk, 0, st, g, c, u, f, r, stride, stride, nrhs,
                               nullptr);
            break;
        case 1:
            if (single) {
                constexpr int RB = 4;
                const dim3 gr = grid_for(g.m, g.m, (nrhs + RB - 1) / RB);
                hipLaunchKernelGGL((k_resid_cast<1, TO, RB>), gr, blk, 0, st, g, c, u, f, r, stride, stride, nrhs,
                                   nullptr);
            } else {
                hipLaunchKernelGGL((k_resid_cast<1, TO>), grid, blk, 0, st, g, c, u, f, r, stride, stride, nrhs,
                                   nullptr);
            }
            break;
        default:
            hipLaunchKernelGGL((k_resid_cast<2, TO>), grid, blk, 0, st, g, c, u, f, r, stride, stride, nrhs,
                               nullptr);
            break;
    }
    PASM_CHECK_LAUNCH();
}
template void launch_resid_to<float>(const Grid&, const Coef<double>&, const double*, const double*, float*, int,
                                     long, hipStream_t);
template void launch_resid_to<double>(const Grid&, const Coef<double>&, const double*, const double*, double*, int,
                                      long, hipStream_t);

namespace {
// Right-hand sides per thread of the member passes: the largest of 5, 4, 2
// that divides the right-hand sides per member.
int member_rb(const Coef<double>& c) {
    const int kpm = std::max(1, c.kpm);
    for (int rb : {5, 4, 2})
        if (kpm % rb == 0) return rb;
    return 1;
}
template <int KIND, bool ADD>
void launch_mass_m(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un, float* r,
                   int nrhs, long stride, const double* lam, hipStream_t st) {
    const int rb = member_rb(c);
    const dim3 gr = grid_for(g.m, g.m, nrhs / rb), blk(BX, BY);
    switch (rb) {
        case 5: hipLaunchKernelGGL((k_resid_mass_m<KIND, 5, ADD>), gr, blk, 0, st, g, c, u, e, un, r, stride, lam); break;
        case 4: hipLaunchKernelGGL((k_resid_mass_m<KIND, 4, ADD>), gr, blk, 0, st, g, c, u, e, un, r, stride, lam); break;
        case 2: hipLaunchKernelGGL((k_resid_mass_m<KIND, 2, ADD>), gr, blk, 0, st, g, c, u, e, un, r, stride, lam); break;
        default: hipLaunchKernelGGL((k_resid_mass_m<KIND, 1, ADD>), gr, blk, 0, st, g, c, u, e, un, r, stride, lam); break;
    }
    PASM_CHECK_LAUNCH();
}
}  // namespace

void launch_resid_mass_members(const Grid& g, const Coef<double>& c, const double* u, const double* lam, float* r,
                               int nrhs, long stride, hipStream_t st) {
    const int kind = coef_kind(c);
    if (g.dim != 2 || (kind != 1 && kind != 2) || nrhs % std::max(1, c.kpm) != 0)
        throw Error(PASM_E_INVALID, "residual with lam M u: 2D, edge weights or the general operator, whole members");
    if (kind == 2) launch_mass_m<2, false>(g, c, u, nullptr, nullptr, r, nrhs, stride, lam, st);
    else launch_mass_m<1, false>(g, c, u, nullptr, nullptr, r, nrhs, stride, lam, st);
}

void launch_add_resid_members(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un,
                              float* r, int nrhs, long stride, const double* lam, hipStream_t st) {
    const int kind = coef_kind(c);
    if (g.dim != 2 || (kind != 1 && kind != 2) || un == u || nrhs % std::max(1, c.kpm) != 0)
        throw Error(PASM_E_INVALID, "add and residual of members: 2D, 5- or 7-point operator, separate output");
    if (kind == 2) launch_mass_m<2, true>(g, c, u, e, un, r, nrhs, stride, lam, st);
    else launch_mass_m<1, true>(g, c, u, e, un, r, nrhs, stride, lam, st);
}

void launch_add_correction(const float* e, double* u, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_add_correction<float>, dim3(flat_blocks(n)), dim3(256), 0, st, e, u, n);
    PASM_CHECK_LAUNCH();
}
bool add_resid_supported(const Grid& g, const Coef<double>& c) {
    return g.dim == 3 || (coef_kind(c) <= 1 && c.kpm <= 1 && c.ms == 0);
}

void launch_add_resid(const Grid& g, const Coef<double>& c, const double* u, const float* e, const double* f,
                      double* un, float* r, int nrhs, long stride, hipStream_t st, const double* lam) {
    if (lam && !mass_rhs_fusable(g, c)) throw Error(PASM_E_INVALID, "add and residual with lam M u: 2D edge weights");
    if (g.dim == 3) return launch_add_resid3(g, c, u, e, f, un, r, nrhs, stride, st, lam);
    if (!add_resid_supported(g, c) || un == u)
        throw Error(PASM_E_INVALID, "add and residual: 2D constant or edge-weight operator, separate output");
    dim3 grid = grid_for(g.m, g.m, nrhs), blk(BX, BY);
    if (coef_kind(c) == 0) {
        hipLaunchKernelGGL((k_add_resid<0, 1>), grid, blk, 0, st, g, c, u, e, f, un, r, stride, nrhs, nullptr);
    } else {
        constexpr int RB = 4;
        const dim3 gr = grid_for(g.m, g.m, (nrhs + RB - 1) / RB);
        if (lam)
            hipLaunchKernelGGL((k_add_resid<1, RB, true>), gr, blk, 0, st, g, c, u, e, f, un, r, stride, nrhs, lam);
        else
            hipLaunchKernelGGL((k_add_resid<1, RB>), gr, blk, 0, st, g, c, u, e, f, un, r, stride, nrhs, nullptr);
    }
    PASM_CHECK_LAUNCH();
}

void launch_resid_of_sum(const Grid& g, const Coef<double>& c, const double* u, const float* e, const double* f,
                         float* r, int nrhs, long stride, hipStream_t st, const double* lam) {
    if (!rows_supported(g, c) || (lam && !mass_rhs_fusable(g, c)))
        throw Error(PASM_E_INVALID, "residual of u + e without storing it: 2D edge weights of a single problem");
    constexpr int RB = 4;
    const dim3 gr = grid_for(g.m, g.m, (nrhs + RB - 1) / RB), blk(BX, BY);
    if (lam)
        hipLaunchKernelGGL((k_add_resid<1, RB, true, false>), gr, blk, 0, st, g, c, u, e, f, (double*)nullptr, r,
                           stride, nrhs, lam);
    else
        hipLaunchKernelGGL((k_add_resid<1, RB, false, false>), gr, blk, 0, st, g, c, u, e, f, (double*)nullptr, r,
                           stride, nrhs, nullptr);
    PASM_CHECK_LAUNCH();
}

void launch_add_correction(const double* e, double* u, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_add_correction<double>, dim3(flat_blocks(n)), dim3(256), 0, st, e, u, n);
    PASM_CHECK_LAUNCH();
}

int launch_border(const Grid& g, const Coef<double>& c, const double* u, double* au, double* mu,
                  double* partial, int nrhs, long stride, hipStream_t st) {
    if (g.dim == 3) return launch_border3(g, c, u, au, mu, partial, nrhs, stride, st);
    dim3 grid = grid_for(g.m, g.m, nrhs), blk(BX, BY);
    switch (coef_kind(c)) {
        case 0: hipLaunchKernelGGL(k_border<0>, grid, blk, 0, st, g, c, u, au, mu, partial, stride); break;
        case 1: hipLaunchKernelGGL(k_border<1>, grid, blk, 0, st, g, c, u, au, mu, partial, stride); break;
        default: hipLaunchKernelGGL(k_border<2>, grid, blk, 0, st, g, c, u, au, mu, partial, stride); break;
    }
    PASM_CHECK_LAUNCH();
    return (int)(grid.x * grid.y);
}

int launch_border_restrict(const Grid& g, const Coef<double>& c, const double* u, const Grid& gc, double* bc,
                           double* cc, double* partial, int nrhs, long stride, long sc, hipStream_t st) {
    if (g.dim != 2 || gc.n * 2 != g.n) throw Error(PASM_E_INVALID, "fused border restriction: 2D, ratio 2");
    dim3 grid((gc.n + BRX - 1) / BRX, (gc.n + BRY - 1) / BRY, nrhs), blk(256);
    const float* e0 = nullptr;
    double* u0 = nullptr;
    const BorderWork bw{(int)grid.x, (int)grid.y, nrhs};
    switch (coef_kind(c)) {
        case 0: hipLaunchKernelGGL(k_border_restrict_t<0>, grid, blk, 0, st, g, c, u, gc, bc, cc, partial, stride, sc, e0, u0, bw); break;
        case 1:
            if (c.kpm <= 1 && c.ms == 0) {
                const int total = (int)(grid.x * grid.y) * nrhs;
                hipLaunchKernelGGL((k_border_restrict_t<1, false, true>), dim3((total + 7) / 8 * 8), blk, 0, st, g, c, u,
                                   gc, bc, cc, partial, stride, sc, e0, u0, bw);
            } else {
                hipLaunchKernelGGL(k_border_restrict_t<1>, grid, blk, 0, st, g, c, u, gc, bc, cc, partial, stride, sc, e0, u0, bw);
            }
            break;
        default: hipLaunchKernelGGL(k_border_restrict_t<2>, grid, blk, 0, st, g, c, u, gc, bc, cc, partial, stride, sc, e0, u0, bw); break;
    }
    PASM_CHECK_LAUNCH();
    return (int)(grid.x * grid.y);
}

int launch_border_restrict_add(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un,
                               const Grid& gc, double* bc, double* cc, double* partial, int nrhs, long stride, long sc,
                               hipStream_t st, const float* e0) {
    if (g.dim != 2 || gc.n * 2 != g.n || un == u || coef_kind(c) > 2)
        throw Error(PASM_E_INVALID, "correction with borders: 2D, ratio 2, 5- or 7-point operator, separate output");
    if (e0) {
        // two corrections: un = (u + e0) + e
        if (!rows_supported(g, c))
            throw Error(PASM_E_INVALID, "two corrections with borders: 2D edge weights of a single problem");
        return launch_border_rows(g, c, u, e, un, gc, bc, cc, partial, nrhs, stride, sc, border_partial_blocks(g), st,
                                  e0);
    }
    if (coef_kind(c) == 2 || c.kpm > 1 || c.ms != 0) {
        // the general operator or batch members: the tile kernel, each
        // right-hand side with its member's coefficient planes
        // (consecutive pieces of work are the right-hand sides of one tile,
        // on one die: a member's coefficient tile is read from HBM once)
        if (coef_kind(c) == 0) throw Error(PASM_E_INVALID, "correction with borders: members need coefficient planes");
        const int ntx = (gc.n + BRX - 1) / BRX, nty = (gc.n + BRY - 1) / BRY;
        const BorderWork bw{ntx, nty, nrhs};
        const int total = ntx * nty * nrhs;
        const dim3 grid((total + 7) / 8 * 8), blk(256);
        if (coef_kind(c) == 2)
            hipLaunchKernelGGL((k_border_restrict_t<2, true, true>), grid, blk, 0, st, g, c, u, gc, bc, cc, partial,
                               stride, sc, e, un, bw);
        else
            hipLaunchKernelGGL((k_border_restrict_t<1, true, true>), grid, blk, 0, st, g, c, u, gc, bc, cc, partial,
                               stride, sc, e, un, bw);
        PASM_CHECK_LAUNCH();
        return ntx * nty;
    }
    if (rows_supported(g, c))
        return launch_border_rows(g, c, u, e, un, gc, bc, cc, partial, nrhs, stride, sc, border_partial_blocks(g), st);
    dim3 grid((gc.n + BRX - 1) / BRX, (gc.n + BRY - 1) / BRY, nrhs), blk(256);
    const BorderWork bw{(int)grid.x, (int)grid.y, nrhs};
    if (coef_kind(c) == 0) {
        hipLaunchKernelGGL((k_border_restrict_t<0, true>), grid, blk, 0, st, g, c, u, gc, bc, cc, partial, stride, sc, e, un,
                           bw);
    } else {
        const int total = (int)(grid.x * grid.y) * nrhs;
        hipLaunchKernelGGL((k_border_restrict_t<1, true, true>), dim3((total + 7) / 8 * 8), blk, 0, st, g, c, u, gc, bc, cc,
                           partial, stride, sc, e, un, bw);
    }
    PASM_CHECK_LAUNCH();
    return (int)(grid.x * grid.y);
}

void launch_reduce_pairs(const double* partial, int nblk, double* out, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_pairs, dim3(nrhs), dim3(256), 0, st, partial, nblk, out);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_pack(const Grid& g, const T* padded, long sp, double* compact, long ld, int nrhs, hipStream_t st) {
    if (g.dim == 3) return launch_pack3<T>(g, padded, sp, compact, ld, nrhs, st);
    hipLaunchKernelGGL((k_pack<T>), grid_for(g.m, g.m, nrhs), dim3(BX, BY), 0, st, g, padded, sp, compact, ld);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_unpack(const Grid& g, const double* compact, long ld, T* padded, long sp, int nrhs, hipStream_t st) {
    if (g.dim == 3) return launch_unpack3<T>(g, compact, ld, padded, sp, nrhs, st);
    hipLaunchKernelGGL((k_unpack<T>), grid_for(g.m, g.m, nrhs), dim3(BX, BY), 0, st, g, compact, ld, padded, sp);
    PASM_CHECK_LAUNCH();
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    hipLaunchKernelGGL(k_fill_zero, dim3(flat_blocks((long)n)), dim3(256), 0, st, (uint32_t*)p, n);
    PASM_CHECK_LAUNCH();
}

#define PASM_INST(T)                                                                                  \
    template void launch_smooth<T>(const Grid&, const Coef<T>&, const T*, const T*, const T*, T*, int,  \
                                   long, Cheb, int, hipStream_t);                                      \
    template void launch_apply_A<T>(const Grid&, const Coef<T>&, const T*, T*, int, long, hipStream_t); \
    template bool launch_smooth_fused<T>(const Grid&, const Coef<T>&, const T*, const T*, T*, int, long,      \
                                         const SmoothSteps&, bool, hipStream_t, int);                         \
    template void launch_resid_restrict<T>(const Grid&, const Coef<T>&, const T*, const T*, const Grid&, \
                                           T*, int, long, long, hipStream_t);                           \
    template void launch_prolong<T>(const Grid&, const T*, const Grid&, T*, int, long, long, bool,      \
                                    const double*, hipStream_t);                                        \
    template void launch_restrict<T>(const Grid&, const T*, const Grid&, T*, int, long, long,           \
                                     hipStream_t);                                                      \
    template void launch_pack<T>(const Grid&, const T*, long, double*, long, int, hipStream_t);         \
    template void launch_unpack<T>(const Grid&, const double*, long, T*, long, int, hipStream_t);
PASM_INST(double)
PASM_INST(float)
#undef PASM_INST

}  // namespace pasm

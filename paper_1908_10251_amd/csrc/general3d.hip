// General 3D operators on the Kuhn mesh: -div(A grad u) + V u with a full,
// symmetric diffusion tensor A_T and a potential V_T constant per element
// (the second example of Section 5: A = I + (x - 1/2)(x - 1/2)^T,
// V = exp(prod (x_i - 1/2)), taken at element centroids).
//
// With a full tensor the P1 element stiffness couples every edge of a Kuhn
// tetrahedron, so the operator is a 15-point stencil: the node itself and
// +-o for the seven edge directions o of the Kuhn mesh,
//     O = (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,0,1) (0,1,1) (1,1,1).
// Stored per level as 8 planes in the padded layout: a0 the diagonal, a_t
// the matrix entry A(i, i + O_t) (t = 1..7); A(i, i - O_t) = a_t(i - O_t).
// Entries that touch a boundary node are zero, so kernels need no branches.
// Coarse levels are Galerkin products P^T A P; P1 interpolation on nested
// Kuhn meshes keeps them 15-point (a coarse basis function is 1 at 2I and
// 1/2 at the 14 fine nodes 2I +- O_t), formed here on the host.
#include <cmath>

#include "common.h"

namespace pasm {

namespace {
constexpr int OX[8] = {0, 1, 0, 0, 1, 1, 0, 1};
constexpr int OY[8] = {0, 0, 1, 0, 1, 0, 1, 1};
constexpr int OZ[8] = {0, 0, 0, 1, 0, 1, 1, 1};

inline long hidx(const Grid& g, int i, int j, int l) { return g.idx(i, j, l); }
inline bool interior(const Grid& g, int i, int j, int l) {
    return i >= 1 && j >= 1 && l >= 1 && i <= g.m && j <= g.m && l <= g.m;
}
// t of the direction (dx, dy, dz) in O, or -1
inline int dir_of(int dx, int dy, int dz) {
    for (int t = 1; t < 8; ++t)
        if (OX[t] == dx && OY[t] == dy && OZ[t] == dz) return t;
    return -1;
}
}  // namespace

Stencil15 fine_stencil_3d(const Grid& g, const std::vector<double>& tensor, const std::vector<double>& kap,
                          const std::vector<double>& pot) {
    Stencil15 s;
    for (auto& a : s.a) a.assign(g.plane, 0.0);
    const int n = g.n;
    const double h = g.h, vol = h * h * h / 6.0;
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int cl = 0; cl < n; ++cl)
        for (int cj = 0; cj < n; ++cj)
            for (int ci = 0; ci < n; ++ci) {
                const long cell = ((long)cl * n + cj) * n + ci;
                for (int p = 0; p < 6; ++p) {
                    const long e = cell * 6 + p;
                    // vertices along the monotone path, gradients of the
                    // barycentric functions: -e_p0, e_p0 - e_p1, e_p1 - e_p2, e_p2 (over h)
                    int v[4][3];
                    v[0][0] = ci, v[0][1] = cj, v[0][2] = cl;
                    for (int m = 0; m < 3; ++m) {
                        for (int a = 0; a < 3; ++a) v[m + 1][a] = v[m][a];
                        v[m + 1][perms[p][m]] += 1;
                    }
                    double G[4][3] = {};
                    G[0][perms[p][0]] = -1.0 / h;
                    G[1][perms[p][0]] += 1.0 / h;
                    G[1][perms[p][1]] -= 1.0 / h;
                    G[2][perms[p][1]] += 1.0 / h;
                    G[2][perms[p][2]] -= 1.0 / h;
                    G[3][perms[p][2]] = 1.0 / h;
                    double A[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                    if (!tensor.empty()) {
                        const double* t = &tensor[6 * e];
                        A[0][0] = t[0], A[1][1] = t[1], A[2][2] = t[2];
                        A[0][1] = A[1][0] = t[3];
                        A[0][2] = A[2][0] = t[4];
                        A[1][2] = A[2][1] = t[5];
                    }
                    const double kv = kap.empty() ? 1.0 : kap[e];
                    const double pv = pot.empty() ? 0.0 : pot[e];
                    for (int a = 0; a < 4; ++a) {
                        if (!interior(g, v[a][0], v[a][1], v[a][2])) continue;
                        const long ia = hidx(g, v[a][0], v[a][1], v[a][2]);
                        for (int b = a; b < 4; ++b) {
                            if (!interior(g, v[b][0], v[b][1], v[b][2])) continue;
                            double k = 0.0;
                            for (int x = 0; x < 3; ++x)
                                for (int y = 0; y < 3; ++y) k += G[a][x] * A[x][y] * G[b][y];
                            const double kab = kv * vol * k + pv * vol * (a == b ? 2.0 : 1.0) / 20.0;
                            if (a == b) {
                                s.a[0][ia] += kab;
                            } else {
                                // along the path the edge a -> b points in a direction of O
                                const int t = dir_of(v[b][0] - v[a][0], v[b][1] - v[a][1], v[b][2] - v[a][2]);
                                s.a[t][ia] += kab;
                            }
                        }
                    }
                }
            }
    return s;
}

Stencil15 galerkin_stencil_3d(const Grid& gf, const Stencil15& sf, const Grid& gc) {
    Stencil15 sc;
    for (auto& a : sc.a) a.assign(gc.plane, 0.0);
    // local box of fine offsets [-4, 4]^3 around 2I
    constexpr int R = 4, W = 2 * R + 1;
    std::vector<double> v((size_t)W * W * W);
    auto lid = [&](int dx, int dy, int dz) { return ((dz + R) * W + (dy + R)) * W + (dx + R); };
    // fine entry A(p, p + d) for d in {0, +-O}
    auto entry = [&](int i, int j, int l, int dx, int dy, int dz) -> double {
        if (dx == 0 && dy == 0 && dz == 0) return sf.a[0][hidx(gf, i, j, l)];
        int t = dir_of(dx, dy, dz);
        if (t > 0) return sf.a[t][hidx(gf, i, j, l)];
        t = dir_of(-dx, -dy, -dz);
        if (t > 0 && interior(gf, i + dx, j + dy, l + dz)) return sf.a[t][hidx(gf, i + dx, j + dy, l + dz)];
        return 0.0;
    };
    for (int L = 1; L <= gc.m; ++L)
        for (int J = 1; J <= gc.m; ++J)
            for (int I = 1; I <= gc.m; ++I) {
                std::fill(v.begin(), v.end(), 0.0);
                const int ci = 2 * I, cj = 2 * J, cl = 2 * L;
                // v = A phi_I on the fine nodes around 2I
                for (int sgn = 0; sgn < 15; ++sgn) {
                    int ox = 0, oy = 0, oz = 0;
                    double w = 1.0;
                    if (sgn > 0) {
                        const int t = 1 + (sgn - 1) / 2, neg = (sgn - 1) & 1;
                        ox = neg ? -OX[t] : OX[t], oy = neg ? -OY[t] : OY[t], oz = neg ? -OZ[t] : OZ[t];
                        w = 0.5;
                    }
                    const int pi = ci + ox, pj = cj + oy, pl = cl + oz;
                    if (!interior(gf, pi, pj, pl)) continue;
                    for (int d = 0; d < 15; ++d) {
                        int dx = 0, dy = 0, dz = 0;
                        if (d > 0) {
                            const int t = 1 + (d - 1) / 2, neg = (d - 1) & 1;
                            dx = neg ? -OX[t] : OX[t], dy = neg ? -OY[t] : OY[t], dz = neg ? -OZ[t] : OZ[t];
                        }
                        if (!interior(gf, pi + dx, pj + dy, pl + dz)) continue;
                        // A(q, p) = A(p, q): row q = p + d of A phi_I gains A(q, p) w
                        v[lid(ox + dx, oy + dy, oz + dz)] += w * entry(pi, pj, pl, dx, dy, dz);
                    }
                }
                // A_c(I, I + O_t) = phi_{I + O_t} . v
                for (int t = 0; t < 8; ++t) {
                    const int Ii = I + OX[t], Jj = J + OY[t], Ll = L + OZ[t];
                    if (!interior(gc, Ii, Jj, Ll)) continue;
                    double acc = 0.0;
                    for (int sgn = 0; sgn < 15; ++sgn) {
                        int ox = 0, oy = 0, oz = 0;
                        double w = 1.0;
                        if (sgn > 0) {
                            const int tt = 1 + (sgn - 1) / 2, neg = (sgn - 1) & 1;
                            ox = neg ? -OX[tt] : OX[tt], oy = neg ? -OY[tt] : OY[tt], oz = neg ? -OZ[tt] : OZ[tt];
                            w = 0.5;
                        }
                        const int dx = 2 * OX[t] + ox, dy = 2 * OY[t] + oy, dz = 2 * OZ[t] + oz;
                        if (!interior(gf, ci + dx, cj + dy, cl + dz)) continue;
                        acc += w * v[lid(dx, dy, dz)];
                    }
                    sc.a[t][hidx(gc, I, J, L)] = acc;
                }
            }
    return sc;
}

double gershgorin_3d(const Grid& g, const Stencil15& s) {
    double rho = 0.0;
    for (int l = 1; l <= g.m; ++l)
        for (int j = 1; j <= g.m; ++j)
            for (int i = 1; i <= g.m; ++i) {
                const long id = hidx(g, i, j, l);
                double r = std::fabs(s.a[0][id]);
                for (int t = 1; t < 8; ++t) {
                    r += std::fabs(s.a[t][id]);
                    const int pi = i - OX[t], pj = j - OY[t], pl = l - OZ[t];
                    if (interior(g, pi, pj, pl)) r += std::fabs(s.a[t][hidx(g, pi, pj, pl)]);
                }
                rho = std::max(rho, r / s.a[0][id]);
            }
    return rho;
}

void dense_from_stencil_3d(const Grid& g, const Stencil15& s, std::vector<double>& A) {
    const int m = g.m;
    const long N = (long)m * m * m;
    A.assign((size_t)N * N, 0.0);
    auto cid = [&](int i, int j, int l) { return ((long)(l - 1) * m + (j - 1)) * m + (i - 1); };
    for (int l = 1; l <= m; ++l)
        for (int j = 1; j <= m; ++j)
            for (int i = 1; i <= m; ++i) {
                const long r = cid(i, j, l), id = hidx(g, i, j, l);
                A[r * N + r] = s.a[0][id];
                for (int t = 1; t < 8; ++t) {
                    const int qi = i + OX[t], qj = j + OY[t], ql = l + OZ[t];
                    if (!interior(g, qi, qj, ql)) continue;
                    const long q = cid(qi, qj, ql);
                    A[r * N + q] = A[q * N + r] = s.a[t][id];
                }
            }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
namespace {

constexpr int GX = 64, GY = 4;
inline dim3 grid3g(int m, int nrhs) { return dim3((m + GX - 1) / GX, (m + GY - 1) / GY, m * nrhs); }

struct P3 {
    long id;
    int r;
    bool ok;
};
__device__ inline P3 p3(const Grid& g) {
    P3 p;
    const int i = blockIdx.x * GX + threadIdx.x + 1;
    const int j = blockIdx.y * GY + threadIdx.y + 1;
    const int l = blockIdx.z % g.m + 1;
    p.r = blockIdx.z / g.m;
    p.ok = i <= g.m && j <= g.m;
    p.id = g.idx(i, j, l);
    return p;
}

__device__ inline long off3(const Grid& g, int t) {
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    return OX[t] + OY[t] * py + OZ[t] * pz;
}

// (A x)(id) of the 15-point operator: s15 holds the 8 planes a0..a7
template <typename T>
__device__ inline T apply15(const Grid& g, const T* __restrict__ s15, const T* __restrict__ x, long id) {
    const long P = g.plane;
    T v = s15[id] * x[id];
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        const long o = off3(g, t);
        v += s15[t * P + id] * x[id + o] + s15[t * P + id - o] * x[id - o];
    }
    return v;
}

// M x of the Kuhn mass matrix: h^3 (0.4 centre, 1/20 axis and body diagonals, 1/30 face diagonals)
__device__ inline double mass15(const Grid& g, const double* __restrict__ x, long id) {
    const double h3 = g.h * g.h * g.h;
    double ax = 0.0, fd = 0.0;
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        const long o = off3(g, t);
        const double s = x[id + o] + x[id - o];
        if (t <= 3 || t == 7) ax += s;
        else fd += s;
    }
    return h3 * (0.4 * x[id] + ax / 20.0 + fd / 30.0);
}

// The 15 coefficients of the operator's row at id, in registers, so that
// kernels looping over several right-hand sides read them once.
template <typename T>
struct Row15 {
    T d, up[7], dn[7];
    __device__ inline void load(const Grid& g, const T* __restrict__ s15, long id) {
        const long P = g.plane;
        d = s15[id];
#pragma unroll
        for (int t = 1; t < 8; ++t) {
            up[t - 1] = s15[t * P + id];
            dn[t - 1] = s15[t * P + id - off3(g, t)];
        }
    }
    template <typename V>
    __device__ inline T apply(const Grid& g, long id, V v) const {
        T a = d * v(id);
#pragma unroll
        for (int t = 1; t < 8; ++t) {
            const long o = off3(g, t);
            a += up[t - 1] * v(id + o) + dn[t - 1] * v(id - o);
        }
        return a;
    }
};

// Kernels over RB right-hand sides per thread: blockIdx.z = (plane, group of RB)
constexpr int RB3 = 4;
inline dim3 grid3rb(int m, int nrhs) { return dim3((m + GX - 1) / GX, (m + GY - 1) / GY, m * ((nrhs + RB3 - 1) / RB3)); }

struct P3b {
    long id;
    int r0;  // first right-hand side of the thread's group
    bool ok;
};
__device__ inline P3b p3b(const Grid& g) {
    P3b p;
    const int i = blockIdx.x * GX + threadIdx.x + 1;
    const int j = blockIdx.y * GY + threadIdx.y + 1;
    const int l = blockIdx.z % g.m + 1;
    p.r0 = (blockIdx.z / g.m) * RB3;
    p.ok = i <= g.m && j <= g.m;
    p.id = g.idx(i, j, l);
    return p;
}

template <typename T>
__global__ __launch_bounds__(GX* GY) void k_smooth3g(Grid g, const T* __restrict__ s15, const T* __restrict__ xc,
                                                     const T* xp, const T* __restrict__ f, T* xn, long stride, T a,
                                                     T b, int zmode, int nrhs) {
    const P3b p = p3b(g);
    if (!p.ok) return;
    Row15<T> row;
    if (zmode & 1) row.d = s15[p.id];
    else row.load(g, s15, p.id);
#pragma unroll
    for (int q = 0; q < RB3; ++q) {
        const int z = p.r0 + q;
        if (z >= nrhs) break;
        const long off = (long)z * stride;
        const T fv = f[off + p.id];
        if (zmode & 1) {
            xn[off + p.id] = b * fv / row.d;
            continue;
        }
        const T* xr = xc + off;
        const T x0 = xr[p.id];
        T v = x0 + b * (fv - row.apply(g, p.id, [&](long k) { return xr[k]; })) / row.d;
        if (a != T(0)) v += a * (x0 - ((zmode & 2) ? T(0) : xp[off + p.id]));
        xn[off + p.id] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(GX* GY) void k_apply3g(Grid g, const T* __restrict__ s15, const T* __restrict__ x,
                                                    T* __restrict__ y, long stride) {
    const P3 p = p3(g);
    if (!p.ok) return;
    const long off = (long)p.r * stride;
    y[off + p.id] = apply15<T>(g, s15, x + off, p.id);
}

// r_c(I) = sum over the 15 fine nodes q of the coarse basis function of I of
// its weight times (f - A x)(q), every (A x)(q) formed on the fly
template <typename T>
__global__ __launch_bounds__(GX* GY) void k_resid_restrict3g(Grid gf, const T* __restrict__ s15,
                                                             const T* __restrict__ x, const T* __restrict__ f,
                                                             Grid gc, T* __restrict__ rc, long sf, long sc) {
    const P3 p = p3(gc);
    if (!p.ok) return;
    const int I = blockIdx.x * GX + threadIdx.x + 1, J = blockIdx.y * GY + threadIdx.y + 1,
              L = blockIdx.z % gc.m + 1;
    const T* xr = x + (long)p.r * sf;
    const T* fr = f + (long)p.r * sf;
    const long c0 = gf.idx(2 * I, 2 * J, 2 * L);
    T acc = fr[c0] - apply15<T>(gf, s15, xr, c0);
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        const long o = off3(gf, t);
        // 2 <= 2I <= n - 2 per axis, so the 15 nodes are interior and their
        // stencils stay inside the grid
        const T r1 = fr[c0 + o] - apply15<T>(gf, s15, xr, c0 + o);
        const T r2 = fr[c0 - o] - apply15<T>(gf, s15, xr, c0 - o);
        acc += T(0.5) * (r1 + r2);
    }
    rc[(long)p.r * sc + gc.idx(I, J, L)] = acc;
}

// r = f - A x (type T), RB right-hand sides per thread
template <typename T>
__global__ __launch_bounds__(GX* GY) void k_resid3g(Grid g, const T* __restrict__ s15, const T* __restrict__ x,
                                                    const T* __restrict__ f, T* __restrict__ r, long stride,
                                                    int nrhs) {
    const P3b p = p3b(g);
    if (!p.ok) return;
    Row15<T> row;
    row.load(g, s15, p.id);
#pragma unroll
    for (int q = 0; q < RB3; ++q) {
        const int z = p.r0 + q;
        if (z >= nrhs) break;
        const long off = (long)z * stride;
        const T* xr = x + off;
        r[off + p.id] = f[off + p.id] - row.apply(g, p.id, [&](long k) { return xr[k]; });
    }
}

// lam M u at id with the arithmetic of the 3D prolongation kernel that forms
// f (axis and body diagonals / 20, face diagonals / 30, summed in its order)
__device__ inline double lam_mass15(const Grid& g, const double* __restrict__ u, long id, double lam) {
    const long py = g.pitch, pz = (long)g.pitch * (g.n + 1);
    const double ax = u[id + 1] + u[id - 1] + u[id + py] + u[id - py] + u[id + pz] + u[id - pz];
    const double fd = u[id + 1 + py] + u[id - 1 - py] + u[id + 1 + pz] + u[id - 1 - pz] + u[id + py + pz] +
                      u[id - py - pz];
    const double bd = u[id + 1 + py + pz] + u[id - 1 - py - pz];
    const double h3 = g.h * g.h * g.h;
    return lam * (h3 * (0.4 * u[id] + (ax + bd) * (1.0 / 20.0) + fd * (1.0 / 30.0)));
}

// MASS: f is not read but formed as lam M u from u itself (u is the start
// of the correction step).
template <bool MASS = false>
__global__ __launch_bounds__(GX* GY) void k_resid_cast3g(Grid g, const double* __restrict__ s15,
                                                         const double* __restrict__ u, const double* __restrict__ f,
                                                         float* __restrict__ r, long stride, int nrhs,
                                                         const double* __restrict__ lam) {
    const P3b p = p3b(g);
    if (!p.ok) return;
    Row15<double> row;
    row.load(g, s15, p.id);
#pragma unroll
    for (int q = 0; q < RB3; ++q) {
        const int z = p.r0 + q;
        if (z >= nrhs) break;
        const long off = (long)z * stride;
        const double* ur = u + off;
        const double fv = MASS ? lam_mass15(g, ur, p.id, lam[z]) : f[off + p.id];
        r[off + p.id] = (float)(fv - row.apply(g, p.id, [&](long k) { return ur[k]; }));
    }
}

// MASS: f formed as lam M u from u (the step's first cycle).
template <bool MASS = false>
__global__ __launch_bounds__(GX* GY) void k_add_resid3g(Grid g, const double* __restrict__ s15,
                                                        const double* __restrict__ u, const float* __restrict__ e,
                                                        const double* __restrict__ f, double* __restrict__ un,
                                                        float* __restrict__ r, long stride, int nrhs,
                                                        const double* __restrict__ lam) {
    const P3b p = p3b(g);
    if (!p.ok) return;
    Row15<double> row;
    row.load(g, s15, p.id);
#pragma unroll
    for (int q = 0; q < RB3; ++q) {
        const int z = p.r0 + q;
        if (z >= nrhs) break;
        const long off = (long)z * stride;
        const double* ur = u + off;
        const float* er = e + off;
        const double fv = MASS ? lam_mass15(g, ur, p.id, lam[z]) : f[off + p.id];
        auto v = [&](long k) { return ur[k] + (double)er[k]; };
        const double x0 = v(p.id);
        const double Ax = row.apply(g, p.id, v);
        un[off + p.id] = x0;
        r[off + p.id] = (float)(fv - Ax);
    }
}

// au = A u, mu = M u and per-workgroup sums of u.Au, u.Mu
// The borders' fine-level vectors and scalars, RB right-hand sides per
// thread: A x, M x and partial sums of x.A x and x.M x per workgroup; with
// ADD, x = u + e (the last FP32 correction added in FP64), written to un.
template <bool ADD>
__global__ __launch_bounds__(GX* GY) void k_border3g(Grid g, const double* __restrict__ s15,
                                                     const double* __restrict__ u, const float* __restrict__ e,
                                                     double* __restrict__ un, double* __restrict__ au,
                                                     double* __restrict__ mu, double* __restrict__ partial,
                                                     long stride, int nrhs) {
    __shared__ double sh[RB3][2][GX * GY / 64];
    const P3b p = p3b(g);
    const int nv = min(RB3, nrhs - p.r0);
    Row15<double> row;
    if (p.ok) row.load(g, s15, p.id);
    double a[RB3], m[RB3];
#pragma unroll
    for (int q = 0; q < RB3; ++q) {
        a[q] = m[q] = 0.0;
        if (p.ok && q < nv) {
            const long off = (long)(p.r0 + q) * stride;
            const double* ur = u + off;
            const float* er = e + off;
            auto v = [&](long k) { return ADD ? ur[k] + (double)er[k] : ur[k]; };
            const double x0 = v(p.id);
            const double Ax = row.apply(g, p.id, v);
            // M x of the Kuhn mass matrix: h^3 (0.4 centre, 1/20 axis and
            // body diagonals, 1/30 face diagonals)
            double ax = 0.0, fd = 0.0;
#pragma unroll
            for (int t = 1; t < 8; ++t) {
                const long o = off3(g, t);
                const double s2 = v(p.id + o) + v(p.id - o);
                if (t <= 3 || t == 7) ax += s2;
                else fd += s2;
            }
            const double Mx = g.h * g.h * g.h * (0.4 * x0 + ax / 20.0 + fd / 30.0);
            if (ADD) un[off + p.id] = x0;
            au[off + p.id] = Ax;
            mu[off + p.id] = Mx;
            a[q] = x0 * Ax;
            m[q] = x0 * Mx;
        }
    }
    const int t = threadIdx.y * GX + threadIdx.x;
#pragma unroll
    for (int q = 0; q < RB3; ++q) {
        double sa = a[q], sm = m[q];
        for (int o = 32; o > 0; o >>= 1) {
            sa += __shfl_down(sa, o, 64);
            sm += __shfl_down(sm, o, 64);
        }
        if ((t & 63) == 0) {
            sh[q][0][t >> 6] = sa;
            sh[q][1][t >> 6] = sm;
        }
    }
    __syncthreads();
    if (t < RB3 && t < nv) {
        double sa = 0.0, sm = 0.0;
        for (int w = 0; w < GX * GY / 64; ++w) {
            sa += sh[t][0][w];
            sm += sh[t][1][w];
        }
        const long nblk = (long)gridDim.x * gridDim.y * g.m;
        const long blk = ((long)(blockIdx.z % g.m) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[2 * ((long)(p.r0 + t) * nblk + blk)] = sa;
        partial[2 * ((long)(p.r0 + t) * nblk + blk) + 1] = sm;
    }
}

}  // namespace

template <typename T>
void launch_smooth3g(const Grid& g, const T* s15, const T* xc, const T* xp, const T* f, T* xn, int nrhs,
                     long stride, Cheb s, int zmode, hipStream_t st) {
    hipLaunchKernelGGL((k_smooth3g<T>), grid3rb(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, xc, xp, f, xn, stride,
                       (T)s.a, (T)s.b, zmode, nrhs);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_apply3g(const Grid& g, const T* s15, const T* x, T* y, int nrhs, long stride, hipStream_t st) {
    hipLaunchKernelGGL((k_apply3g<T>), grid3g(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, x, y, stride);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_resid_restrict3g(const Grid& gf, const T* s15, const T* x, const T* f, const Grid& gc, T* rc, int nrhs,
                             long sf, long sc, hipStream_t st) {
    if (gc.n * 2 != gf.n) throw Error(PASM_E_INVALID, "general 3D restriction: ratio 2");
    hipLaunchKernelGGL((k_resid_restrict3g<T>), grid3g(gc.m, nrhs), dim3(GX, GY), 0, st, gf, s15, x, f, gc, rc, sf,
                       sc);
    PASM_CHECK_LAUNCH();
}

void launch_resid_cast3g(const Grid& g, const double* s15, const double* u, const double* f, float* r, int nrhs,
                         long stride, hipStream_t st, const double* lam) {
    if (lam)
        hipLaunchKernelGGL(k_resid_cast3g<true>, grid3rb(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, u, f, r, stride,
                           nrhs, lam);
    else
        hipLaunchKernelGGL(k_resid_cast3g<false>, grid3rb(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, u, f, r, stride,
                           nrhs, nullptr);
    PASM_CHECK_LAUNCH();
}

void launch_add_resid3g(const Grid& g, const double* s15, const double* u, const float* e, const double* f,
                        double* un, float* r, int nrhs, long stride, hipStream_t st, const double* lam) {
    if (lam)
        hipLaunchKernelGGL(k_add_resid3g<true>, grid3rb(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, u, e, f, un, r,
                           stride, nrhs, lam);
    else
        hipLaunchKernelGGL(k_add_resid3g<false>, grid3rb(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, u, e, f, un, r,
                           stride, nrhs, nullptr);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_resid3g(const Grid& g, const T* s15, const T* x, const T* f, T* r, int nrhs, long stride,
                    hipStream_t st) {
    hipLaunchKernelGGL((k_resid3g<T>), grid3rb(g.m, nrhs), dim3(GX, GY), 0, st, g, s15, x, f, r, stride, nrhs);
    PASM_CHECK_LAUNCH();
}
template void launch_resid3g<double>(const Grid&, const double*, const double*, const double*, double*, int, long,
                                     hipStream_t);
template void launch_resid3g<float>(const Grid&, const float*, const float*, const float*, float*, int, long,
                                    hipStream_t);

int launch_border3g(const Grid& g, const double* s15, const double* u, double* au, double* mu, double* partial,
                    int nrhs, long stride, hipStream_t st, const float* e, double* un) {
    if ((e == nullptr) != (un == nullptr)) throw Error(PASM_E_INVALID, "general 3D borders: correction and output");
    const dim3 grid = grid3rb(g.m, nrhs);
    if (e)
        hipLaunchKernelGGL(k_border3g<true>, grid, dim3(GX, GY), 0, st, g, s15, u, e, un, au, mu, partial, stride,
                           nrhs);
    else
        hipLaunchKernelGGL(k_border3g<false>, grid, dim3(GX, GY), 0, st, g, s15, u, e, un, au, mu, partial, stride,
                           nrhs);
    PASM_CHECK_LAUNCH();
    return (int)(grid.x * grid.y * g.m);
}

template void launch_smooth3g<double>(const Grid&, const double*, const double*, const double*, const double*,
                                      double*, int, long, Cheb, int, hipStream_t);
template void launch_smooth3g<float>(const Grid&, const float*, const float*, const float*, const float*, float*,
                                     int, long, Cheb, int, hipStream_t);
template void launch_apply3g<double>(const Grid&, const double*, const double*, double*, int, long, hipStream_t);
template void launch_apply3g<float>(const Grid&, const float*, const float*, float*, int, long, hipStream_t);
template void launch_resid_restrict3g<double>(const Grid&, const double*, const double*, const double*, const Grid&,
                                              double*, int, long, long, hipStream_t);
template void launch_resid_restrict3g<float>(const Grid&, const float*, const float*, const float*, const Grid&,
                                             float*, int, long, long, hipStream_t);

}  // namespace pasm

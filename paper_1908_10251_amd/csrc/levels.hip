// Construction of the level operators and other set-up work.
//
// The finest level is assembled element by element on the "/" mesh
// (Section 2: a(u, v) = int kappa grad u . grad v + int V u v, with kappa
// and V constant per element; the potential term of the paper's second
// example, taken at the element centroid).  Coarser levels are Galerkin
// products P^T A P with P the nodal interpolation between nested meshes
// (Section 3), which is what the augmented pencil needs (its blocks are
// restrictions of the fine forms to V_H).
#include <cmath>

#include "common.h"

namespace pasm {

// Edge weights of the 2D stiffness from per-element kappa on a level with n
// cells (element order: cell x-fastest, lower then upper triangle).  The edge
// (i,j)-(i+1,j) is a leg of the lower triangle of cell (i,j) and of the upper
// triangle of cell (i,j-1); the edge (i,j)-(i,j+1) of the upper triangle of
// cell (i,j) and of the lower triangle of cell (i-1,j); each leg couples with
// kappa_T / 2.
void edge_weights_2d(const Grid& g, const std::vector<double>& kap, std::vector<double>& wx,
                     std::vector<double>& wy) {
    const int n = g.n;
    wx.assign(g.plane, 0.0);
    wy.assign(g.plane, 0.0);
    const bool one = kap.empty();
    auto kl = [&](int ci, int cj) { return one ? 1.0 : kap[2 * ((size_t)cj * n + ci)]; };
    auto ku = [&](int ci, int cj) { return one ? 1.0 : kap[2 * ((size_t)cj * n + ci) + 1]; };
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            if (i < n) {
                double w = 0.0;
                if (j < n) w += kl(i, j);
                if (j > 0) w += ku(i, j - 1);
                wx[g.idx(i, j)] = 0.5 * w;
            }
            if (j < n) {
                double w = 0.0;
                if (i < n) w += ku(i, j);
                if (i > 0) w += kl(i - 1, j);
                wy[g.idx(i, j)] = 0.5 * w;
            }
        }
}

// Galerkin coarsening of a per-element coefficient (2D): the coarse triangle's
// value is the mean over its four children, which makes the rediscretised
// coarse stiffness equal to P^T A P (coarse basis gradients are constant on
// the coarse triangle).  Children of the lower coarse triangle of cell (I,J):
// lower of fine cell (2I,2J), both of (2I+1,2J), lower of (2I+1,2J+1); of the
// upper: upper of (2I,2J), both of (2I,2J+1), upper of (2I+1,2J+1).
std::vector<double> coarsen_kappa_2d(const std::vector<double>& kf, int nf) {
    const int nc = nf / 2;
    std::vector<double> kc(2 * (size_t)nc * nc);
    auto K = [&](int ci, int cj, int p) { return kf[2 * ((size_t)cj * nf + ci) + p]; };
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I) {
            const int i = 2 * I, j = 2 * J;
            kc[2 * ((size_t)J * nc + I)] = 0.25 * (K(i, j, 0) + K(i + 1, j, 0) + K(i + 1, j, 1) + K(i + 1, j + 1, 0));
            kc[2 * ((size_t)J * nc + I) + 1] =
                0.25 * (K(i, j, 1) + K(i, j + 1, 0) + K(i, j + 1, 1) + K(i + 1, j + 1, 1));
        }
    return kc;
}

// Finest-level general stencil: stiffness from kappa (empty: 1) plus the
// potential's mass-type term.  On a triangle T with area |T| = h^2/2 the
// element mass matrix is |T|(1 + delta_ij)/12, so V_T contributes V_T h^2/12
// to the diagonal of each of its vertices and V_T h^2/24 to each of its three
// vertex pairs (stored with the sign convention w = -a).  Vertex pairs: the
// east edge at (i,j) lies in the lower triangle of cell (i,j) and the upper
// of cell (i,j-1); the north edge in the upper of (i,j) and the lower of
// (i-1,j); the north-east diagonal in both triangles of cell (i,j).  The six
// triangles around node (i,j): both of cells (i,j) and (i-1,j-1), the lower
// of (i-1,j) and the upper of (i,j-1).
Stencil7 fine_stencil_2d(const Grid& g, const std::vector<double>& kap, const std::vector<double>& pot) {
    const int n = g.n;
    Stencil7 s;
    edge_weights_2d(g, kap, s.wx, s.wy);
    s.d.assign(g.plane, 0.0);
    s.wne.assign(g.plane, 0.0);
    const double h2 = g.h * g.h;
    auto V = [&](int ci, int cj, int p) -> double {
        if (ci < 0 || cj < 0 || ci >= n || cj >= n) return 0.0;
        return pot.empty() ? 0.0 : pot[2 * ((size_t)cj * n + ci) + p];
    };
    // diagonal first, from the stiffness weights alone (zero row sums)
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            const long id = g.idx(i, j);
            double dk = s.wx[id] + s.wy[id];
            if (i > 0) dk += s.wx[g.idx(i - 1, j)];
            if (j > 0) dk += s.wy[g.idx(i, j - 1)];
            const double vsum = V(i, j, 0) + V(i, j, 1) + V(i - 1, j - 1, 0) + V(i - 1, j - 1, 1) + V(i - 1, j, 0) +
                                V(i, j - 1, 1);
            s.d[id] = dk + vsum * h2 / 12.0;
        }
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            const long id = g.idx(i, j);
            if (i < n) s.wx[id] -= (V(i, j, 0) + V(i, j - 1, 1)) * h2 / 24.0;
            if (j < n) s.wy[id] -= (V(i, j, 1) + V(i - 1, j, 0)) * h2 / 24.0;
            if (i < n && j < n) s.wne[id] = -(V(i, j, 0) + V(i, j, 1)) * h2 / 24.0;
        }
    return s;
}

namespace {

// matrix entry a(x, x + o) of a general stencil at interior node x = (i, j)
double entry(const Grid& g, const Stencil7& s, int i, int j, int oi, int oj) {
    if (oi == 0 && oj == 0) return s.d[g.idx(i, j)];
    if (oi == 1 && oj == 0) return -s.wx[g.idx(i, j)];
    if (oi == -1 && oj == 0) return -s.wx[g.idx(i - 1, j)];
    if (oi == 0 && oj == 1) return -s.wy[g.idx(i, j)];
    if (oi == 0 && oj == -1) return -s.wy[g.idx(i, j - 1)];
    if (oi == 1 && oj == 1) return -s.wne[g.idx(i, j)];
    if (oi == -1 && oj == -1) return -s.wne[g.idx(i - 1, j - 1)];
    return 0.0;
}

constexpr int kOff[7][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};

// coarse nodes whose interpolation reaches fine node (i, j), with weights:
// (I, J) and (I + a, J + b) for a = i & 1, b = j & 1 (one node, weight 1,
// when both are even)
int parents(int i, int j, int P[2][2], double w[2]) {
    const int a = i & 1, b = j & 1, I = i >> 1, J = j >> 1;
    if (!a && !b) {
        P[0][0] = I;
        P[0][1] = J;
        w[0] = 1.0;
        return 1;
    }
    P[0][0] = I;
    P[0][1] = J;
    P[1][0] = I + a;
    P[1][1] = J + b;
    w[0] = w[1] = 0.5;
    return 2;
}

}  // namespace

// P^T A P on the next coarser grid, accumulated over a 5 x 5 window of coarse
// offsets; entries outside the 7-point pattern cancel (the coarse basis
// functions of non-neighbouring coarse nodes have disjoint supports) and are
// checked to vanish to rounding.
Stencil7 galerkin_stencil_2d(const Grid& gf, const Stencil7& sf, const Grid& gc) {
    const int m = gc.m;
    const size_t nn = (size_t)m * m;
    std::vector<double> acc(nn * 25, 0.0);
    auto slot = [&](int I, int J, int di, int dj) -> double& {
        return acc[(((size_t)(J - 1) * m + (I - 1)) * 5 + (dj + 2)) * 5 + (di + 2)];
    };
    for (int j = 1; j <= gf.m; ++j)
        for (int i = 1; i <= gf.m; ++i) {
            int Pf[2][2];
            double wf[2];
            const int nf = parents(i, j, Pf, wf);
            for (int o = 0; o < 7; ++o) {
                const int i2 = i + kOff[o][0], j2 = j + kOff[o][1];
                if (i2 < 1 || j2 < 1 || i2 > gf.m || j2 > gf.m) continue;
                const double a = entry(gf, sf, i, j, kOff[o][0], kOff[o][1]);
                if (a == 0.0) continue;
                int Pg[2][2];
                double wg[2];
                const int ng = parents(i2, j2, Pg, wg);
                for (int p = 0; p < nf; ++p) {
                    const int I = Pf[p][0], J = Pf[p][1];
                    if (I < 1 || J < 1 || I > m || J > m) continue;
                    for (int q = 0; q < ng; ++q) {
                        const int I2 = Pg[q][0], J2 = Pg[q][1];
                        if (I2 < 1 || J2 < 1 || I2 > m || J2 > m) continue;
                        const int di = I2 - I, dj = J2 - J;
                        if (di < -2 || di > 2 || dj < -2 || dj > 2)
                            throw Error(PASM_E_DEVICE, "Galerkin coarsening: coupling beyond the 5x5 window");
                        slot(I, J, di, dj) += wf[p] * a * wg[q];
                    }
                }
            }
        }
    Stencil7 sc;
    sc.d.assign(gc.plane, 0.0);
    sc.wx.assign(gc.plane, 0.0);
    sc.wy.assign(gc.plane, 0.0);
    sc.wne.assign(gc.plane, 0.0);
    double dmax = 0.0;
    for (int J = 1; J <= m; ++J)
        for (int I = 1; I <= m; ++I) dmax = std::max(dmax, std::fabs(slot(I, J, 0, 0)));
    for (int J = 1; J <= m; ++J)
        for (int I = 1; I <= m; ++I) {
            for (int dj = -2; dj <= 2; ++dj)
                for (int di = -2; di <= 2; ++di) {
                    bool in7 = false;
                    for (int o = 0; o < 7; ++o) in7 |= (kOff[o][0] == di && kOff[o][1] == dj);
                    if (!in7 && std::fabs(slot(I, J, di, dj)) > 1e-12 * dmax)
                        throw Error(PASM_E_DEVICE, "Galerkin coarsening left the 7-point pattern");
                }
            const long id = gc.idx(I, J);
            sc.d[id] = slot(I, J, 0, 0);
            if (I < m) sc.wx[id] = -slot(I, J, 1, 0);
            if (J < m) sc.wy[id] = -slot(I, J, 0, 1);
            if (I < m && J < m) sc.wne[id] = -slot(I, J, 1, 1);
        }
    return sc;
}

// Gershgorin bound of D^{-1} A: max over interior rows of sum |a_ij| / a_ii.
double gershgorin_2d(const Grid& g, const Stencil7& s) {
    double r = 0.0;
    for (int j = 1; j <= g.m; ++j)
        for (int i = 1; i <= g.m; ++i) {
            double t = 0.0;
            for (int o = 0; o < 7; ++o) {
                const int i2 = i + kOff[o][0], j2 = j + kOff[o][1];
                if (i2 < 1 || j2 < 1 || i2 > g.m || j2 > g.m) continue;
                t += std::fabs(entry(g, s, i, j, kOff[o][0], kOff[o][1]));
            }
            r = std::max(r, t / s.d[g.idx(i, j)]);
        }
    return r;
}

// Dense A (column-major N x N, N = m^2, interior nodes x-fastest) of a level.
void dense_from_stencil_2d(const Grid& g, const Stencil7& s, std::vector<double>& A) {
    const int m = g.m;
    const long N = (long)m * m;
    A.assign((size_t)N * N, 0.0);
    for (int j = 1; j <= m; ++j)
        for (int i = 1; i <= m; ++i) {
            const long r = (long)(j - 1) * m + (i - 1);
            for (int o = 0; o < 7; ++o) {
                const int i2 = i + kOff[o][0], j2 = j + kOff[o][1];
                if (i2 < 1 || j2 < 1 || i2 > m || j2 > m) continue;
                const long q = (long)(j2 - 1) * m + (i2 - 1);
                A[(size_t)q * N + r] = entry(g, s, i, j, kOff[o][0], kOff[o][1]);
            }
        }
}

// ---------------------------------------------------------------------------
// Smoother coefficients
// ---------------------------------------------------------------------------
// Chebyshev semi-iteration of degree s on D^{-1}A over [rho/alpha, rho], as
// the three-term recurrence x_{j+1} = x_j + a_j (x_j - x_{j-1}) + b_j D^{-1} r_j:
// theta = (b+a)/2, delta = (b-a)/2, sigma = theta/delta, rho_0 = 1/sigma,
// b_0 = 1/theta, a_0 = 0; rho_j = 1/(2 sigma - rho_{j-1}),
// a_j = rho_j rho_{j-1}, b_j = 2 rho_j / delta.
std::vector<Cheb> cheb_steps(double rho, double alpha, int s) {
    std::vector<Cheb> v;
    const double lo = rho / alpha, hi = rho;
    const double th = 0.5 * (hi + lo), de = 0.5 * (hi - lo), sg = th / de;
    double rj = 1.0 / sg;
    for (int j = 0; j < s; ++j) {
        if (j == 0) v.push_back({0.0, 1.0 / th});
        else {
            const double rn = 1.0 / (2.0 * sg - rj);
            v.push_back({rn * rj, 2.0 * rn / de});
            rj = rn;
        }
    }
    return v;
}

std::vector<Cheb> jacobi_steps(double omega, int s) { return std::vector<Cheb>(s, Cheb{0.0, omega}); }

// ---------------------------------------------------------------------------
// Small set-up and bookkeeping kernels
// ---------------------------------------------------------------------------
namespace {

__global__ void k_transpose(const double* __restrict__ a, double* __restrict__ b, int n) {
    const int i = blockIdx.x * 16 + threadIdx.x, j = blockIdx.y * 16 + threadIdx.y;
    if (i < n && j < n) b[(long)i * n + j] = a[(long)j * n + i];
}
__global__ void k_scale_cols(const double* __restrict__ q, const double* __restrict__ th, double* __restrict__ o,
                             int n) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i < n) o[(long)j * n + i] = q[(long)j * n + i] / th[j];
}
__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        b[t] = (float)a[t];
}
__global__ void k_unit_coefs(double* __restrict__ y, int N, int kpm) {
    const int j = blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
    if (j < N) y[(long)r * N + j] = (j == r % kpm) ? 1.0 : 0.0;
}
__global__ void k_copy_d(const double* __restrict__ a, double* __restrict__ b, int n) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) b[t] = a[t];
}

}  // namespace

void launch_transpose(const double* a, double* b, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose, dim3((n + 15) / 16, (n + 15) / 16), dim3(16, 16), 0, st, a, b, n);
    PASM_CHECK_LAUNCH();
}
void launch_scale_cols(const double* q, const double* th, double* o, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_cols, dim3((n + 255) / 256, n), dim3(256), 0, st, q, th, o, n);
    PASM_CHECK_LAUNCH();
}
void launch_d2f(const double* a, float* b, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_d2f, dim3(1024), dim3(256), 0, st, a, b, n);
    PASM_CHECK_LAUNCH();
}
void launch_unit_coefs(double* y, int N, int nrhs, int kpm, hipStream_t st) {
    hipLaunchKernelGGL(k_unit_coefs, dim3((N + 255) / 256, nrhs), dim3(256), 0, st, y, N, kpm);
    PASM_CHECK_LAUNCH();
}
void launch_copy(const double* a, double* b, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_d, dim3((n + 255) / 256), dim3(256), 0, st, a, b, n);
    PASM_CHECK_LAUNCH();
}

}  // namespace pasm

// Internal definitions shared by the HIP sources of the library.
//
// Storage of a level (one nested mesh of the hierarchy of Section 3): every
// right-hand side is one block of `plane` elements holding ALL nodes of the
// level, boundary included; boundary entries are kept at zero (homogeneous
// Dirichlet data), so stencils need no boundary branches.  Node (i, j[, l]) of
// a level with n cells per side lives at
//     ((l * (n + 1) + j) * pitch) + ORIGIN + i
// ORIGIN = 15 puts node i = 1 (the first interior node of a row) on a 128-byte
// boundary when pitch is a multiple of 16, so a wavefront reading 64
// consecutive interior nodes of a row touches whole cache lines.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/pasm.h"

namespace pasm {

constexpr int ORIGIN = 15;

struct Grid {
    int dim = 2;
    int n = 0;        // cells per side
    int m = 0;        // interior nodes per side (n - 1)
    int pitch = 0;    // elements per padded row
    long plane = 0;   // elements per right-hand side block
    double h = 0.0;

    __host__ __device__ inline long idx(int i, int j) const {
        return (long)j * pitch + ORIGIN + i;
    }
    __host__ __device__ inline long idx(int i, int j, int l) const {
        return ((long)l * (n + 1) + j) * pitch + ORIGIN + i;
    }
    long interior() const {
        long r = 1;
        for (int a = 0; a < dim; ++a) r *= m;
        return r;
    }
};

Grid make_grid(int dim, int n);

// Operator coefficients of one level, in one of three forms:
//  constant  (wx == nullptr): every edge has weight w0, A x = sum over edges
//            (x, y) of w0 (x_x - x_y): the 5-point (2D) or 7-point (3D)
//            stencil;
//  edge      (wx set, d == nullptr): w[a] holds, at node x, the weight of the
//            edge (x, x + e_a) (2D: a = 0 east, 1 north); the diagonal is the
//            sum of the four edge weights at the node (zero row sums);
//  general   (d set, 2D): (A x)_x = d_x x_x - sum over the six neighbours y of
//            the "/" mesh of w_xy x_y, with w_xy in wx (east), wy (north) and
//            wne (north-east) at the lower-left node of the edge.  This holds
//            the stiffness plus a potential's mass-type term, and their
//            Galerkin coarsenings.
// A batch of several problems of the same grid stores one coefficient plane
// per member, ms elements apart; right-hand side z belongs to member z / kpm.
// bsc (optional, per member) scales the b coefficients of the smoother steps.
template <typename T>
struct Coef {
    const T* wx = nullptr;
    const T* wy = nullptr;
    const T* wz = nullptr;
    const T* d = nullptr;
    const T* wne = nullptr;
    const T* s15 = nullptr;  // 3D general 15-point operator: 8 planes (diagonal, then the entries towards +O_t)
    T w0 = T(1);
    long ms = 0;
    int kpm = 1;
    const T* bsc = nullptr;
};

// 0: constant, 1: edge weights, 2: general 7-point (2D), 3: general 15-point (3D)
template <typename T>
inline int coef_kind(const Coef<T>& c) {
    return c.s15 ? 3 : (c.d ? 2 : (c.wx ? 1 : 0));
}

#define PASM_HIP(call)                                                              \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            throw pasm::Error(PASM_E_DEVICE, std::string(#call) + ": " +            \
                                                 hipGetErrorString(e_));            \
    } while (0)

#define PASM_CHECK_LAUNCH() PASM_HIP(hipGetLastError())

struct Error {
    pasm_status status;
    std::string msg;
    Error(pasm_status s, std::string m) : status(s), msg(std::move(m)) {}
};

// ----------------------------------------------------------------------------
// Launchers (2D stencils, transfers), implemented in stencil2d.hip.
// All take `nrhs` right-hand sides stored `stride` elements apart.
// ----------------------------------------------------------------------------
struct Cheb {
    double a;   // weight of (x_k - x_{k-1})
    double b;   // weight of D^{-1}(f - A x_k)
};

// zmode bit 0: x_k is zero (not read); bit 1: x_{k-1} is zero (not read)
template <typename T>
void launch_smooth(const Grid& g, const Coef<T>& c, const T* xc, const T* xp, const T* f, T* xn,
                   int nrhs, long stride, Cheb s, int zmode, hipStream_t st);

// Coefficients of the steps of one smoothing phase (fused kernel).
struct SmoothSteps {
    double a[8];
    double b[8];
    int s;
};

bool fused_supported(const Grid& g, int steps);

// Tile heights of the fused smoothing phase: a workgroup covers 4 * rows LDS
// rows of 64 columns.  rows must be one of these.
constexpr int kFusedRows[3] = {2, 4, 8};
// LDS bytes a fused launch of this shape needs (must stay within 64 KiB).
size_t fused_lds_bytes(int kind, size_t elem, int rows);

// All steps of a phase in one launch (2D, s <= 4): out = x_s from x_0 (or 0).
// Returns false when the shape is not covered (caller falls back to steps).
template <typename T>
bool launch_smooth_fused(const Grid& g, const Coef<T>& c, const T* x0, const T* f, T* out, int nrhs,
                         long stride, const SmoothSteps& ss, bool x_zero, hipStream_t st, int rows = 8);

// Marching smoothing phases (2D, constant coefficients, 1..4 steps).
// pre:  out = x_s (from x0, or from 0), rc = P^T (f - A x_s) on the coarser grid gc
// post: out = x_s starting from x + P ec
// rows: rows of the band a wavefront marches down (even); 0 picks it so that
// the whole grid is resident at once where possible.
bool march_supported(const Grid& g, bool const_coef, int steps);
// Conjugate-gradient smoothing (the paper's multigrid step): steps of plain
// CG on A x = f for nrhs right-hand sides of one level, x updated in place
// (x_zero: from x = 0, x overwritten).  Work vectors r, pa, pb, q of the
// cycle's type (one padded plane per right-hand side each), partial sums
// (cg_partials(g) per right-hand side), and three scalars per right-hand side.
struct CgWork {
    void* r;
    void* pa;
    void* pb;
    void* q;
    double* partial;
    double* rr;
    double* alpha;
    double* beta;
};
long cg_partials(const Grid& g);
template <typename T>
void cg_smooth(const Grid& g, const Coef<T>& c, T* x, const T* f, int nrhs, int steps, bool x_zero, const CgWork& w,
               hipStream_t st);

// Levels with edge weights (per-element kappa) or the general 7-point
// operator (kappa and a potential), FP32, single problems or every member of
// a batch level: the marching pre-smoothing with residual restriction and
// post-smoothing with prolongation.
bool march_ew_supported(const Grid& g, int steps);
bool march_coef_supported(const Grid& g, const Coef<float>& c, int steps);
void launch_march_pre_ew(const Grid& g, const Coef<float>& c, const float* x0, const float* f, float* out,
                         const Grid& gc, float* rc, int nrhs, const SmoothSteps& ss, bool x_zero, hipStream_t st);
void launch_march_post_ew(const Grid& g, const Coef<float>& c, const float* x, const float* f, float* out,
                          const Grid& gc, const float* ec, int nrhs, const SmoothSteps& ss, hipStream_t st);
struct MarchShape {
    int strips, segs, mseg, work, blocks;
    int nrhs;
};
template <typename T>
void launch_march_pre(const Grid& g, T w0, const T* x0, const T* f, T* out, const Grid& gc, T* rc, int nrhs,
                      const SmoothSteps& ss, bool x_zero, hipStream_t st, int rows = 0);
template <typename T>
void launch_march_post(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                       const SmoothSteps& ss, hipStream_t st, int rows = 0);
// launch_march_post, then from its output u also b_c = P^T A u and
// c_c = P^T M u on gc (as launch_border_restrict) and the pairs (u.Au, u.Mu)
// of every wavefront's own nodes in partial; returns the pairs per
// right-hand side (for launch_reduce_pairs).
int launch_march_post_border(const Grid& g, double w0, const double* x, const double* f, double* out, const Grid& gc,
                             const double* ec, double* bc, double* cc, double* partial, int nrhs,
                             const SmoothSteps& ss, hipStream_t st, int rows = 0);
// The post-smoothing of one V-cycle and the pre-smoothing of the next in one
// pass (FP64): out = the pre-smoothed x of the next cycle, starting from
// x + P ec, and rc = P^T (f - A out) on gc; post.s + pre.s <= 8.  Equal to
// launch_march_post followed by launch_march_pre on its output.
bool march_pair_supported(const Grid& g, bool const_coef, int post, int pre);
void launch_march_post_pre(const Grid& g, double w0, const double* x, const double* f, double* out, const Grid& gc,
                           const double* ec, double* rc, int nrhs, const SmoothSteps& post, const SmoothSteps& pre,
                           hipStream_t st);
// The first pre-smoothing of a correction step (FP64) with the previous
// step's prolongation in the pass: x_0 = P q + beta u (u the old field, q the
// coarse-space field on gq, P1 interpolation on the coarse "/" triangles,
// power-of-two ratio), f = lam M x_0 written to fout, out = x_s and
// rc = P^T (f - A out) on gc.  Equal to launch_prolong_mass followed by
// launch_march_pre on its output.
bool march_prolong_supported(const Grid& g, bool const_coef, int pre, const Grid& gq);
void launch_march_pre_prolong(const Grid& g, double w0, const double* u, double* fout, double* out, const Grid& gc,
                              double* rc, const Grid& gq, const double* q, const double* beta, const double* lam,
                              int nrhs, const SmoothSteps& pre, hipStream_t st);

// Marching smoothing phases (3D, constant coefficients, 128 cells per side,
// 1 or 2 steps): out = x_s from x0 (or from 0), or (post) from x + P ec.
bool march3_supported(const Grid& g, bool const_coef, int steps);
template <typename T>
void launch_march3_smooth(const Grid& g, T w0, const T* x0, const T* f, T* out, int nrhs, const SmoothSteps& ss,
                          bool x_zero, hipStream_t st);
template <typename T>
void launch_march3_post(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                        const SmoothSteps& ss, hipStream_t st);

template <typename T>
void launch_resid_restrict(const Grid& gf, const Coef<T>& c, const T* x, const T* f, const Grid& gc,
                           T* rc, int nrhs, long sf, long sc, hipStream_t st);

// Exact solve with a constant-coefficient 2D coarse operator w0 (5-point) by
// its sine transform (n <= 64 cells per side): tables built on the host once.
bool dst_solve_supported(const Grid& g);
void dst_solve_tables(const Grid& g, double w0, std::vector<double>& S, std::vector<double>& inv);
template <typename T>
void launch_dst_solve(const Grid& g, const double* S, const double* inv, const T* f, long sf, T* x, long sx,
                      int nrhs, hipStream_t st);

// un = u + e and r = f - A un (to FP32) in one pass (3D, or 2D with constant
// coefficients or edge weights); un must not alias u.  With lam (2D edge
// weights, mass_rhs_fusable): f is not read but formed as lam M u.
bool add_resid_supported(const Grid& g, const Coef<double>& c);
void launch_add_resid(const Grid& g, const Coef<double>& c, const double* u, const float* e, const double* f,
                      double* un, float* r, int nrhs, long stride, hipStream_t st, const double* lam = nullptr);
// The same without storing un = u + e (2D edge weights): u and e stay, and
// the border pass after the next cycle forms (u + e) + e' itself.
void launch_resid_of_sum(const Grid& g, const Coef<double>& c, const double* u, const float* e, const double* f,
                         float* r, int nrhs, long stride, hipStream_t st, const double* lam = nullptr);
// the residual kernels can form f = lam M u from u themselves (2D edge
// weights of a single problem)
bool mass_rhs_fusable(const Grid& g, const Coef<double>& c);
// Batch members (2D, edge weights or the general 7-point operator, each
// right-hand side with its member's coefficient planes), f = lam M u formed
// from u: r = lam M u - A u; and un = u + e with r = lam M u - A un in one
// pass (un must not alias u).  lam holds one value per right-hand side.
void launch_resid_mass_members(const Grid& g, const Coef<double>& c, const double* u, const double* lam, float* r,
                               int nrhs, long stride, hipStream_t st);
void launch_add_resid_members(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un,
                              float* r, int nrhs, long stride, const double* lam, hipStream_t st);
// un = u + e and r = f - A un (to FP32) in one pass (3D); un must not alias u.
// With lam (constant coefficients): f is not read but formed as lam M u.
void launch_add_resid3(const Grid& g, const Coef<double>& c, const double* u, const float* e, const double* f,
                       double* un, float* r, int nrhs, long stride, hipStream_t st, const double* lam = nullptr);
// r32 = f - A u (3D); with lam (constant coefficients) f = lam M u is formed
void launch_resid_cast3(const Grid& g, const Coef<double>& c, const double* u, const double* f, float* r,
                        int nrhs, long stride, hipStream_t st, const double* lam = nullptr);
// xn = P xc + beta[r] xo and the next step's first residual
// r32 = lam[r] M xn - A xn (3D, constant coefficients, ratio 2; xn != xo)
void launch_prolong_resid3(const Grid& gc, const double* xc, const Grid& gf, const Coef<double>& c, const double* xo,
                           double* xn, float* r, int nrhs, long sc, long sf, const double* beta, const double* lam,
                           hipStream_t st);
void launch_prolong_mass3(const Grid& gc, const double* xc, const Grid& gf, const double* xo, double* xn,
                          double* f, int nrhs, long sc, long sf, const double* beta, const double* lam,
                          hipStream_t st);
// xn = P xc + beta[r] xo and f = lam[r] M xn (double; xn != xo; f may be
// null).  With r32 (2D, edge weights wx, wy of the fine level, f null):
// r32 = lam[r] M xn - A xn in FP32 instead of f.
void launch_prolong_mass(const Grid& gc, const double* xc, const Grid& gf, const double* xo, double* xn,
                         double* f, int nrhs, long sc, long sf, const double* beta, const double* lam,
                         hipStream_t st, const double* wx = nullptr, const double* wy = nullptr,
                         float* r32 = nullptr);
// x_f = alpha * (P x_c) + beta[r] * x_f  (beta == nullptr: x_f = P x_c;
// add = true: x_f += P x_c)
template <typename T>
void launch_prolong(const Grid& gc, const T* xc, const Grid& gf, T* xf, int nrhs, long sc, long sf,
                    bool add, const double* beta, hipStream_t st);

// Three 2D restrictions in a row (g3 -> g2 -> g1 -> g0, FP64) in one pass:
// equal to three launch_restrict calls; the intermediate levels are not written.
void launch_restrict_chain3(const Grid& g3, const double* x3, const Grid& g2, const Grid& g1, const Grid& g0,
                            double* x0, int nrhs, long s3, long s0, hipStream_t st);
template <typename T>
void launch_restrict(const Grid& gf, const T* xf, const Grid& gc, T* xc, int nrhs, long sf, long sc,
                     hipStream_t st);

template <typename T>
void launch_apply_A(const Grid& g, const Coef<T>& c, const T* x, T* y, int nrhs, long stride,
                    hipStream_t st);

// f = lambda[r] * M_h u  (finest level, FP64)
void launch_mass_rhs(const Grid& g, const double* u, const double* lam, double* f, int nrhs,
                     long stride, hipStream_t st);
// y = M_h x
void launch_apply_M(const Grid& g, const double* x, double* y, int nrhs, long stride, hipStream_t st);

// r32 = (f - A u) in FP64, rounded to FP32; with lam (mass_rhs_fusable), f
// is not read but formed as lam M u
void launch_resid_cast(const Grid& g, const Coef<double>& c, const double* u, const double* f,
                       float* r, int nrhs, long stride, hipStream_t st, const double* lam = nullptr);
// r = f - A u in FP64, stored as TO (2D)
template <typename TO>
void launch_resid_to(const Grid& g, const Coef<double>& c, const double* u, const double* f, TO* r, int nrhs,
                     long stride, hipStream_t st);

// u += e (whole blocks, boundary entries stay zero)
void launch_add_correction(const float* e, double* u, long n, hipStream_t st);
void launch_add_correction(const double* e, double* u, long n, hipStream_t st);

// Border sweep: au = A u, mu = M u, partial[r][blk][2] = block sums of
// (u . au, u . mu).  Returns the number of blocks per right-hand side.
// 3D: b_c = P^T A u, c_c = P^T M u on the next coarser grid and the pairs
// (u.Au, u.Mu) per workgroup in partial (through an LDS tile); returns the
// pairs per right-hand side.  With e and un (constant coefficients): of
// u + e (the last FP32 correction, added in FP64), written to un.
int launch_border_restrict3(const Grid& g, const Coef<double>& c, const double* u, const Grid& gc, double* bc,
                            double* cc, double* partial, int nrhs, long stride, long sc, hipStream_t st,
                            const float* e = nullptr, double* un = nullptr);
int launch_border(const Grid& g, const Coef<double>& c, const double* u, double* au, double* mu,
                  double* partial, int nrhs, long stride, hipStream_t st);

// 2D borders fused with the restriction to the next coarser grid gc:
// bc = P^T A u, cc = P^T M u on gc, partial as for launch_border (blocks over
// the coarse grid).  Returns the number of blocks per right-hand side.
int launch_border_restrict(const Grid& g, const Coef<double>& c, const double* u, const Grid& gc, double* bc,
                           double* cc, double* partial, int nrhs, long stride, long sc, hipStream_t st);
// The same after the last V-cycle's correction: borders of un = u + e (e the
// FP32 correction, added in FP64), un written (2D, constant or edge weights).
int launch_border_restrict_add(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un,
                               const Grid& gc, double* bc, double* cc, double* partial, int nrhs, long stride, long sc,
                               hipStream_t st, const float* e0 = nullptr);

// The borders after the last correction as a row-marching pass (rows2d.hip),
// used by launch_border_restrict_add where rows_supported holds (2D edge
// weights of a single problem); max_blocks is the capacity of partial in
// pairs per right-hand side.
bool rows_supported(const Grid& g, const Coef<double>& c);
int launch_border_rows(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un,
                       const Grid& gc, double* bc, double* cc, double* partial, int nrhs, long stride, long sc,
                       long max_blocks, hipStream_t st, const float* e0 = nullptr);
// Pairs of partial sums per right-hand side that the borders' buffer holds
// (2D: one per 64 x 4 block of the finest level).
inline long border_partial_blocks(const Grid& g) {
    const long b = (long)((g.m + 63) / 64) * ((g.m + 3) / 4);
    return g.dim == 2 ? b : b * g.m;
}

// out[r][0..1] = sums of partial[r][0..nblk)[0..1] in a fixed order.
void launch_reduce_pairs(const double* partial, int nblk, double* out, int nrhs, hipStream_t st);

// Pack / unpack between the padded level layout and compact interior vectors.
template <typename T>
void launch_pack(const Grid& g, const T* padded, long sp, double* compact, long ld, int nrhs,
                 hipStream_t st);
template <typename T>
void launch_unpack(const Grid& g, const double* compact, long ld, T* padded, long sp, int nrhs,
                   hipStream_t st);

void launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// ----------------------------------------------------------------------------
// Host-side level construction (levels.hip)
// ----------------------------------------------------------------------------
// A general 2D stencil on a padded plane (see Coef): diagonal d and the
// weights of the east, north and north-east edges at their lower-left node.
struct Stencil7 {
    std::vector<double> d, wx, wy, wne;
};
void edge_weights_2d(const Grid& g, const std::vector<double>& kap, std::vector<double>& wx,
                     std::vector<double>& wy);
std::vector<double> coarsen_kappa_2d(const std::vector<double>& kf, int nf);
Stencil7 fine_stencil_2d(const Grid& g, const std::vector<double>& kap, const std::vector<double>& pot);
Stencil7 galerkin_stencil_2d(const Grid& gf, const Stencil7& sf, const Grid& gc);
double gershgorin_2d(const Grid& g, const Stencil7& s);
void dense_from_stencil_2d(const Grid& g, const Stencil7& s, std::vector<double>& A);

// 3D general operators (full diffusion tensor and potential per element,
// Kuhn mesh): 15-point stencils, 8 planes a[0] (diagonal), a[t] = A(i, i + O_t).
struct Stencil15 {
    std::vector<double> a[8];
};
// tensor: 6 values per element (a11 a22 a33 a12 a13 a23) or empty (identity);
// kap: per element factor or empty; pot: V per element or empty
Stencil15 fine_stencil_3d(const Grid& g, const std::vector<double>& tensor, const std::vector<double>& kap,
                          const std::vector<double>& pot);
Stencil15 galerkin_stencil_3d(const Grid& gf, const Stencil15& sf, const Grid& gc);
double gershgorin_3d(const Grid& g, const Stencil15& s);
void dense_from_stencil_3d(const Grid& g, const Stencil15& s, std::vector<double>& A);
template <typename T>
void launch_smooth3g(const Grid& g, const T* s15, const T* xc, const T* xp, const T* f, T* xn, int nrhs,
                     long stride, Cheb s, int zmode, hipStream_t st);
template <typename T>
void launch_apply3g(const Grid& g, const T* s15, const T* x, T* y, int nrhs, long stride, hipStream_t st);
template <typename T>
void launch_resid_restrict3g(const Grid& gf, const T* s15, const T* x, const T* f, const Grid& gc, T* rc, int nrhs,
                             long sf, long sc, hipStream_t st);
template <typename T>
void launch_resid3g(const Grid& g, const T* s15, const T* x, const T* f, T* r, int nrhs, long stride,
                    hipStream_t st);
void launch_resid_cast3g(const Grid& g, const double* s15, const double* u, const double* f, float* r, int nrhs,
                         long stride, hipStream_t st,
                         const double* lam = nullptr);
void launch_add_resid3g(const Grid& g, const double* s15, const double* u, const float* e, const double* f,
                        double* un, float* r, int nrhs, long stride, hipStream_t st,
                        const double* lam = nullptr);
// the borders' fine-level vectors of the 15-point operator; with e (and un),
// of u + e, written to un
int launch_border3g(const Grid& g, const double* s15, const double* u, double* au, double* mu, double* partial,
                    int nrhs, long stride, hipStream_t st, const float* e = nullptr, double* un = nullptr);

// Chebyshev steps of degree s on [rho/alpha, rho]; damped Jacobi steps.
std::vector<Cheb> cheb_steps(double rho, double alpha, int s);
std::vector<Cheb> jacobi_steps(double omega, int s);

// b = a^T (n x n); o[:, j] = q[:, j] / th[j]; b = (float) a; y[r][j] = (j == r mod kpm);
// b = a (n doubles)
void launch_transpose(const double* a, double* b, int n, hipStream_t st);
void launch_scale_cols(const double* q, const double* th, double* o, int n, hipStream_t st);
void launch_d2f(const double* a, float* b, long n, hipStream_t st);
void launch_unit_coefs(double* y, int N, int nrhs, int kpm, hipStream_t st);
void launch_copy(const double* a, double* b, int n, hipStream_t st);
// Restart: y_r = column (r mod kpm) of member r / kpm's Q (padded layout, stride
// sy), unit coefficients in ycoef, lam = lam_prev = theta[member * tstride + j].
void launch_restart_coarse(const double* Mat, int N, const Grid& g, double* y, long sy, double* ycoef, int nrhs,
                           int kpm, long mstride, const double* theta, long tstride, double* lam, double* lam_prev,
                           hipStream_t st);

// ----------------------------------------------------------------------------
// Coarse-space kernels (coarse.hip)
// ----------------------------------------------------------------------------
// y[r] = Mat x[r] with Mat(row, col) stored at Mat[col * N + row]; x and y in
// either the padded layout of level g (flag true) or compact (flag false).
// `work` holds dense_mv_workspace_bytes(N, nrhs) bytes.
// Batches: kpm right-hand sides per member, member m multiplies by the
// matrix at Mat + m * mstride (kpm = 0: one matrix for all).
template <typename T>
void launch_dense_mv(const T* Mat, int N, const Grid& g, const T* x, long sx, bool x_padded,
                     T* y, long sy, bool y_padded, int nrhs, void* work, hipStream_t st, int kpm = 0,
                     long mstride = 0);
size_t dense_mv_workspace_bytes(int N, int nrhs);

struct ArrowIn {
    const double* theta;    // N coarse Ritz values, ascending
    const int* group;       // N: index of the first member of the group of equal theta
    const double* p;        // [k][N] Q^T b
    const double* q;        // [k][N] Q^T c
    const double* bz;       // [k][2] (beta, zeta)
    const double* lam_prev; // [k]
    int N;
    int exhaustive;         // 1: never skip the full root pass
    int kpm = 0;            // eigenpairs per member: theta and group hold N values per member
};
struct ArrowOut {
    double* ycoef;  // [k][N] coefficients y' of the new eigenvector in the Q basis
    double* s;      // [k] weight of u~ in the new eigenvector
    double* mu;     // [k] selected augmented eigenvalue
    int* rank;      // [k]
    double* score;  // [k]
    int* flags;     // [k]
    double* work;   // [k][3N + 8] scratch
};
void launch_arrowhead(const ArrowIn& in, const ArrowOut& out, int k, hipStream_t st);
size_t arrow_workspace_bytes(int N, int k);

// ----------------------------------------------------------------------------
// Learned smoother (learned3d.hip): 3D constant-coefficient levels
// ----------------------------------------------------------------------------
// Operand words of the two weight arrays W[16][27] (see learned3d.hip).
void learned_pack_taps_by_channel(const float* W, unsigned long long* out);   // 128 words
void learned_pack_channels_by_tap(const float* W, unsigned long long* out);   // 128 words
void learned_pack_step(const float* W, unsigned long long* out);            // kLearnedStepOps words
constexpr int kLearnedStepOps = 512;
// out = x + N((f - A x) / D) (x treated as zero when x_zero); ops =
// learned_pack_step(W1 W2).  out must not alias x or f.
template <typename T>
void launch_learned_step(const Grid& g, T w0, const T* x, const T* f, T* out, int nrhs, long stride,
                         const unsigned long long* ops, bool x_zero, hipStream_t st);
// partial[rhs][blk][2] = (sum of (f - A x)^2, sum of f^2 over the block); returns blocks per rhs
template <typename T>
int launch_resid_norm3(const Grid& g, T w0, const T* x, const T* f, double* partial, int nrhs, long stride,
                       hipStream_t st);
template <typename T>
void launch_fill_normal3(const Grid& g, T* x, int nrhs, long stride, unsigned long long seed, hipStream_t st);
template <typename T>
void launch_pack_negA3(const Grid& g, T w0, const T* x, int nrhs, long stride, float* pool, hipStream_t st);

// Training buffers and the loss/gradient evaluation on an m^3 interior grid.
struct LearnedTrainer {
    int m = 0, S = 0;
    float w0 = 1.f;
    unsigned short *rho_p = nullptr, *h_p = nullptr, *g_p = nullptr, *gh = nullptr;
    float *z1 = nullptr, *y_p = nullptr, *d_p = nullptr, *res_p = nullptr;
    float *nr_part = nullptr, *res_part = nullptr, *coef = nullptr, *dw_part = nullptr;
    double* sums = nullptr;
    unsigned long long* ops = nullptr;
    int nblk_vox = 0, dw_blocks = 0, dw_kpw = 16;
    void init(int m, int S, float w0, std::function<void*(size_t)> alloc);
    // loss of the samples r[0..S) (FP32 compact m^3 each) and its gradient
    // (grad [2][16][27]) for the weights W [2][16][27]
    double loss_grad(const float* r, const float* W, double* grad, hipStream_t st);
};

}  // namespace pasm

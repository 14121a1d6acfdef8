// Coarse-space work of Algorithm 1, step 2: the (N_H+1)-dimensional
// generalized eigenproblem of Section 3.1 (matrix form)
//
//     [[A_H, b], [b^T, beta]] z = mu [[M_H, c], [c^T, zeta]] z
//
// and the choice of the eigenvector with the largest component along u~.
//
// The coarse pencil is factored once, A_H Q = M_H Q Theta with Q^T M_H Q = I.
// In the basis [Q, w], w = (u~ - P Q q) / sqrt(zeta_perp), q = Q^T c,
// zeta_perp = zeta - q.q (w is u~ made M-orthogonal to V_H and normalised),
// the augmented mass becomes the identity and the augmented stiffness becomes
// the symmetric arrowhead matrix
//
//     [[Theta, g], [g^T, rho]],  g = (p - Theta q) / sqrt(zeta_perp),
//     rho = (beta - 2 q.p + q.Theta q) / zeta_perp,   p = Q^T b.
//
// Its eigenvalues are the roots of the secular equation
//     f(mu) = rho - mu + sum_j g_j^2 / (mu - theta_j) = 0,
// one in each gap between consecutive poles and one beyond each end; the
// eigenvector is y_j = g_j t / (mu - theta_j) on Q and t on w, with
// t^2 (1 + sum_j (g_j / (mu - theta_j))^2) = 1.  Its component along u~,
// b(u_new, u~) = y.q + t sqrt(zeta_perp), is the selection score of the paper.
//
// Deflation: a group of equal theta (symmetry makes coarse spectra
// degenerate) is rotated so that g has one component in the group; the rest
// of the group is an eigenspace at theta with t = 0, and its best direction
// for the score is the part of q orthogonal to g in the group.  A pole with
// negligible g is itself an eigenvalue with t = 0.
// If u~ lies in V_H (zeta_perp <= 1e-13 zeta) the augmentation is skipped and
// the coarse Ritz pairs are scored instead.
#include <algorithm>
#include <cfloat>

#include <type_traits>

#include <cmath>

#include "common.h"

namespace pasm {

namespace {

constexpr double EPS = DBL_EPSILON;
constexpr double SKIP_RTOL = 1e-13;
constexpr double TIE_RTOL = 1e-12;

// ---------------------------------------------------------------------------
// dense matrix times k vectors, y[r] = Mat x[r], Mat(row,col) at Mat[col*N+row]
//
// Split over column chunks so that even N ~ 10^3 gives hundreds of
// workgroups: pass 1 writes per-chunk partial sums, pass 2 adds the chunks in
// a fixed order (deterministic, no atomics).
// ---------------------------------------------------------------------------
// Shapes: WAVES wavefronts of 64 rows each per workgroup, DC columns per
// chunk, KB right-hand sides per workgroup (the member's k rounded up to a
// multiple of 4, at most 48) -- small coarse spaces take one-wavefront
// workgroups and 64-column chunks, large ones four wavefronts and 128.

__device__ inline long compact_to_padded(const Grid& g, int c) {
    const int i = c % g.m + 1;
    if (g.dim == 2) return g.idx(i, c / g.m + 1);
    const int j = (c / g.m) % g.m + 1;
    return g.idx(i, j, c / (g.m * g.m) + 1);
}

// Batches: right-hand side r belongs to member r / kpm, whose matrix starts
// mstride elements after the previous member's; a workgroup's right-hand
// sides never straddle two members.
template <typename T, int KB, int WAVES, int DC>
__global__ __launch_bounds__(64 * WAVES) void k_dmv_part(const T* __restrict__ Mat, int N, Grid g,
                                                         const T* __restrict__ x, long sx, int xpad,
                                                         T* __restrict__ part, int nrhs, int kpm, long mstride) {
    __shared__ T xs[KB][DC];
    const int row = blockIdx.x * (64 * WAVES) + threadIdx.x;
    const int c0 = blockIdx.y * DC;
    const int zb = (kpm + KB - 1) / KB;  // workgroups per member
    const int mem = blockIdx.z / zb;
    const int rlo = (blockIdx.z % zb) * KB;  // first right-hand side within the member
    const int r0 = mem * kpm + rlo;
    const int rn = min(KB, kpm - rlo);       // right-hand sides of this workgroup
    Mat += (long)mem * mstride;
    const int cn = min(DC, N - c0);
    for (int t = threadIdx.x; t < KB * DC; t += 64 * WAVES) {
        const int rr = t / DC, cc = t % DC;
        T v = T(0);
        if (rr < rn && cc < cn) {
            const long base = (long)(r0 + rr) * sx;
            v = xpad ? x[base + compact_to_padded(g, c0 + cc)] : x[base + c0 + cc];
        }
        xs[rr][cc] = v;
    }
    __syncthreads();
    if (row >= N) return;
    T acc[KB];
#pragma unroll
    for (int rr = 0; rr < KB; ++rr) acc[rr] = T(0);
    // Columns go in groups of PF whose loads are issued one group ahead
    // (enough bytes in flight to cover the memory latency); a partial last
    // chunk re-reads its last column, which meets a zero of xs.
    const T* mc = Mat + (long)c0 * N + row;
    constexpr int PF = 8;
    static_assert(DC % PF == 0, "column chunk must hold whole groups");
    T a[PF], b[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) a[u] = mc[(long)min(u, cn - 1) * N];
    for (int cc = 0; cc < DC; cc += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) b[u] = mc[(long)min(cc + PF + u, cn - 1) * N];
#pragma unroll
        for (int u = 0; u < PF; ++u)
#pragma unroll
            for (int rr = 0; rr < KB; ++rr) acc[rr] += a[u] * xs[rr][cc + u];
#pragma unroll
        for (int u = 0; u < PF; ++u) a[u] = b[u];
    }
#pragma unroll
    for (int rr = 0; rr < KB; ++rr)
        if (rr < rn) part[((long)blockIdx.y * nrhs + r0 + rr) * N + row] = acc[rr];
}

// Double-precision products on the matrix cores (v_mfma_f64_16x16x4_f64):
// a wavefront owns 64 rows (four 16-row tiles) of a DC-column chunk and 16 NT
// right-hand sides; per K-step of 4 columns it loads one matrix element per
// lane and tile (A: lane l holds A[l % 16][l / 16], a coalesced 16-row run
// of each of 4 columns) and reads the staged x as B (lane l holds
// B[l / 16][l % 16]); D comes back as D[4 j + l / 16][l % 16].  Partial sums
// go to part[chunk][row][rhs], summed by k_dmv_sum_rm.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int DMW = 4;  // wavefronts per workgroup (256 rows)
template <int NT, int DC>
__global__ __launch_bounds__(64 * DMW) void k_dmv_mfma(const double* __restrict__ Mat, int N, Grid g,
                                                       const double* __restrict__ x, long sx, int xpad,
                                                       double* __restrict__ part, int nrhs, int kpm, long mstride) {
    constexpr int KBP = 16 * NT;
    constexpr int PF = 4;  // K-steps whose loads are in flight
    __shared__ double xs[DC][KBP + 1];  // padded rows: the staging stores spread over the banks
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row0 = blockIdx.x * (64 * DMW) + wave * 64;
    const int c0 = blockIdx.y * DC;
    const int zb = (kpm + KBP - 1) / KBP;  // workgroups per member
    const int mem = blockIdx.z / zb;
    const int rlo = (blockIdx.z % zb) * KBP;
    const int r0 = mem * kpm + rlo;
    const int rn = min(KBP, kpm - rlo);
    Mat += (long)mem * mstride;
    const int cn = min(DC, N - c0);
    const int ar = lane & 15, ak = lane >> 4;
    // rows past N read row N - 1 (never stored); columns past the chunk read
    // its last column, which meets zeros in xs
    const double* mp[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) mp[mt] = Mat + (long)c0 * N + min(row0 + 16 * mt + ar, N - 1);
    constexpr int KS = DC / 4;
    static_assert(KS % PF == 0, "whole prefetch groups");
    double a[PF][4];
    auto load = [&](int ks, double* dst) {
        const long col = min(4 * ks + ak, cn - 1);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) dst[mt] = mp[mt][col * N];
    };
    // the first K-steps' matrix loads go out before the staging of x, which
    // they do not need
#pragma unroll
    for (int p = 0; p < PF; ++p) load(p, a[p]);
    {
        // consecutive threads take consecutive columns (coalesced), and a
        // thread issues a batch of loads before storing any of them
        constexpr int TPB = 64 * DMW, E = DC * KBP / TPB, BATCH = 8;
        static_assert(DC % TPB == 0 || TPB % DC == 0, "staging layout");
        const int cc = threadIdx.x % DC;
        const long xc = cc < cn ? (xpad ? compact_to_padded(g, c0 + cc) : c0 + cc) : 0;
        for (int e0 = 0; e0 < E; e0 += BATCH) {
            double v[BATCH];
#pragma unroll
            for (int e = 0; e < BATCH; ++e) {
                const int rr = (threadIdx.x + TPB * (e0 + e)) / DC;
                v[e] = (e0 + e < E && rr < rn && cc < cn) ? x[(long)(r0 + rr) * sx + xc] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < BATCH; ++e) {
                const int rr = (threadIdx.x + TPB * (e0 + e)) / DC;
                if (e0 + e < E) xs[cc][rr] = v[e];
            }
        }
    }
    __syncthreads();
    f64x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < KS; k0 += PF) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int ks = k0 + p;
            double b[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = xs[4 * ks + ak][16 * nt + ar];
            double cur[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) cur[mt] = a[p][mt];
            load(min(ks + PF, KS - 1), a[p]);  // the slot refills at once
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[mt], b[nt], acc[mt][nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int rr = 16 * nt + ar;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = row0 + 16 * mt + 4 * j + ak;
                if (rr < rn && row < N) part[((long)blockIdx.y * N + row) * nrhs + r0 + rr] = acc[mt][nt][j];
            }
        }
}

// y[r][row] = sum over chunks of part[chunk][row][r]
__global__ __launch_bounds__(256) void k_dmv_sum_rm(int N, int nchunk, const double* __restrict__ part, int nrhs,
                                                    Grid g, double* __restrict__ y, long sy, int ypad) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)N * nrhs) return;
    const int row = (int)(t / nrhs), r = (int)(t % nrhs);
    const long cs = (long)N * nrhs;
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= nchunk; c += 8) {  // eight loads in flight, summed in chunk order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(c + u) * cs + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nchunk; ++c) s += part[c * cs + t];
    const long base = (long)r * sy;
    if (ypad) y[base + compact_to_padded(g, row)] = s;
    else y[base + row] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dmv_sum(int N, int nchunk, const T* __restrict__ part, int nrhs, Grid g,
                                                 T* __restrict__ y, long sy, int ypad) {
    const int row = blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
    if (row >= N) return;
    T s = T(0);
    for (int c = 0; c < nchunk; ++c) s += part[((long)c * nrhs + r) * N + row];
    const long base = (long)r * sy;
    if (ypad) y[base + compact_to_padded(g, row)] = s;
    else y[base + row] = s;
}

// ---------------------------------------------------------------------------
// arrowhead workspace layout, per eigenpair (doubles)
// ---------------------------------------------------------------------------
struct WS {
    double* g;       // N   g_j
    double* d;       // N   active pole values (ascending)
    double* z;       // N   active pole weights (signed for singletons, |g_G| for groups)
    double* qa;      // N   component of q along the active direction
    double* rmu;     // N+1 root values
    double* rtau;    // N+1 root offsets from their origin pole
    double* rorg;    // N+1 origin pole values
    double* sc;      // 16 scalars, see below
    int* amap;       // N   active index of j's group, -1 if deflated
    double* best;    // [nchunk][4] per-block best root (score, mu, root, 0)
};
// scalar slots
enum {
    S_RHO = 0, S_SQ, S_ZPERP, S_NA, S_LO, S_HI, S_SKIP, S_DSCORE, S_DMU, S_DLEAD, S_DTYPE, S_TOLZ,
    S_DMASS,   // sum of the squared scores of all deflated candidates
    S_CERT,    // 1: the roots next to the previous eigenvalue provably contain the winner
    S_NSCORE, S_NMU  // best of those roots (score, root index in S_NMU + 1 slot below)
};

__host__ __device__ inline long ws_doubles(int N) { return 7L * N + 3 + 20; }

__device__ inline WS ws_of(double* work, int* iwork, double* best, int N, int nchunk, int r) {
    WS w;
    double* b = work + (long)r * ws_doubles(N);
    w.g = b;
    w.d = b + N;
    w.z = b + 2L * N;
    w.qa = b + 3L * N;
    w.rmu = b + 4L * N;
    w.rtau = b + 5L * N + 1;
    w.rorg = b + 6L * N + 2;
    w.sc = b + 7L * N + 3;
    w.amap = iwork + (long)r * N;
    w.best = best + (long)r * nchunk * 4;
    return w;
}

// candidate comparison: larger score; within TIE_RTOL the one nearer to the
// previous eigenvalue, then the lower eigenvalue.
__device__ inline bool better(double s1, double m1, double s2, double m2, double lp) {
    if (s1 > s2 * (1.0 + TIE_RTOL)) return true;
    if (s2 > s1 * (1.0 + TIE_RTOL)) return false;
    const double d1 = fabs(m1 - lp), d2 = fabs(m2 - lp);
    if (d1 != d2) return d1 < d2;
    return m1 < m2;
}

constexpr int PT = 256;
constexpr int PP = 1024;  // threads of the preparation workgroup

__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = sh[0] + sh[1] + sh[2] + sh[3];
    return s;
}
// the same for NW wavefronts, in a fixed order
template <int NW>
__device__ inline double block_sum_n(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += sh[w];
    return s;
}
template <int NW>
__device__ inline double block_max_n(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = fmax(s, sh[w]);
    return s;
}

__device__ inline double block_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// Stage A, one block per eigenpair: scalars, g, deflation, compaction of the
// active poles, and the best deflated candidate.
// ST: the group map, g and q of the eigenpair staged in LDS (N <= PMAXN), so
// that the group scans below read LDS instead of waiting on global loads.
constexpr int PMAXN = 4096;
template <bool ST>
__global__ __launch_bounds__(PP) void k_arrow_prep(ArrowIn in, double* work, int* iwork, double* best, int nchunk) {
    constexpr int NWV = PP / 64;
    constexpr int NS = ST ? PMAXN : 1;
    __shared__ int lgrp[NS];
    __shared__ double lg[NS], lq[NS];
    __shared__ double sh[NWV];
    __shared__ int wtot[NWV];
    __shared__ int cnt[PP];
    __shared__ double bs[PP], bm[PP];
    __shared__ int bl[PP], bt[PP];
    const int r = blockIdx.x, N = in.N;
    in.theta += (long)(r / in.kpm) * N;  // this eigenpair's member
    in.group += (long)(r / in.kpm) * N;
    WS w = ws_of(work, iwork, best, N, nchunk, r);
    const double* p = in.p + (long)r * N;
    const double* q = in.q + (long)r * N;
    auto GRP = [&](int j) -> int {
        if constexpr (ST) return lgrp[j];
        else return in.group[j];
    };
    auto GG = [&](int j) -> double {
        if constexpr (ST) return lg[j];
        else return w.g[j];
    };
    auto QQ = [&](int j) -> double {
        if constexpr (ST) return lq[j];
        else return q[j];
    };
    const double beta = in.bz[2 * r], zeta = in.bz[2 * r + 1], lp = in.lam_prev[r];

    // the first CE poles of the thread in registers, their loads issued
    // together (the sums keep the order of a plain strided loop)
    constexpr int CE = 4;
    static_assert(!ST || CE * PP >= PMAXN, "staged poles all in the register cache");
    double qv[CE], pv[CE], tv[CE];
    int gv[CE];
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int j = min((int)threadIdx.x + e * PP, N - 1);
        qv[e] = q[j];
        pv[e] = p[j];
        tv[e] = in.theta[j];
        if constexpr (ST) gv[e] = in.group[j];
    }
    if constexpr (ST) {
#pragma unroll
        for (int e = 0; e < CE; ++e) {
            const int j = threadIdx.x + e * PP;
            if (j < N) {
                lgrp[j] = gv[e];
                lq[j] = qv[e];
            }
        }
    }
    double qq = 0, qp = 0, qtq = 0;
#pragma unroll
    for (int e = 0; e < CE; ++e)
        if ((int)threadIdx.x + e * PP < N) {
            qq += qv[e] * qv[e];
            qp += qv[e] * pv[e];
            qtq += tv[e] * qv[e] * qv[e];
        }
    for (int j = threadIdx.x + CE * PP; j < N; j += PP) {
        qq += q[j] * q[j];
        qp += q[j] * p[j];
        qtq += in.theta[j] * q[j] * q[j];
    }
    qq = block_sum_n<NWV>(qq, sh);
    qp = block_sum_n<NWV>(qp, sh);
    qtq = block_sum_n<NWV>(qtq, sh);
    const double zperp = zeta - qq;
    const bool skip = !(zperp > SKIP_RTOL * zeta);
    const double sq = skip ? 0.0 : sqrt(zperp);
    const double rho = skip ? 0.0 : (beta - 2.0 * qp + qtq) / zperp;

    double gmax = 0.0;
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int j = threadIdx.x + e * PP;
        if (j < N) {
            const double gj = skip ? 0.0 : (pv[e] - tv[e] * qv[e]) / sq;
            w.g[j] = gj;
            if constexpr (ST) lg[j] = gj;
            gmax = fmax(gmax, fabs(gj));
        }
    }
    for (int j = threadIdx.x + CE * PP; j < N; j += PP) {
        const double gj = skip ? 0.0 : (p[j] - in.theta[j] * q[j]) / sq;
        w.g[j] = gj;
        if constexpr (ST) lg[j] = gj;
        gmax = fmax(gmax, fabs(gj));
    }
    gmax = block_max_n<NWV>(gmax, sh);
    const double tolz = 8.0 * EPS * fmax(fmax(fabs(in.theta[N - 1]), fabs(rho)), gmax);
    __syncthreads();

    // contiguous chunk of indices per thread, so the compaction keeps order
    const int per = (N + PP - 1) / PP;
    const int j0 = threadIdx.x * per, j1 = min(N, j0 + per);
    int mine = 0;
    double ds = -1.0, dm = 0.0, dmass = 0.0;
    int dl = -1, dt = 0;
    for (int j = j0; j < j1; ++j) {
        if (GRP(j) != j) continue;  // not a group leader
        int e = j + 1;
        while (e < N && GRP(e) == j) ++e;
        double gn2 = 0.0, q2 = 0.0, gq = 0.0;
        for (int m = j; m < e; ++m) {
            gn2 += GG(m) * GG(m);
            q2 += QQ(m) * QQ(m);
            gq += GG(m) * QQ(m);
        }
        const double gn = sqrt(gn2);
        double cs = -1.0;
        int ct = 0;
        if (skip || gn <= tolz) {
            cs = sqrt(q2);
            ct = 1;
        } else {
            ++mine;
            if (e - j > 1) {
                const double qg = gq / gn;
                cs = sqrt(fmax(q2 - qg * qg, 0.0));
                ct = 2;
            }
        }
        if (ct) dmass += cs * cs;
        if (ct && (dl < 0 || better(cs, in.theta[j], ds, dm, lp))) {
            ds = cs;
            dm = in.theta[j];
            dl = j;
            dt = ct;
        }
    }
    dmass = block_sum_n<NWV>(dmass, sh);
    // exclusive prefix of the active counts (wavefront scans, then the
    // wavefront totals), so that active poles keep their order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[wv] = inc;
    bs[threadIdx.x] = ds;
    bm[threadIdx.x] = dm;
    bl[threadIdx.x] = dl;
    bt[threadIdx.x] = dt;
    __syncthreads();
    int woff = 0, acc = 0;
    for (int t = 0; t < NWV; ++t) {
        if (t < wv) woff += wtot[t];
        acc += wtot[t];
    }
    cnt[threadIdx.x] = woff + inc - mine;
    // best deflated candidate: pairwise reduction in a fixed tree
    for (int h = PP / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int o = threadIdx.x + h;
            const bool take = bl[o] >= 0 &&
                              (bl[threadIdx.x] < 0 || better(bs[o], bm[o], bs[threadIdx.x], bm[threadIdx.x], lp) ||
                               (!better(bs[threadIdx.x], bm[threadIdx.x], bs[o], bm[o], lp) && bl[o] < bl[threadIdx.x]));
            if (take) {
                bs[threadIdx.x] = bs[o];
                bm[threadIdx.x] = bm[o];
                bl[threadIdx.x] = bl[o];
                bt[threadIdx.x] = bt[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int bi = bl[0] >= 0 ? 0 : -1;
        w.sc[S_NA] = skip ? -1.0 : (double)acc;
        w.sc[S_RHO] = rho;
        w.sc[S_SQ] = sq;
        w.sc[S_ZPERP] = zperp;
        w.sc[S_SKIP] = skip ? 1.0 : 0.0;
        w.sc[S_TOLZ] = tolz;
        w.sc[S_DMASS] = dmass;
        w.sc[S_CERT] = 0.0;
        w.sc[S_DSCORE] = bi < 0 ? -1.0 : bs[bi];
        w.sc[S_DMU] = bi < 0 ? 0.0 : bm[bi];
        w.sc[S_DLEAD] = bi < 0 ? -1.0 : (double)bl[bi];
        w.sc[S_DTYPE] = bi < 0 ? 0.0 : (double)bt[bi];
    }
    __syncthreads();
    // write active poles in order
    int a = cnt[threadIdx.x];
    for (int j = j0; j < j1; ++j) {
        if (GRP(j) != j) continue;
        int e = j + 1;
        while (e < N && GRP(e) == j) ++e;
        double gn2 = 0.0, gq = 0.0;
        for (int m = j; m < e; ++m) {
            gn2 += GG(m) * GG(m);
            gq += GG(m) * QQ(m);
        }
        const double gn = sqrt(gn2);
        const bool act = !skip && gn > tolz;
        for (int m = j; m < e; ++m) w.amap[m] = act ? a : -1;
        if (act) {
            w.d[a] = in.theta[j];
            if (e - j == 1) {
                w.z[a] = GG(j);
                w.qa[a] = QQ(j);
            } else {
                w.z[a] = gn;
                w.qa[a] = gq / gn;
            }
            ++a;
        }
    }
    __syncthreads();
    // |z| over the active poles (a block reduction, fixed order)
    const int nact = skip ? 0 : (int)w.sc[S_NA];
    double zn2 = 0.0;
    for (int t = threadIdx.x; t < nact; t += PP) zn2 += w.z[t] * w.z[t];
    zn2 = block_sum_n<NWV>(zn2, sh);
    if (threadIdx.x == 0 && nact > 0) {
        const double zn = sqrt(zn2);
        w.sc[S_LO] = fmin(w.d[0], rho) - zn;
        w.sc[S_HI] = fmax(w.d[nact - 1], rho) + zn;
    }
}

// Stage B: roots of the secular equation, one wavefront per root; the 64
// lanes split the sums over the poles and combine them with an xor butterfly,
// which leaves the same (bitwise) value in every lane, so the iteration stays
// uniform across the wavefront.
//
// Root r lies between consecutive poles (or beyond an end).  The pole nearer
// to the root (decided from the sign of f at the interval midpoint) becomes
// the origin, tau = mu - origin, and Newton's method is applied to
// h(tau) = tau f(tau), which no longer has a pole at the origin; iterates are
// kept inside the shrinking sign bracket (bisection otherwise).
constexpr int RW = 64;          // lanes per root
constexpr int RWAVES = 4;       // wavefronts per block
constexpr int RPB = 16;         // roots per block (each wavefront takes 4 in turn)
constexpr int LDS_POLES = 2600; // poles kept in LDS up to this count
constexpr int LDS_POLES_BIG = 6400;  // ... for the one-workgroup-per-eigenpair NEAR pass (150 KiB of LDS)

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Root offset of the NEAR pass: the RPB roots around the interval that holds
// the previous eigenvalue (root a lies between active poles a-1 and a).
__device__ inline int near_base(const double* d, int na, double lp) {
    int lo = 0, hi = na;  // number of active poles below lp, by bisection
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (d[mid] < lp) lo = mid + 1;
        else hi = mid;
    }
    int base = lo - RPB / 2;
    if (base > na + 1 - RPB) base = na + 1 - RPB;
    if (base < 0) base = 0;
    return base;
}

// NEAR = true: one workgroup per eigenpair computes the RPB roots next to the
// previous eigenvalue and decides whether they certainly contain the winner.
// Every eigenvector of the arrowhead matrix has a score (its component along
// m = [q; sqrt(zeta_perp)]); the eigenvectors are orthonormal, so the squared
// scores of ALL candidates add up to |m|^2 = zeta.  If the best computed root
// beats every deflated candidate and its squared score exceeds what is left
// for the uncomputed roots (zeta minus the computed squared scores), no other
// root can win, ties included.  NEAR = false: all roots, skipped when the
// NEAR pass certified its winner.
template <int LDSN, bool NEAR, int NW = RWAVES>
__global__ __launch_bounds__(RW* NW) void k_arrow_roots(ArrowIn in, double* work, int* iwork, double* best,
                                                        int nchunk) {
    constexpr bool LDS = LDSN > 0;
    __shared__ double sd[LDS ? LDSN : 1], sz[LDS ? LDSN : 1], sqa[LDS ? LDSN : 1];
    __shared__ double ss[RPB], sm[RPB];
    const int r = blockIdx.x, N = in.N;
    WS w = ws_of(work, iwork, best, N, nchunk, r);
    if (!NEAR && w.sc[S_CERT] != 0.0) return;  // uniform per workgroup
    const int na = (int)w.sc[S_NA];
    const double rho = w.sc[S_RHO], sq = w.sc[S_SQ], lp = in.lam_prev[r];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double* d = w.d;
    const double* z = w.z;
    const double* qa = w.qa;
    if (LDS) {
        for (int a = threadIdx.x; a < na; a += RW * NW) {
            sd[a] = w.d[a];
            sz[a] = w.z[a];
            sqa[a] = w.qa[a];
        }
        __syncthreads();
        d = sd;
        z = sz;
        qa = sqa;
    }
    const int base = NEAR ? (na > 0 ? near_base(d, na, lp) : 0) : blockIdx.y * RPB;
    for (int slot = wave; slot < RPB; slot += NW) {
        const int root = base + slot;
        double score = -1.0, mu = 0.0;
        if (na >= 0 && root <= na) {
            if (na == 0) {
                mu = rho;
                score = sq;
                if (lane == 0) {
                    w.rmu[0] = rho;
                    w.rtau[0] = 0.0;
                    w.rorg[0] = rho;
                }
            } else {
                const double left = root == 0 ? w.sc[S_LO] : d[root - 1];
                const double right = root == na ? w.sc[S_HI] : d[root];
                double org, lo, hi;
                if (root == 0) {
                    org = d[0];
                    lo = left - org;
                    hi = 0.0;
                } else if (root == na) {
                    org = d[na - 1];
                    lo = 0.0;
                    hi = right - org;
                } else {
                    const double mid = 0.5 * (left + right);
                    double fm = 0.0;
                    for (int a = lane; a < na; a += RW) fm += z[a] * z[a] / (mid - d[a]);
                    fm = wave_sum(fm) + (rho - mid);
                    if (fm > 0.0) {  // root in (mid, right): origin at the right pole
                        org = right;
                        lo = mid - org;
                        hi = 0.0;
                    } else {
                        org = left;
                        lo = 0.0;
                        hi = mid - org;
                    }
                }
                const double c0 = rho - org;
                double tau = 0.5 * (lo + hi);
                for (int it = 0; it < 100; ++it) {
                    double F = 0.0, dF = 0.0, mag = 0.0;
                    for (int a = lane; a < na; a += RW) {
                        const double t1 = z[a] / (tau - (d[a] - org));
                        F += z[a] * t1;
                        dF -= t1 * t1;
                        mag += fabs(z[a] * t1);
                    }
                    F = wave_sum(F) + (c0 - tau);
                    dF = wave_sum(dF) - 1.0;
                    mag = wave_sum(mag) + fabs(c0) + fabs(tau);
                    if (F == 0.0) break;
                    if (F > 0.0) lo = tau;
                    else hi = tau;
                    if (fabs(F) <= 4.0 * EPS * mag) break;
                    const double hval = tau * F, dh = F + tau * dF;
                    double tn = tau - hval / dh;
                    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
                    const double step = fabs(tn - tau);
                    tau = tn;
                    if (step <= 2.0 * EPS * fabs(tau) || hi - lo <= 4.0 * EPS * fmax(fabs(lo), fabs(hi))) break;
                }
                double S1 = 0.0, S2 = 0.0;
                for (int a = lane; a < na; a += RW) {
                    const double v = z[a] / (tau - (d[a] - org));
                    S1 += v * v;
                    S2 += v * qa[a];
                }
                S1 = wave_sum(S1);
                S2 = wave_sum(S2);
                const double t = 1.0 / sqrt(1.0 + S1);
                score = fabs(t * (S2 + sq));
                mu = org + tau;
                if (lane == 0) {
                    w.rmu[root] = mu;
                    w.rtau[root] = tau;
                    w.rorg[root] = org;
                }
            }
        }
        if (lane == 0) {
            ss[slot] = score;
            sm[slot] = mu;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int bi = -1;
        double mass = 0.0;
        for (int t = 0; t < RPB; ++t) {
            if (ss[t] < 0.0) continue;
            mass += ss[t] * ss[t];
            if (bi < 0 || better(ss[t], sm[t], ss[bi], sm[bi], lp)) bi = t;
        }
        if (NEAR) {
            w.sc[S_NSCORE] = bi < 0 ? -1.0 : ss[bi];
            w.sc[S_NMU] = bi < 0 ? 0.0 : sm[bi];
            w.sc[S_NMU + 1] = bi < 0 ? -1.0 : (double)(base + bi);
            bool cert = false;
            if (bi >= 0) {
                const double zeta = in.bz[2 * r + 1];
                const double rest = zeta - w.sc[S_DMASS] - mass;
                const double b2 = ss[bi] * ss[bi];
                const bool beats_deflated =
                    w.sc[S_DSCORE] < 0.0 || better(ss[bi], sm[bi], w.sc[S_DSCORE], w.sc[S_DMU], lp);
                cert = beats_deflated && b2 > fmax(rest, 0.0) * (1.0 + 1e-10) + 1e-10 * zeta * EPS;
                if (base == 0 && na + 1 <= RPB) cert = beats_deflated;  // every root was computed
                if (in.exhaustive) cert = false;
            }
            w.sc[S_CERT] = cert ? 1.0 : 0.0;
        } else {
            double* b = w.best + 4L * blockIdx.y;
            b[0] = bi < 0 ? -1.0 : ss[bi];
            b[1] = bi < 0 ? 0.0 : sm[bi];
            b[2] = bi < 0 ? -1.0 : (double)(blockIdx.y * RPB + bi);
            b[3] = 0.0;
        }
    }
}

// The NEAR pass spread over the machine: one workgroup of four wavefronts
// per (eigenpair, root), the active poles in registers (PPL per lane), the
// sums over poles reduced across the workgroup in a fixed order so that every
// wavefront takes the same Newton steps.  Same iteration as k_arrow_roots;
// its (score, root value) goes to nres for k_arrow_near_cert.
constexpr int NT = 256;  // threads per root
template <int PPL>
__global__ __launch_bounds__(NT) void k_arrow_near_root(ArrowIn in, double* work, int* iwork, double* best,
                                                        int nchunk, double* nres) {
    __shared__ double red[2][3][NT / 64];
    const int r = blockIdx.x, slot = blockIdx.y, N = in.N;
    const int tid = threadIdx.x, wave = tid >> 6;
    WS w = ws_of(work, iwork, best, N, nchunk, r);
    double* res = nres + ((long)r * RPB + slot) * 2;
    const int na = (int)w.sc[S_NA];
    const double rho = w.sc[S_RHO], sq = w.sc[S_SQ], lp = in.lam_prev[r];
    const int base = na > 0 ? near_base(w.d, na, lp) : 0;
    const int root = base + slot;
    if (na < 0 || root > na) {  // uniform
        if (tid == 0) {
            res[0] = -1.0;
            res[1] = 0.0;
        }
        return;
    }
    if (na == 0) {
        if (tid == 0) {
            w.rmu[0] = rho;
            w.rtau[0] = 0.0;
            w.rorg[0] = rho;
            res[0] = sq;
            res[1] = rho;
        }
        return;
    }
    // poles beyond na: weight 0 and a far pole, so that they add exact zeros
    double dr[PPL], zr[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int a = tid + NT * p;
        dr[p] = a < na ? w.d[a] : 1e300;
        zr[p] = a < na ? w.z[a] : 0.0;
    }
    int par = 0;
    auto sum3 = [&](double& x, double& y, double& z) {
        x = wave_sum(x);
        y = wave_sum(y);
        z = wave_sum(z);
        if ((tid & 63) == 0) {
            red[par][0][wave] = x;
            red[par][1][wave] = y;
            red[par][2][wave] = z;
        }
        __syncthreads();
        x = y = z = 0.0;
#pragma unroll
        for (int v = 0; v < NT / 64; ++v) {
            x += red[par][0][v];
            y += red[par][1][v];
            z += red[par][2][v];
        }
        par ^= 1;
    };
    const double left = root == 0 ? w.sc[S_LO] : w.d[root - 1];
    const double right = root == na ? w.sc[S_HI] : w.d[root];
    double org, lo, hi;
    if (root == 0) {
        org = w.d[0];
        lo = left - org;
        hi = 0.0;
    } else if (root == na) {
        org = w.d[na - 1];
        lo = 0.0;
        hi = right - org;
    } else {
        const double mid = 0.5 * (left + right);
        double fm = 0.0, u1 = 0.0, u2 = 0.0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) fm += zr[p] * zr[p] / (mid - dr[p]);
        sum3(fm, u1, u2);
        fm += rho - mid;
        if (fm > 0.0) {  // root in (mid, right): origin at the right pole
            org = right;
            lo = mid - org;
            hi = 0.0;
        } else {
            org = left;
            lo = 0.0;
            hi = mid - org;
        }
    }
    const double c0 = rho - org;
    double tau = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double F = 0.0, dF = 0.0, mag = 0.0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const double t1 = zr[p] / (tau - (dr[p] - org));
            F += zr[p] * t1;
            dF -= t1 * t1;
            mag += fabs(zr[p] * t1);
        }
        sum3(F, dF, mag);
        F += c0 - tau;
        dF -= 1.0;
        mag += fabs(c0) + fabs(tau);
        if (F == 0.0) break;
        if (F > 0.0) lo = tau;
        else hi = tau;
        if (fabs(F) <= 4.0 * EPS * mag) break;
        const double hval = tau * F, dh = F + tau * dF;
        double tn = tau - hval / dh;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        const double step = fabs(tn - tau);
        tau = tn;
        if (step <= 2.0 * EPS * fabs(tau) || hi - lo <= 4.0 * EPS * fmax(fabs(lo), fabs(hi))) break;
    }
    double S1 = 0.0, S2 = 0.0, u3 = 0.0;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int a = tid + NT * p;
        const double v = zr[p] / (tau - (dr[p] - org));
        S1 += v * v;
        S2 += v * (a < na ? w.qa[a] : 0.0);
    }
    sum3(S1, S2, u3);
    if (tid == 0) {
        const double t = 1.0 / sqrt(1.0 + S1);
        const double mu = org + tau;
        w.rmu[root] = mu;
        w.rtau[root] = tau;
        w.rorg[root] = org;
        res[0] = fabs(t * (S2 + sq));
        res[1] = mu;
    }
}

// Selection and certificate of the NEAR pass (as at the end of k_arrow_roots).
__global__ __launch_bounds__(64) void k_arrow_near_cert(ArrowIn in, double* work, int* iwork, double* best,
                                                        int nchunk, const double* nres) {
    if (threadIdx.x != 0) return;
    const int r = blockIdx.x, N = in.N;
    WS w = ws_of(work, iwork, best, N, nchunk, r);
    const int na = (int)w.sc[S_NA];
    const double lp = in.lam_prev[r];
    const int base = na > 0 ? near_base(w.d, na, lp) : 0;
    const double* res = nres + (long)r * RPB * 2;
    int bi = -1;
    double mass = 0.0;
    for (int t = 0; t < RPB; ++t) {
        const double st = res[2 * t], mt = res[2 * t + 1];
        if (st < 0.0) continue;
        mass += st * st;
        if (bi < 0 || better(st, mt, res[2 * bi], res[2 * bi + 1], lp)) bi = t;
    }
    const double sb = bi < 0 ? -1.0 : res[2 * bi], mb = bi < 0 ? 0.0 : res[2 * bi + 1];
    w.sc[S_NSCORE] = sb;
    w.sc[S_NMU] = mb;
    w.sc[S_NMU + 1] = bi < 0 ? -1.0 : (double)(base + bi);
    bool cert = false;
    if (bi >= 0) {
        const double zeta = in.bz[2 * r + 1];
        const double rest = zeta - w.sc[S_DMASS] - mass;
        const double b2 = sb * sb;
        const bool beats_deflated = w.sc[S_DSCORE] < 0.0 || better(sb, mb, w.sc[S_DSCORE], w.sc[S_DMU], lp);
        cert = beats_deflated && b2 > fmax(rest, 0.0) * (1.0 + 1e-10) + 1e-10 * zeta * EPS;
        if (base == 0 && na + 1 <= RPB) cert = beats_deflated;  // every root was computed
        if (in.exhaustive) cert = false;
    }
    w.sc[S_CERT] = cert ? 1.0 : 0.0;
}

// Stage C, one block per eigenpair: final choice, rank, new coefficients.
constexpr int PF_T = 1024;  // threads of the final stage
__global__ __launch_bounds__(PF_T) void k_arrow_final(ArrowIn in, ArrowOut out, double* work, int* iwork, double* best,
                                                    int nchunk) {
    __shared__ double sh[PF_T / 64];
    __shared__ double win[4];  // score, mu, kind (0 root, 1 deflated), id
    __shared__ int rk;
    const int r = blockIdx.x, N = in.N;
    in.theta += (long)(r / in.kpm) * N;  // this eigenpair's member
    in.group += (long)(r / in.kpm) * N;
    WS w = ws_of(work, iwork, best, N, nchunk, r);
    const double* q = in.q + (long)r * N;
    const double lp = in.lam_prev[r];
    const int na = (int)w.sc[S_NA];
    const double sq = w.sc[S_SQ];
    if (threadIdx.x == 0) {
        double bsc = -1.0, bmu = 0.0, kind = 0.0, id = -1.0;
        if (na >= 0 && w.sc[S_CERT] != 0.0) {
            bsc = w.sc[S_NSCORE];
            bmu = w.sc[S_NMU];
            id = w.sc[S_NMU + 1];
        } else if (na >= 0) {
            for (int c = 0; c < nchunk; ++c) {
                const double* b = w.best + 4L * c;
                if (b[0] < 0.0) continue;
                if (id < 0.0 || better(b[0], b[1], bsc, bmu, lp)) {
                    bsc = b[0];
                    bmu = b[1];
                    kind = 0.0;
                    id = b[2];
                }
            }
        }
        const double ds = w.sc[S_DSCORE];
        if (ds >= 0.0 && (id < 0.0 || better(ds, w.sc[S_DMU], bsc, bmu, lp))) {
            bsc = ds;
            bmu = w.sc[S_DMU];
            kind = 1.0;
            id = w.sc[S_DLEAD];
        }
        win[0] = bsc;
        win[1] = bmu;
        win[2] = kind;
        win[3] = id;
        rk = 0;
    }
    __syncthreads();
    const double mu = win[1];
    const bool is_root = win[2] == 0.0;
    const int id = (int)win[3];

    // rank: augmented eigenvalues strictly below mu (roots, then deflated
    // eigenvalues with their multiplicities)
    int cntb = 0;
    if (na >= 0) {
        const int nroots = na == 0 ? 1 : na + 1;
        for (int t = threadIdx.x; t < nroots; t += PF_T)
            if (is_root ? t < id : w.rmu[t] < mu) ++cntb;
    }
    for (int j = threadIdx.x; j < N; j += PF_T) {
        if (in.group[j] != j || in.theta[j] >= mu) continue;
        int e = j + 1;
        while (e < N && in.group[e] == j) ++e;
        if (w.amap[j] < 0) cntb += e - j;
        else cntb += e - j - 1;
    }
    atomicAdd(&rk, cntb);

    // eigenvector coefficients in the Q basis, and t; the thread's first CE
    // coefficients (and q values) stay in registers until the final write
    constexpr int CE = 4;
    double yv[CE], qv[CE];
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        qv[e] = q[min((int)threadIdx.x + e * PF_T, N - 1)];
        yv[e] = 0.0;
    }
    double t = 0.0;
    double* y = out.ycoef + (long)r * N;
    if (is_root) {
        if (na == 0) {
            t = 1.0;
            for (int j = threadIdx.x + CE * PF_T; j < N; j += PF_T) y[j] = 0.0;
        } else {
            const double tau = w.rtau[id], org = w.rorg[id];
            double s1 = 0.0;
            for (int a = threadIdx.x; a < na; a += PF_T) {
                const double v = w.z[a] / (tau - (w.d[a] - org));
                s1 += v * v;
            }
            s1 = block_sum_n<PF_T / 64>(s1, sh);
            t = 1.0 / sqrt(1.0 + s1);
#pragma unroll
            for (int e = 0; e < CE; ++e) {
                const int j = threadIdx.x + e * PF_T;
                if (j < N) {
                    const int a = w.amap[j];
                    yv[e] = a < 0 ? 0.0 : w.g[j] * t / (tau - (w.d[a] - org));
                }
            }
            for (int j = threadIdx.x + CE * PF_T; j < N; j += PF_T) {
                const int a = w.amap[j];
                y[j] = a < 0 ? 0.0 : w.g[j] * t / (tau - (w.d[a] - org));
            }
        }
    } else {
        const int lead = id;
        int e = lead + 1;
        while (e < N && in.group[e] == lead) ++e;
        const int type = (int)w.sc[S_DTYPE];
        // direction in the group: q (type 1) or q minus its g component (type 2)
        double gn2 = 0.0, gq = 0.0;
        for (int m = lead; m < e; ++m) {
            gn2 += w.g[m] * w.g[m];
            gq += w.g[m] * q[m];
        }
        const double coef = (type == 2 && gn2 > 0.0) ? gq / gn2 : 0.0;
        double nrm2 = 0.0;
        for (int m = lead; m < e; ++m) {
            const double v = q[m] - coef * w.g[m];
            nrm2 += v * v;
        }
        const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
#pragma unroll
        for (int ce = 0; ce < CE; ++ce) {
            const int j = threadIdx.x + ce * PF_T;
            if (j < N && j >= lead && j < e) yv[ce] = (qv[ce] - coef * w.g[j]) * inv;
        }
        for (int j = threadIdx.x + CE * PF_T; j < N; j += PF_T)
            y[j] = (j >= lead && j < e) ? (q[j] - coef * w.g[j]) * inv : 0.0;
    }
    __syncthreads();
    // signed score, then y' = y - (t / sq) q and s = t / sq
    double ys = 0.0;
#pragma unroll
    for (int e = 0; e < CE; ++e)
        if ((int)threadIdx.x + e * PF_T < N) ys += yv[e] * qv[e];
    for (int j = threadIdx.x + CE * PF_T; j < N; j += PF_T) ys += y[j] * q[j];
    ys = block_sum_n<PF_T / 64>(ys, sh);
    const double signed_score = ys + t * sq;
    const double sgn = signed_score < 0.0 ? -1.0 : 1.0;
    const double s = (sq > 0.0) ? t / sq : 0.0;
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int j = threadIdx.x + e * PF_T;
        if (j < N) y[j] = sgn * (yv[e] - s * qv[e]);
    }
    for (int j = threadIdx.x + CE * PF_T; j < N; j += PF_T) y[j] = sgn * (y[j] - s * q[j]);
    __syncthreads();
    if (threadIdx.x == 0) {
        out.s[r] = sgn * s;
        out.mu[r] = mu;
        out.rank[r] = rk;
        out.score[r] = fabs(signed_score);
        out.flags[r] = (w.sc[S_SKIP] != 0.0 ? 1 : 0) | (is_root ? 0 : 2);
    }
}


// Exact coarse solve for the constant-coefficient 2D operator: A_H = w0 (4 at
// the centre, -1 at the four axis neighbours) is diagonalised by the sine
// transform in each direction, A_H = (S x S) diag(w0 (c_a + c_b)) (S x S),
// with S the orthonormal DST-I matrix of order n - 1 (S = S^T = S^-1,
// S_aj = sqrt(2/n) sin(pi (a+1)(j+1)/n)) and c_a = 2 - 2 cos(pi (a+1)/n), so
// x = S (inv .* (S r S)) S with inv_ab = 1 / (w0 (c_a + c_b)).  One workgroup
// of four wavefronts per right-hand side; fields padded with zeros to 64 x 64;
// the four 64 x 64 x 64 products on the FP64 matrix cores (layouts as in
// k_dmv_mfma), in FP64 for either field type.
constexpr int DSTN = 64;
template <typename T>
__global__ __launch_bounds__(256) void k_dst_solve(Grid g, const double* __restrict__ S,
                                                   const double* __restrict__ inv, const T* __restrict__ f, long sf,
                                                   T* __restrict__ x, long sx) {
    __shared__ double Sl[DSTN][DSTN + 1];
    __shared__ double Ba[DSTN][DSTN + 1];
    __shared__ double Bb[DSTN][DSTN + 1];
    const int r = blockIdx.x, tid = threadIdx.x, m = g.m;
    const T* fr = f + (long)r * sf;
    const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    {
        // every load of the thread in flight at once, then the LDS stores
        constexpr int E = DSTN * DSTN / 256;
        double sv[E], fv[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int e = tid + 256 * u, a = e / DSTN, b = e % DSTN;  // row a: node row a + 1; column b: column b + 1
            sv[u] = S[e];
            const bool in = a < m && b < m;
            const T v = fr[g.idx(in ? b + 1 : 1, in ? a + 1 : 1)];
            fv[u] = in ? (double)v : 0.0;
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int e = tid + 256 * u, a = e / DSTN, b = e % DSTN;
            Sl[a][b] = sv[u];
            Ba[a][b] = fv[u];
        }
    }
    // the eigenvalue factors of this thread's outputs of the scaled product
    double iv[4][4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = w + 4 * s4, ti = t >> 2, tj = t & 3;
            iv[s4][j] = inv[(16 * ti + 4 * j + lk) * DSTN + 16 * tj + lr];
        }
    __syncthreads();
    // Out = Lm * Rm; wavefront w owns the 16 x 16 output tiles w, w + 4, w + 8, w + 12
    auto gemm = [&](const double (*Lm)[DSTN + 1], const double (*Rm)[DSTN + 1], auto&& emit) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int t = w + 4 * s4, ti = t >> 2, tj = t & 3;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < DSTN / 4; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Lm[16 * ti + lr][4 * ks + lk], Rm[4 * ks + lk][16 * tj + lr],
                                                           acc, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) emit(s4, j, 16 * ti + 4 * j + lk, 16 * tj + lr, acc[j]);
        }
    };
    gemm(Sl, Ba, [&](int, int, int i, int j, double v) { Bb[i][j] = v; });  // S r
    __syncthreads();
    gemm(Bb, Sl, [&](int s4, int jj, int i, int j, double v) { Ba[i][j] = v * iv[s4][jj]; });  // (S r S) ./ eigenvalues
    __syncthreads();
    gemm(Sl, Ba, [&](int, int, int i, int j, double v) { Bb[i][j] = v; });  // S y
    __syncthreads();
    T* xr = x + (long)r * sx;
    gemm(Bb, Sl, [&](int, int, int i, int j, double v) {
        if (i < m && j < m) xr[g.idx(j + 1, i + 1)] = (T)v;
    });
}

}  // namespace

constexpr int kDmvBigN = 2048;  // coarse spaces from this size take the large shape

inline int dmv_chunk(int N) { return N >= kDmvBigN ? 128 : 64; }

template <typename T, int WAVES, int DC>
void dmv_part_launch(int kb, const T* Mat, int N, const Grid& g, const T* x, long sx, bool x_padded, T* part,
                     int nrhs, int kpm, long mstride, hipStream_t st) {
    const int nchunk = (N + DC - 1) / DC;
    const int zb = (kpm + kb - 1) / kb;
    dim3 grid((N + 64 * WAVES - 1) / (64 * WAVES), nchunk, (nrhs / kpm) * zb);
    dim3 blk(64 * WAVES);
#define PASM_DMV(KB)                                                                                            \
    case KB:                                                                                                    \
        hipLaunchKernelGGL((k_dmv_part<T, KB, WAVES, DC>), grid, blk, 0, st, Mat, N, g, x, sx, (int)x_padded,   \
                           part, nrhs, kpm, mstride);                                                           \
        break;
    switch (kb) {
        PASM_DMV(4) PASM_DMV(8) PASM_DMV(12) PASM_DMV(16) PASM_DMV(20) PASM_DMV(24) PASM_DMV(28) PASM_DMV(32)
        PASM_DMV(36) PASM_DMV(40) PASM_DMV(44) PASM_DMV(48)
        default: throw Error(PASM_E_INVALID, "dense products: bad block width");
    }
#undef PASM_DMV
    PASM_CHECK_LAUNCH();
}

// Restart of the iteration.  With unit coefficients y_r = e_j (j = r mod kpm)
// the coarse vector Q y_r is column j of Q itself, so it is gathered (the
// value the dense product gives, without streaming the whole of Q); the same
// launch sets the unit coefficients and lambda = lambda_prev = theta_j.
__global__ __launch_bounds__(256) void k_restart_coarse(const double* __restrict__ Mat, int N, Grid g,
                                                        double* __restrict__ y, long sy, double* __restrict__ ycoef,
                                                        int kpm, long mstride, const double* __restrict__ theta,
                                                        long tstride, double* __restrict__ lam,
                                                        double* __restrict__ lam_prev) {
    const int row = blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
    const int mem = r / kpm, j = r % kpm;
    if (row < N) {
        ycoef[(long)r * N + row] = row == j ? 1.0 : 0.0;
        y[(long)r * sy + compact_to_padded(g, row)] = Mat[(long)mem * mstride + (long)j * N + row];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double t = theta[(long)mem * tstride + j];
        lam[r] = t;
        lam_prev[r] = t;
    }
}

void launch_restart_coarse(const double* Mat, int N, const Grid& g, double* y, long sy, double* ycoef, int nrhs,
                           int kpm, long mstride, const double* theta, long tstride, double* lam, double* lam_prev,
                           hipStream_t st) {
    if (nrhs <= 0 || kpm <= 0 || nrhs % kpm != 0 || kpm > N)
        throw Error(PASM_E_INVALID, "restart: right-hand sides not a multiple per member");
    hipLaunchKernelGGL(k_restart_coarse, dim3((N + 255) / 256, nrhs), dim3(256), 0, st, Mat, N, g, y, sy, ycoef, kpm,
                       mstride, theta, tstride, lam, lam_prev);
    PASM_CHECK_LAUNCH();
}

template <typename T>
void launch_dense_mv(const T* Mat, int N, const Grid& g, const T* x, long sx, bool x_padded, T* y, long sy,
                     bool y_padded, int nrhs, void* work, hipStream_t st, int kpm, long mstride) {
    if (kpm <= 0) kpm = nrhs;
    if (nrhs % kpm != 0) throw Error(PASM_E_INVALID, "dense products: right-hand sides not a multiple per member");
    if constexpr (std::is_same<T, double>::value) {
        if (N >= kDmvBigN) {
            // large coarse spaces: matrix-core products, 128-column chunks
            constexpr int DC = 128;
            const int nchunk = (N + DC - 1) / DC;
            const int nt = std::min(3, (kpm + 15) / 16);
            const int zb = (kpm + 16 * nt - 1) / (16 * nt);
            dim3 grid((N + 64 * DMW - 1) / (64 * DMW), nchunk, (nrhs / kpm) * zb), blk(64 * DMW);
            double* part = static_cast<double*>(work);
            switch (nt) {
                case 1: hipLaunchKernelGGL((k_dmv_mfma<1, DC>), grid, blk, 0, st, Mat, N, g, x, sx, (int)x_padded, part, nrhs, kpm, mstride); break;
                case 2: hipLaunchKernelGGL((k_dmv_mfma<2, DC>), grid, blk, 0, st, Mat, N, g, x, sx, (int)x_padded, part, nrhs, kpm, mstride); break;
                default: hipLaunchKernelGGL((k_dmv_mfma<3, DC>), grid, blk, 0, st, Mat, N, g, x, sx, (int)x_padded, part, nrhs, kpm, mstride); break;
            }
            PASM_CHECK_LAUNCH();
            const long tot = (long)N * nrhs;
            hipLaunchKernelGGL(k_dmv_sum_rm, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, N, nchunk, part, nrhs,
                               g, y, sy, (int)y_padded);
            PASM_CHECK_LAUNCH();
            return;
        }
    }
    const int kb = std::min(48, (kpm + 3) / 4 * 4);
    const int DC = dmv_chunk(N);
    const int nchunk = (N + DC - 1) / DC;
    T* part = static_cast<T*>(work);
    if (N >= kDmvBigN)
        dmv_part_launch<T, 4, 128>(kb, Mat, N, g, x, sx, x_padded, part, nrhs, kpm, mstride, st);
    else
        dmv_part_launch<T, 1, 64>(kb, Mat, N, g, x, sx, x_padded, part, nrhs, kpm, mstride, st);
    hipLaunchKernelGGL((k_dmv_sum<T>), dim3((N + 255) / 256, nrhs), dim3(256), 0, st, N, nchunk, part, nrhs, g, y, sy,
                       (int)y_padded);
    PASM_CHECK_LAUNCH();
}
template void launch_dense_mv<double>(const double*, int, const Grid&, const double*, long, bool, double*, long,
                                      bool, int, void*, hipStream_t, int, long);
template void launch_dense_mv<float>(const float*, int, const Grid&, const float*, long, bool, float*, long, bool,
                                     int, void*, hipStream_t, int, long);

bool dst_solve_supported(const Grid& g) { return g.dim == 2 && g.n >= 2 && g.n <= DSTN; }

void dst_solve_tables(const Grid& g, double w0, std::vector<double>& S, std::vector<double>& inv) {
    const int n = g.n, m = g.m;
    const double pi = 3.14159265358979323846;
    S.assign((size_t)DSTN * DSTN, 0.0);
    inv.assign((size_t)DSTN * DSTN, 0.0);
    std::vector<double> c(m);
    for (int a = 0; a < m; ++a) c[a] = 2.0 - 2.0 * std::cos(pi * (a + 1) / n);
    const double sc = std::sqrt(2.0 / n);
    for (int a = 0; a < m; ++a)
        for (int j = 0; j < m; ++j) {
            // sin of pi (a+1)(j+1)/n with the argument reduced modulo 2n exactly
            const long q = ((long)(a + 1) * (j + 1)) % (2 * n);
            S[(size_t)a * DSTN + j] = sc * std::sin(pi * (double)q / n);
            inv[(size_t)a * DSTN + j] = 1.0 / (w0 * (c[a] + c[j]));
        }
}

template <typename T>
void launch_dst_solve(const Grid& g, const double* S, const double* inv, const T* f, long sf, T* x, long sx,
                      int nrhs, hipStream_t st) {
    if (!dst_solve_supported(g)) throw Error(PASM_E_INVALID, "sine-transform coarse solve: 2D, at most 64 cells");
    hipLaunchKernelGGL((k_dst_solve<T>), dim3(nrhs), dim3(256), 0, st, g, S, inv, f, sf, x, sx);
    PASM_CHECK_LAUNCH();
}
template void launch_dst_solve<double>(const Grid&, const double*, const double*, const double*, long, double*, long,
                                       int, hipStream_t);
template void launch_dst_solve<float>(const Grid&, const double*, const double*, const float*, long, float*, long,
                                      int, hipStream_t);

size_t dense_mv_workspace_bytes(int N, int nrhs) {
    return sizeof(double) * (size_t)((N + 63) / 64) * nrhs * N;
}

long arrow_work_doubles(int N, int k) { return ws_doubles(N) * (long)k; }
int arrow_chunks(int N) { return (N + 1 + RPB - 1) / RPB; }

void launch_arrowhead(const ArrowIn& in0, const ArrowOut& out, int k, hipStream_t st) {
    ArrowIn in = in0;
    if (in.kpm <= 0) in.kpm = k;
    const int nchunk = arrow_chunks(in.N);
    double* work = out.work;
    int* iwork = reinterpret_cast<int*>(work + arrow_work_doubles(in.N, k));
    double* best = reinterpret_cast<double*>(iwork + (long)in.N * k + ((long)in.N * k & 1));
    if (in.N <= PMAXN)
        hipLaunchKernelGGL(k_arrow_prep<true>, dim3(k), dim3(PP), 0, st, in, work, iwork, best, nchunk);
    else
        hipLaunchKernelGGL(k_arrow_prep<false>, dim3(k), dim3(PP), 0, st, in, work, iwork, best, nchunk);
    PASM_CHECK_LAUNCH();
    // NEAR pass: one workgroup per (eigenpair, root) with the poles in
    // registers up to 8192 of them, else one workgroup per eigenpair and one
    // wavefront per root
    double* nres = best + 4L * nchunk * k;
    auto near = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(k, RPB), dim3(NT), 0, st, in, work, iwork, best, nchunk, nres);
        PASM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_arrow_near_cert, dim3(k), dim3(64), 0, st, in, work, iwork, best, nchunk,
                           (const double*)nres);
    };
    if (in.N <= 4 * NT) near(k_arrow_near_root<4>);
    else if (in.N <= 8 * NT) near(k_arrow_near_root<8>);
    else if (in.N <= 16 * NT) near(k_arrow_near_root<16>);
    else if (in.N <= 32 * NT) near(k_arrow_near_root<32>);
    else if (in.N <= LDS_POLES_BIG)
        hipLaunchKernelGGL((k_arrow_roots<LDS_POLES_BIG, true, RPB>), dim3(k, 1), dim3(RW * RPB), 0, st, in, work,
                           iwork, best, nchunk);
    else
        hipLaunchKernelGGL((k_arrow_roots<0, true, RPB>), dim3(k, 1), dim3(RW * RPB), 0, st, in, work, iwork, best,
                           nchunk);
    // full pass (its workgroups return at once when the NEAR pass certified
    // its winner); many workgroups per eigenpair, so the smaller LDS copy
    if (in.N <= LDS_POLES)
        hipLaunchKernelGGL((k_arrow_roots<LDS_POLES, false>), dim3(k, nchunk), dim3(RW * RWAVES), 0, st, in, work,
                           iwork, best, nchunk);
    else
        hipLaunchKernelGGL((k_arrow_roots<0, false>), dim3(k, nchunk), dim3(RW * RWAVES), 0, st, in, work, iwork,
                           best, nchunk);
    PASM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_arrow_final, dim3(k), dim3(PF_T), 0, st, in, out, work, iwork, best, nchunk);
    PASM_CHECK_LAUNCH();
}

size_t arrow_workspace_bytes(int N, int k) {
    const int nchunk = arrow_chunks(N);
    return sizeof(double) * (size_t)arrow_work_doubles(N, k) + sizeof(int) * ((size_t)N * k + 2) +
           sizeof(double) * 4 * (size_t)nchunk * k + sizeof(double) * 2 * RPB * (size_t)k + 256;
}

}  // namespace pasm

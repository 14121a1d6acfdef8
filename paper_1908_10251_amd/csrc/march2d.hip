// Smoothing phases of the V-cycle on the 2D mesh as marching, temporally
// blocked sweeps (constant coefficients).
//
// One wavefront owns a strip of 128 columns (two adjacent columns per lane) and
// marches down a segment of rows.  Each lane holds, in registers, a 3-row
// window of every smoothing stage x_0, x_1, ..., x_S of its two columns, plus
// the last S+2 rows of f; the columns of the neighbouring lanes come by DPP
// wavefront shifts, and the next PF rows are loaded ahead.
// When row r is loaded, stage t advances row r - t; stage S therefore emits
// x_S of row r - S.  Every node is read and written once per phase, apart
// from an (S+2)-column halo on each side of a strip and S+2 rows at the ends
// of a segment.  Lanes and rows within t of the loaded region's edge hold
// garbage after t stages; nothing that is stored depends on them.
//
// Fused variants (finest-grid traffic of a V-cycle drops from ~15 to ~6.5
// words per node):
//   PRE   after the S steps, the residual r = f - A x_S and its restriction
//         r_c = P^T r to the next coarser grid (the transpose of nodal
//         interpolation: centre 1, the six neighbours of the "/" mesh 1/2);
//   POST  the coarse correction is prolongated while loading:
//         x_0 = x + P e_c;
//   POST with borders (double): as POST, then from u = x_S also A u and
//         M u, their restrictions b_c = P^T A u and c_c = P^T M u, and the
//         sums u.Au, u.Mu over the wavefront's own nodes (one pair per
//         wavefront), which the augmented pencil needs next.
// Steps follow x_{t+1} = x_t + a_t (x_t - x_{t-1}) + b_t D^{-1} (f - A x_t)
// with a_0 = 0 (a phase starts fresh).
//
// Levels with edge weights (per-element kappa, FP32 cycles) march in
// k_march_ew below: PRE and POST as above, two right-hand sides per
// wavefront sharing the weights.
#include <algorithm>

#include "common.h"

namespace pasm {

namespace {

constexpr int NL = 64;      // lanes per wavefront
constexpr int MW = 2 * NL;  // strip width: each lane owns two adjacent columns
constexpr int XCDS = 8;     // accelerator dies; workgroup w runs on die w % 8
// Rows loaded ahead of the one being processed.  The loop over rows is
// unrolled by PF so that every prefetch slot is a fixed set of registers: a
// slot is consumed and refilled in the same unrolled body, and the only wait
// is for the oldest row in flight (rotating a register queue instead would
// make the compiler wait for every outstanding load).
template <typename T>
constexpr int prefetch_rows() { return sizeof(T) == 8 ? 3 : 6; }
constexpr int gcd_(int a, int b) { return b == 0 ? a : gcd_(b, a % b); }
constexpr int lcm_(int a, int b) { return a / gcd_(a, b) * b; }
constexpr int march_unroll(int S, int PF) { return lcm_(lcm_(3, S + 2), PF); }
// Columns of halo on each side of a strip: S + 2 (S smoothing steps, then the
// residual and its restriction one node further each), rounded up to even so
// that every lane's first column, the centre of a restriction, is even.
constexpr int march_halo(int S) { return (S + 3) & ~1; }

// Cross-lane moves by one lane (DPP wave shifts).  The lane at the wavefront
// edge has no source and receives 0 (bound control), which only ever reaches
// halo columns; with no old value to merge, no register has to be zeroed first.
__device__ inline double from_left(double v) {  // value of lane l - 1
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ inline double from_right(double v) {  // value of lane l + 1
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ inline float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ inline float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}

// A register copy the compiler cannot fold away: the copy, not the loaded
// register, lives on in the row windows.
__device__ inline double detach(double v) {
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ inline float detach(float v) {
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Waits until every vector memory access of the wavefront has completed
// (s_waitcnt vmcnt(0), the other counters left at their maximum).  Issued once
// after the prologue's loads: the loop header then joins the back edge with
// an empty state, so its wait is for the oldest row in flight only; without
// it the header waits for every outstanding access once per unrolled body,
// because the prologue leaves the first rows in other registers.
__device__ inline void drain_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Fused multiply-add in the type of the operands.
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1 / d for the diagonal of an edge-weight row (positive, normal): the
// hardware reciprocal refined by one Newton step (within an ulp of the
// quotient, without the division's scaling and fix-up).
__device__ inline float recip(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return __builtin_fmaf(r, __builtin_fmaf(-d, r, 1.0f), r);
}
__device__ inline double recip(double d) { return 1.0 / d; }

// MODE 5: the coarse-space field q (padded level, ratio 2^lr to the fine grid)
// that the first pre-smoothing interpolates, with the weights beta of the old
// field and the eigenvalues lam of the right-hand side f = lam M x_0 it forms.
struct ProlongSrc {
    Grid gq;
    const double* q;
    long sq;
    int lr;
    const double* beta;
    const double* lam;
    double* fout;
};

// The level's edge weights (per-element kappa): wx at node (i, j) is the
// weight of the edge to (i + 1, j), wy the weight of the edge to (i, j + 1);
// A x = sum over the four edges of w (x - x_neighbour), D = sum of the four.
// GEN (a potential term: the general 7-point operator of the "/" mesh):
// (A x)_(i,j) = d x - the four edge terms - wne(i,j) x(i+1,j+1)
// - wne(i-1,j-1) x(i-1,j-1), with the diagonal d given.  Batches: the planes
// of right-hand side z belong to member z / kpm, ms elements apart, whose
// smoothing steps b are scaled by bsc[member].
template <typename T>
struct EdgeW {
    const T* wx;
    const T* wy;
    const T* d = nullptr;
    const T* wne = nullptr;
    long ms = 0;
    int kpm = 1;
    const T* bsc = nullptr;
};

template <typename T, int S, int MODE, bool XZ>
__global__ __launch_bounds__(NL) __attribute__((amdgpu_waves_per_eu(2))) void k_march(Grid g, T w0, const T* __restrict__ x0, const T* __restrict__ f,
                                              T* __restrict__ out, const T* __restrict__ ec, Grid gc,
                                              T* __restrict__ rc, T* __restrict__ rc2, double* __restrict__ part,
                                              long sf, long sc, SmoothSteps st, MarchShape sh, ProlongSrc ps) {
    // MODE 4: the post-smoothing of one V-cycle and the pre-smoothing of the
    // next in one pass (S = post + pre stages; the host zeroes the momentum
    // coefficient of the first pre-smoothing stage)
    constexpr bool POSTLIKE = MODE == 2 || MODE == 3 || MODE == 4;
    // MODE 5: pre-smoothing whose x_0 = P q + beta u (P1 interpolation on the
    // coarse "/" triangles) and whose right-hand side f = lam M x_0 are formed
    // in the pass (f is also written out): the prolongation of the previous
    // correction step and this step's first pre-smoothing in one pass
    constexpr bool PROLONG = MODE == 5;
    static_assert(!PROLONG || sizeof(T) == 8, "the prolonging pass is FP64");
    constexpr int PF = prefetch_rows<T>();
    constexpr int HX = march_halo(S);
    constexpr int TXO = MW - 2 * HX;
    // One wavefront per workgroup.  Consecutive pieces of work (strips of a
    // band of rows, then the next band, then the next right-hand side) go to
    // the same die, so the halos that neighbouring strips and bands share are
    // found in that die's L2.
    const int per = sh.blocks / XCDS;
    const int work = (blockIdx.x % XCDS) * per + blockIdx.x / XCDS;
    if (work >= sh.work) return;  // uniform per wavefront
    const int strip = work % sh.strips;
    const int band = (work / sh.strips) % sh.segs;
    const int z = work / (sh.strips * sh.segs);
    const int MSEG = sh.mseg;
    const int lane = threadIdx.x;
    // Odd bands run point-reflected: kernel position (i, r) is grid node
    // (n - i, n - r), coarse (I, J) is (nc - I, nc - J).  The operator, the
    // mass matrix and both transfers of the "/" mesh are symmetric under that
    // reflection, so the arithmetic is unchanged; each band boundary is then
    // reached by both neighbouring bands at the same time (both start there or
    // both end there), and the rows they share come from HBM once and from the
    // die's L2 the second time.
    const bool flip = band & 1;
    const int y0 = flip ? g.n + 1 - (band + 1) * MSEG : band * MSEG;
    const int fs = flip ? -1 : 1;
    auto gx = [&](int i) { return flip ? g.n - i : i; };
    auto gcx = [&](int I) { return flip ? gc.n - I : I; };
    const int c0 = 2 * lane;                      // strip column of the lane's first column
    const int i0 = strip * TXO - HX + c0;         // global column (even)
    bool inner[2], owned[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        inner[cc] = (i0 + cc) >= 1 && (i0 + cc) <= g.m;
        owned[cc] = (c0 + cc) >= HX && (c0 + cc) < MW - HX;
    }
    const long off = (long)z * sf;
    const T* xr = x0 + off;
    const T* fr = f + off;
    T* outr = out + off;
    const T* ecr = ec + (long)z * sc;
    double bz = 0.0, lz = 0.0;
    const double* qr = nullptr;
    double* fo = nullptr;
    if constexpr (PROLONG) {
        bz = ps.beta[z];
        lz = ps.lam[z];
        qr = ps.q + (long)z * ps.sq;
        fo = ps.fout + off;
    }
    const int PR = 1 << ps.lr;
    const double invPR = 1.0 / PR;
    const double h2 = g.h * g.h;
    const T invD = T(1) / (T(4) * w0);
    // MODE 4: the steps come scaled by 1 / D from the host, the stages form
    // x + b' (f - A x) with masks; the one-phase modes form
    // x + b ((f + w0 sum x_nb) / D - x) with 1 / D = 0 on boundary and outside
    // nodes (a row outside the grid selects 0 for the whole row, a column
    // outside has 0 in cdl), where x then stays at the loaded 0 and needs no
    // mask
    T bs[S], as[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        bs[t] = (T)st.b[t];
        as[t] = (T)st.a[t];
    }
    const T cdl[2] = {inner[0] ? invD : T(0), inner[1] ? invD : T(0)};

    T xw[S + 1][3][2];
    T fw[S + 2][2];
    T rw[3][2];
    T mw[3][2];  // MODE 3: rw holds A u, mw holds M u
    double ua = 0.0, um = 0.0;
#pragma unroll
    for (int t = 0; t <= S; ++t)
#pragma unroll
        for (int k = 0; k < 3; ++k) xw[t][k][0] = xw[t][k][1] = T(0);
#pragma unroll
    for (int j = 0; j < S + 2; ++j) fw[j][0] = fw[j][1] = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) rw[k][0] = rw[k][1] = mw[k][0] = mw[k][1] = T(0);

    const int r_begin = y0 - 2 - S;
    // the restriction centred on the band's last row (even in a reflected
    // band) is formed one row after x_S of the row below it
    const int r_end = y0 + MSEG + S + 1;

    // Loads are branch-free so that rows requested PF steps ahead stay in
    // flight: positions outside the grid are clamped onto the boundary ring,
    // whose stored values are zero (the Dirichlet data), which is exactly the
    // value such positions must have.
    const int ia = min(max(i0, 0), g.n), ib = min(max(i0 + 1, 0), g.n);
    const int ga = gx(ia), gb = gx(ib);  // their grid columns
    // One prefetched row: the raw loaded values, combined only when the row
    // is consumed, PF rows later (combining at load time would wait for the
    // loads at once).  POST reads the two coarse nodes whose mean is the
    // nodal interpolation of the coarse correction at the fine node: coarse
    // (I, J) and (I + a, J + b), a = i & 1, b = r & 1; for a = b = 0 both
    // reads are the same node and the mean is exact, so there is no branch.
    struct Slot {
        T x[2], f[2], e0[2], e1[2];
        T q[2][3];  // MODE 5: the three coarse nodes of the triangle under each column
    };
    auto load = [&](int r, Slot& sl) {
        const int rr = min(max(r, 0), g.n);
        const long row = (long)gx(rr) * g.pitch + ORIGIN;
        if constexpr (PROLONG) {
            // the old field (used when its weight is nonzero) and the corners
            // (I, J), (I + 1, J) or (I, J + 1), (I + 1, J + 1) of the coarse
            // triangle, indices clamped onto the last coarse line where their
            // weights are zero
            sl.x[0] = xr[row + ga];
            sl.x[1] = xr[row + gb];
            const int gj = gx(rr), J = gj >> ps.lr, b = gj & (PR - 1), J1 = min(J + 1, ps.gq.n);
            const int gcol[2] = {ga, gb};
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const int gi = gcol[cc], I = gi >> ps.lr, a = gi & (PR - 1), I1 = min(I + 1, ps.gq.n);
                sl.q[cc][0] = qr[ps.gq.idx(I, J)];
                sl.q[cc][1] = a >= b ? qr[ps.gq.idx(I1, J)] : qr[ps.gq.idx(I, J1)];
                sl.q[cc][2] = qr[ps.gq.idx(I1, J1)];
            }
            return;
        }
        sl.f[0] = fr[row + ga];
        sl.f[1] = fr[row + gb];
        if (POSTLIKE || !XZ) {
            sl.x[0] = xr[row + ga];
            sl.x[1] = xr[row + gb];
        }
        if (POSTLIKE) {
            const int cols[2] = {ia, ib};
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const int i = cols[cc], a = i & 1, b = rr & 1;
                const long cid = gc.idx(gcx(i >> 1), gcx(rr >> 1));
                sl.e0[cc] = ecr[cid];
                sl.e1[cc] = ecr[cid + fs * (a + (long)b * gc.pitch)];
            }
        }
    };

    // Row r enters the windows of x_0 and f.  The window registers are fresh
    // copies, so the slot's registers are free for the next load at once.
    auto shift_in = [&](const Slot& sl, const int r) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            T cx;
            if constexpr (PROLONG) {
                // P1 weights (R - wa, wa - wb, wb) / R in the grid's own
                // coordinates, as the stand-alone prolongation computes them
                const int rr = min(max(r, 0), g.n);
                const int b = gx(rr) & (PR - 1), a = (cc ? gb : ga) & (PR - 1);
                const int wa = a >= b ? a : b, wb = a >= b ? b : a;
                double v = __builtin_fma((double)wb, sl.q[cc][2],
                                         __builtin_fma((double)(wa - wb), sl.q[cc][1], (double)(PR - wa) * sl.q[cc][0])) *
                           invPR;
                if (bz != 0.0) v = __builtin_fma(bz, sl.x[cc], v);
                cx = (r >= 1 && r <= g.m && inner[cc]) ? v : 0.0;
            } else if (POSTLIKE) {
                cx = sl.x[cc] + T(0.5) * (sl.e0[cc] + sl.e1[cc]);
            } else if (!XZ) {
                cx = detach(sl.x[cc]);
            } else {
                cx = T(0);
            }
#pragma unroll
            for (int j = S + 1; j > 0; --j) fw[j][cc] = fw[j - 1][cc];
            fw[0][cc] = PROLONG ? T(0) : detach(sl.f[cc]);
            xw[0][2][cc] = xw[0][1][cc];
            xw[0][1][cc] = xw[0][0][cc];
            xw[0][0][cc] = cx;
        }
        if constexpr (PROLONG) {
            // f = lam M x_0 at row r - 1 from the x_0 rows (r, r-1, r-2): the
            // six neighbours summed in the grid's order (right, left, up, down,
            // (i+1, j+1), (i-1, j-1)); a reflected band sees each pair swapped
            const int q = r - 1;
            const T m0 = xw[0][1][0], m1 = xw[0][1][1];
            const T up0 = xw[0][0][0], up1 = xw[0][0][1], dn0 = xw[0][2][0], dn1 = xw[0][2][1];
            const T lf[2] = {from_left(m1), m0}, rt[2] = {m1, from_right(m0)};
            const T up[2] = {up0, up1}, dn[2] = {dn0, dn1};
            const T ne[2] = {up1, from_right(up0)}, sw[2] = {from_left(dn1), dn0};
            const T mc[2] = {m0, m1};
            const bool row_in = q >= 1 && q <= g.m;
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const T sn = (flip ? lf[cc] : rt[cc]) + (flip ? rt[cc] : lf[cc]) + (flip ? dn[cc] : up[cc]) +
                             (flip ? up[cc] : dn[cc]) + (flip ? sw[cc] : ne[cc]) + (flip ? ne[cc] : sw[cc]);
                const T fv = lz * (h2 * __builtin_fma(sn, 1.0 / 12.0, 0.5 * mc[cc]));
                fw[1][cc] = (row_in && inner[cc]) ? fv : T(0);
            }
            if (q >= y0 && q < y0 + MSEG && row_in) {
                const long id = g.idx(gx(i0), gx(q));
#pragma unroll
                for (int cc = 0; cc < 2; ++cc)
                    if (owned[cc] && inner[cc]) fo[id + fs * cc] = fw[1][cc];
            }
        }
    };
    // After row r entered: advance every stage by one row, store x_S of row
    // r - S, and (PRE) the residual and its restriction.
    auto advance = [&](const int r) {
#pragma unroll
        for (int t = 1; t <= S; ++t) {
            const int q = r - t;
            const bool row_in = q >= 1 && q <= g.m;  // uniform
            const T m0 = xw[t - 1][1][0], m1 = xw[t - 1][1][1];
            const T left = from_left(m1), right = from_right(m0);
            T v[2];
            const T nb0 = left + m1 + xw[t - 1][0][0] + xw[t - 1][2][0];
            const T nb1 = m0 + right + xw[t - 1][0][1] + xw[t - 1][2][1];
            const T mc[2] = {m0, m1};
            const T nb[2] = {nb0, nb1};
            if constexpr (MODE == 4) {
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    const T Ax = w0 * (T(4) * mc[cc] - nb[cc]);
                    T val = mc[cc] + bs[t - 1] * (fw[t][cc] - Ax);
                    if (t >= 2) val += as[t - 1] * (mc[cc] - xw[t - 2][2][cc]);
                    v[cc] = (row_in && inner[cc]) ? val : T(0);
                }
            } else {
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    const T cd = row_in ? cdl[cc] : T(0);
                    const T sn = fma_t(w0, nb[cc], fw[t][cc]);
                    T val = fma_t(bs[t - 1], fma_t(sn, cd, -mc[cc]), mc[cc]);
                    if (t >= 2) val += as[t - 1] * (mc[cc] - xw[t - 2][2][cc]);
                    v[cc] = val;
                }
            }
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                xw[t][2][cc] = xw[t][1][cc];
                xw[t][1][cc] = xw[t][0][cc];
                xw[t][0][cc] = v[cc];
            }
        }
        {
            const int q = r - S;
            if (q >= y0 && q < y0 + MSEG && q >= 1 && q <= g.m) {
                const long id = g.idx(gx(i0), gx(q));
#pragma unroll
                for (int cc = 0; cc < 2; ++cc)
                    if (owned[cc] && inner[cc]) outr[id + fs * cc] = xw[S][0][cc];
            }
        }
        if (MODE == 1 || MODE == 4 || MODE == 5) {
            // residual at row r - S - 1 from x_S rows (r-S, r-S-1, r-S-2)
            const int q1 = r - S - 1;
            const bool row_in = q1 >= 1 && q1 <= g.m;
            const T m0 = xw[S][1][0], m1 = xw[S][1][1];
            const T left = from_left(m1), right = from_right(m0);
            const T nb0 = left + m1 + xw[S][0][0] + xw[S][2][0];
            const T nb1 = m0 + right + xw[S][0][1] + xw[S][2][1];
            T res0, res1;
            {
                res0 = fw[S + 1][0] - w0 * (T(4) * m0 - nb0);
                res1 = fw[S + 1][1] - w0 * (T(4) * m1 - nb1);
            }
            // (an interior coarse node's seven fine nodes are interior: the
            // residuals of other nodes, finite, reach no stored value)
            if constexpr (MODE == 4) {
                res0 = (row_in && inner[0]) ? res0 : T(0);
                res1 = (row_in && inner[1]) ? res1 : T(0);
            }
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                rw[2][cc] = rw[1][cc];
                rw[1][cc] = rw[0][cc];
            }
            rw[0][0] = res0;
            rw[0][1] = res1;
            // restriction to the coarse node centred at (i0, r - S - 2), i0 even
            const int q2 = r - S - 2;
            const T mid_left = from_left(rw[1][1]);   // (i0-1, q2)
            const T dn_left = from_left(rw[2][1]);    // (i0-1, q2-1)
            if (((q2 & 1) == 0) && q2 >= y0 && q2 < y0 + MSEG && owned[0]) {
                const int I = i0 >> 1, J = q2 >> 1;
                if (I >= 1 && I <= gc.m && J >= 1 && J <= gc.m)
                    rc[(long)z * sc + gc.idx(gcx(I), gcx(J))] =
                        rw[1][0] + T(0.5) * (rw[1][1] + mid_left + rw[0][0] + rw[2][0] + rw[0][1] + dn_left);
            }
        }
        if (MODE == 3) {
            // A u and M u at row r - S - 1 from u = x_S rows (r-S, r-S-1, r-S-2)
            const int q1 = r - S - 1;
            const T m0 = xw[S][1][0], m1 = xw[S][1][1];
            const T left = from_left(m1), right = from_right(m0);
            const T up0 = xw[S][0][0], up1 = xw[S][0][1], dn0 = xw[S][2][0], dn1 = xw[S][2][1];
            const T nb0 = left + m1 + up0 + dn0;
            const T nb1 = m0 + right + up1 + dn1;
            // the "/" diagonal: (i + 1, q1 + 1) and (i - 1, q1 - 1)
            const T ne0 = up1, ne1 = from_right(up0);
            const T sw0 = from_left(dn1), sw1 = dn0;
            const T h2 = T(g.h * g.h);
            T a0 = w0 * (T(4) * m0 - nb0), a1 = w0 * (T(4) * m1 - nb1);
            T b0 = h2 * (T(0.5) * m0 + (nb0 + ne0 + sw0) * T(1.0 / 12.0));
            T b1 = h2 * (T(0.5) * m1 + (nb1 + ne1 + sw1) * T(1.0 / 12.0));
            // no masks: u = 0 off the interior, so those nodes add nothing to
            // the sums, and the restrictions to interior coarse nodes read
            // interior fine nodes only
            if (q1 >= y0 && q1 < y0 + MSEG) {  // this wavefront's own rows (and columns) for the sums
                if (owned[0]) {
                    ua += (double)(m0 * a0);
                    um += (double)(m0 * b0);
                }
                if (owned[1]) {
                    ua += (double)(m1 * a1);
                    um += (double)(m1 * b1);
                }
            }
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                rw[2][cc] = rw[1][cc];
                rw[1][cc] = rw[0][cc];
                mw[2][cc] = mw[1][cc];
                mw[1][cc] = mw[0][cc];
            }
            rw[0][0] = a0;
            rw[0][1] = a1;
            mw[0][0] = b0;
            mw[0][1] = b1;
            const int q2 = r - S - 2;
            const T ra = from_left(rw[1][1]), rb = from_left(rw[2][1]);
            const T ma = from_left(mw[1][1]), mb = from_left(mw[2][1]);
            if (((q2 & 1) == 0) && q2 >= y0 && q2 < y0 + MSEG && owned[0]) {
                const int I = i0 >> 1, J = q2 >> 1;
                if (I >= 1 && I <= gc.m && J >= 1 && J <= gc.m) {
                    const long cid = (long)z * sc + gc.idx(gcx(I), gcx(J));
                    rc[cid] = rw[1][0] + T(0.5) * (rw[1][1] + ra + rw[0][0] + rw[2][0] + rw[0][1] + rb);
                    rc2[cid] = mw[1][0] + T(0.5) * (mw[1][1] + ma + mw[0][0] + mw[2][0] + mw[0][1] + mb);
                }
            }
        }
    };

    Slot q[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) load(r_begin + p, q[p]);
    drain_vmem();
    // The loop body covers UNR rows, a multiple of PF and of the periods of
    // the rotating row windows (3 rows of x, S + 2 rows of f), so that after
    // unrolling every window and slot is back in its own registers at the
    // back edge.  Rows past r_end (at most UNR - 1) only feed halo stages:
    // nothing stored depends on them.
    // (MODE 4's f window of S + 2 rows is left out of the period: its
    // registers are moved once per body instead of unrolling 30 rows.)
    constexpr int UNR = MODE == 4 ? lcm_(3, PF) : march_unroll(S, PF);
    const int iters = (r_end - r_begin + UNR) / UNR;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            // the slot is refilled as soon as its row is in the windows
            const int r = r_begin + it * UNR + u;
            shift_in(q[u % PF], r);
            load(r + PF, q[u % PF]);
            advance(r);
        }
    }
    if (MODE == 3) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            ua += __shfl_xor(ua, o, 64);
            um += __shfl_xor(um, o, 64);
        }
        if (lane == 0) {
            const long b = (long)z * (sh.strips * sh.segs) + (long)band * sh.strips + strip;
            part[2 * b] = ua;
            part[2 * b + 1] = um;
        }
    }
}

// ---------------------------------------------------------------------------
// Edge-weight marching (per-element kappa, FP32 cycles) over NR right-hand
// sides per wavefront.  The same marching order, windows and arithmetic as
// k_march's edge-weight phases (PRE: S steps from x_0, residual, restriction;
// POST: x_0 = x + P e_c, S steps), but a wavefront carries NR right-hand
// sides of one strip and band together, so the two weight planes and 1/D are
// read and formed once for all of them: the weights are as many bytes per node
// as an FP32 vector pair, and reading them once per right-hand side made them
// half of the launch's traffic.
//
// Loads and stores are raw buffer accesses over the NR right-hand sides'
// blocks: each lane's column offsets are fixed for the whole march, a row's
// offset and a right-hand side's block offset are uniform scalar offsets, so
// no lane forms a 64-bit address per row.  Accesses of a right-hand side past
// the last one (a ragged last group) fall outside the resource: loads return
// 0, stores are dropped.  Stores that must not happen (halo columns, rows of
// other bands) take an offset past the end of the resource instead of a
// branch.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRawBufferWord3 = 0x00020000;  // 32-bit data format, raw (stride 0) addressing
constexpr unsigned kDropped = 0x80000000u;   // out of range of every resource below (blocks < 2 GiB)
__device__ inline rsrc_t make_rsrc(const void* p, long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kRawBufferWord3);
}
__device__ inline float bload(rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ inline void bstore(float v, rsrc_t r, unsigned vo) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, 0, 0);
}

template <int S, int PF>
constexpr int ew_unroll() { return lcm_(lcm_(3, S + 2), PF); }

template <int S, int MODE, bool XZ, int NR, bool GEN>
__global__ __launch_bounds__(NL) __attribute__((amdgpu_waves_per_eu(2))) void k_march_ew(
    Grid g, const float* __restrict__ x0, const float* __restrict__ f, float* __restrict__ out,
    const float* __restrict__ ec, Grid gc, float* __restrict__ rc, long sf, long sc, SmoothSteps st, MarchShape sh,
    EdgeW<float> ew) {
    static_assert(MODE == 1 || MODE == 2, "edge-weight marching: PRE and POST phases");
    using T = float;
    constexpr bool POST = MODE == 2;
    constexpr int PF = 6 / NR > 2 ? 6 / NR : 3;  // rows in flight
    constexpr int HX = march_halo(S);
    constexpr int TXO = MW - 2 * HX;
    const int per = sh.blocks / XCDS;
    const int work = (blockIdx.x % XCDS) * per + blockIdx.x / XCDS;
    if (work >= sh.work) return;  // uniform per wavefront
    const int strip = work % sh.strips;
    const int band = (work / sh.strips) % sh.segs;
    const int z0 = (work / (sh.strips * sh.segs)) * NR;
    const int nv = min(NR, sh.nrhs - z0);
    const int MSEG = sh.mseg;
    const int lane = threadIdx.x;
    // odd bands point-reflected, as in k_march
    const bool flip = band & 1;
    const int y0 = flip ? g.n + 1 - (band + 1) * MSEG : band * MSEG;
    const int fs = flip ? -1 : 1;
    auto gx = [&](int i) { return flip ? g.n - i : i; };
    auto gcx = [&](int I) { return flip ? gc.n - I : I; };
    const int c0 = 2 * lane;
    const int i0 = strip * TXO - HX + c0;  // global column (even)
    bool inner[2], owned[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        inner[cc] = (i0 + cc) >= 1 && (i0 + cc) <= g.m;
        owned[cc] = (c0 + cc) >= HX && (c0 + cc) < MW - HX;
    }
    // resources over the group's right-hand sides (blocks of sf words; the
    // coarse blocks of sc words) and the two weight planes
    const unsigned pb = (unsigned)(sf * 4), cb = (unsigned)(sc * 4);
    const rsrc_t xs = make_rsrc((POST || !XZ) ? x0 + (long)z0 * sf : f, (long)nv * pb);
    const rsrc_t fsr = make_rsrc(f + (long)z0 * sf, (long)nv * pb);
    const rsrc_t os = make_rsrc(out + (long)z0 * sf, (long)nv * pb);
    const rsrc_t es = make_rsrc(POST ? ec + (long)z0 * sc : f, POST ? (long)nv * cb : 0);
    const rsrc_t rs = make_rsrc(POST ? out : rc + (long)z0 * sc, POST ? 0 : (long)nv * cb);
    // the coefficient planes of the group's member (every group lies within
    // one member: NR divides the right-hand sides per member)
    const int mem = z0 / ew.kpm;
    const long wo = (long)mem * ew.ms;
    const rsrc_t wxs = make_rsrc(ew.wx + wo, (long)sf * 4), wys = make_rsrc(ew.wy + wo, (long)sf * 4);
    const rsrc_t dds = make_rsrc(GEN ? ew.d + wo : ew.wx, GEN ? (long)sf * 4 : 0);
    const rsrc_t nes = make_rsrc(GEN ? ew.wne + wo : ew.wx, GEN ? (long)sf * 4 : 0);
    const T bsm = ew.bsc ? ew.bsc[mem] : T(1);

    T bs[S], as[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        bs[t] = (T)st.b[t] * bsm;
        as[t] = (T)st.a[t];
    }
    T xw[NR][S + 1][3][2];
    T fw[NR][S + 2][2];
    T rw[NR][3][2];
    // the weights and 1/D of the last S + 2 rows (index j: row r - j), the
    // west weight of the first column, and the north weights of row
    // r - S - 2 (the residual's south weights); S + 2 rows, the f window's
    // period
    T cwx[S + 2][2], cwy[S + 2][2], cdi[S + 2][2], cww[S + 2];
    T cwys[2] = {T(0), T(0)};
#pragma unroll
    for (int j = 0; j < S + 2; ++j) cwx[j][0] = cwx[j][1] = cwy[j][0] = cwy[j][1] = cdi[j][0] = cdi[j][1] = cww[j] = T(0);
    // GEN: the north-east weights of the last S + 2 rows, the south-west
    // weight of the first column (the left lane's north-east weight one row
    // lower), the diagonal (PRE: the residual), and the north-east weights of
    // row r - S - 2 (the residual's south-west weights)
    constexpr int GW = GEN ? S + 2 : 1, GD = GEN && !POST ? S + 2 : 1;
    T cne[GW][2], csw[GW], cdd[GD][2];
    T cnes[2] = {T(0), T(0)}, csws = T(0);
#pragma unroll
    for (int j = 0; j < GW; ++j) cne[j][0] = cne[j][1] = csw[j] = T(0);
#pragma unroll
    for (int j = 0; j < GD; ++j) cdd[j][0] = cdd[j][1] = T(0);
#pragma unroll
    for (int n = 0; n < NR; ++n) {
#pragma unroll
        for (int t = 0; t <= S; ++t)
#pragma unroll
            for (int k = 0; k < 3; ++k) xw[n][t][k][0] = xw[n][t][k][1] = T(0);
#pragma unroll
        for (int j = 0; j < S + 2; ++j) fw[n][j][0] = fw[n][j][1] = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) rw[n][k][0] = rw[n][k][1] = T(0);
    }

    const int r_begin = y0 - 2 - S;
    const int r_end = y0 + MSEG + S + 1;
    // per-lane column offsets (bytes), fixed for the march; positions outside
    // the grid clamp onto the boundary ring, whose stored values are zero
    const int ia = min(max(i0, 0), g.n), ib = min(max(i0 + 1, 0), g.n);
    const int ga = gx(ia), gb = gx(ib);
    const unsigned va = 4u * ga, vb = 4u * gb;
    // in a reflected band the kernel's east edge is the grid's west edge (wx
    // one column lower) and its north edge the grid's south edge (wy one row
    // lower)
    const unsigned vwa = 4u * (flip ? max(ga - 1, 0) : ga), vwb = 4u * (flip ? max(gb - 1, 0) : gb);
    // POST: coarse nodes (I, J) and (I + a, J + b) of each column's nodal
    // interpolation (a = i & 1 per lane, b = r & 1 per row)
    unsigned ve0[2], ve1[2];
    {
        const int cols[2] = {ia, ib};
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const int i = cols[cc];
            ve0[cc] = 4u * gcx(i >> 1);
            ve1[cc] = 4u * (gcx(i >> 1) + fs * (i & 1));
        }
    }
    // store offsets of the lane's columns (dropped outside the owned,
    // interior columns)
    const unsigned sa = (owned[0] && inner[0]) ? va : kDropped, sb = (owned[1] && inner[1]) ? vb : kDropped;
    // restriction (PRE): the coarse node centred on the lane's first column
    const int Ir = i0 >> 1;
    const bool rown = owned[0] && Ir >= 1 && Ir <= gc.m;
    const unsigned vr = 4u * gcx(Ir);

    struct Slot {
        T x[NR][2], f[NR][2], e0[NR][2], e1[NR][2];
        T wx[2], wy[2], ne[GEN ? 2 : 1], dd[GEN ? 2 : 1];
    };
    auto load = [&](int r, Slot& sl) {
        const int rr = min(max(r, 0), g.n);
        const unsigned so = 4u * (unsigned)(gx(rr) * g.pitch + ORIGIN);
        const unsigned sw = 4u * (unsigned)((flip ? max(gx(rr) - 1, 0) : rr) * g.pitch + ORIGIN);
        sl.wx[0] = bload(wxs, vwa, so);
        sl.wx[1] = bload(wxs, vwb, so);
        sl.wy[0] = bload(wys, va, sw);
        sl.wy[1] = bload(wys, vb, sw);
        if constexpr (GEN) {
            // the kernel's north-east neighbour is the grid's south-west one
            // in a reflected band: the weight one column and one row lower
            sl.ne[0] = bload(nes, vwa, sw);
            sl.ne[1] = bload(nes, vwb, sw);
            sl.dd[0] = bload(dds, va, so);
            sl.dd[1] = bload(dds, vb, so);
        }
        unsigned sc0 = 0, sc1 = 0;
        if constexpr (POST) {
            const int b = rr & 1;
            sc0 = 4u * (unsigned)(gcx(rr >> 1) * gc.pitch + ORIGIN);
            sc1 = 4u * (unsigned)(gcx(rr >> 1) * gc.pitch + ORIGIN + fs * b * gc.pitch);
        }
#pragma unroll
        for (int n = 0; n < NR; ++n) {
            sl.f[n][0] = bload(fsr, va, so + n * pb);
            sl.f[n][1] = bload(fsr, vb, so + n * pb);
            if (POST || !XZ) {
                sl.x[n][0] = bload(xs, va, so + n * pb);
                sl.x[n][1] = bload(xs, vb, so + n * pb);
            }
            if constexpr (POST) {
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    sl.e0[n][cc] = bload(es, ve0[cc], sc0 + n * cb);
                    sl.e1[n][cc] = bload(es, ve1[cc], sc1 + n * cb);
                }
            }
        }
    };
    // row r enters the windows
    auto shift_in = [&](const Slot& sl, const int r) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
#pragma unroll
            for (int n = 0; n < NR; ++n) {
                T cx;
                if constexpr (POST) cx = sl.x[n][cc] + T(0.5) * (sl.e0[n][cc] + sl.e1[n][cc]);
                else if constexpr (!XZ) cx = detach(sl.x[n][cc]);
                else cx = T(0);
#pragma unroll
                for (int j = S + 1; j > 0; --j) fw[n][j][cc] = fw[n][j - 1][cc];
                fw[n][0][cc] = detach(sl.f[n][cc]);
                xw[n][0][2][cc] = xw[n][0][1][cc];
                xw[n][0][1][cc] = xw[n][0][0][cc];
                xw[n][0][0][cc] = cx;
            }
            cwys[cc] = cwy[S + 1][cc];
#pragma unroll
            for (int j = S + 1; j > 0; --j) {
                cwx[j][cc] = cwx[j - 1][cc];
                cwy[j][cc] = cwy[j - 1][cc];
                cdi[j][cc] = cdi[j - 1][cc];
            }
            cwx[0][cc] = detach(sl.wx[cc]);
            cwy[0][cc] = detach(sl.wy[cc]);
            if constexpr (GEN) {
                cnes[cc] = cne[S + 1][cc];
#pragma unroll
                for (int j = S + 1; j > 0; --j) cne[j][cc] = cne[j - 1][cc];
                cne[0][cc] = detach(sl.ne[cc]);
                if constexpr (!POST) {
#pragma unroll
                    for (int j = S + 1; j > 0; --j) cdd[j][cc] = cdd[j - 1][cc];
                    cdd[0][cc] = detach(sl.dd[cc]);
                }
            }
        }
        if constexpr (GEN) {
            csws = csw[S + 1];
#pragma unroll
            for (int j = S + 1; j > 0; --j) csw[j] = csw[j - 1];
            csw[0] = from_left(cne[0][1]);
        }
#pragma unroll
        for (int j = S + 1; j > 0; --j) cww[j] = cww[j - 1];
        // 1 / D of row r: east, west (the left lane's east weight for the
        // first column), north and south (row r - 1's north) weights.  On
        // boundary and outside nodes it is 0: there every stage keeps
        // x = (1 - b) x + a (x - x_prev), which stays at the loaded 0, so the
        // stages need no mask (and no branch on the row)
        cww[0] = from_left(cwx[0][1]);
        const bool rin = r >= 1 && r <= g.m;
        T d0, d1;
        if constexpr (GEN) {
            d0 = recip(sl.dd[0]);
            d1 = recip(sl.dd[1]);
        } else {
            d0 = recip(cwx[0][0] + cww[0] + cwy[0][0] + cwy[1][0]);
            d1 = recip(cwx[0][1] + cwx[0][0] + cwy[0][1] + cwy[1][1]);
        }
        cdi[0][0] = (rin && inner[0]) ? d0 : T(0);
        cdi[0][1] = (rin && inner[1]) ? d1 : T(0);
    };
    // after row r entered: every stage advances one row, x_S of row r - S is
    // stored, and (PRE) the residual and its restriction
    auto advance = [&](const int r) {
#pragma unroll
        for (int t = 1; t <= S; ++t) {
            const T we[2] = {cwx[t][0], cwx[t][1]};
            const T ww[2] = {cww[t], cwx[t][0]};
#pragma unroll
            for (int n = 0; n < NR; ++n) {
                const T m0 = xw[n][t - 1][1][0], m1 = xw[n][t - 1][1][1];
                const T left = from_left(m1), right = from_right(m0);
                const T mc[2] = {m0, m1};
                const T xe[2] = {m1, right}, xwv[2] = {left, m0};
                T v[2];
                // GEN: the diagonal neighbours (i + 1, q + 1), (i - 1, q - 1)
                T xne[2], xsw[2], wa[2], wb[2];
                if constexpr (GEN) {
                    xne[0] = xw[n][t - 1][0][1];
                    xne[1] = from_right(xw[n][t - 1][0][0]);
                    xsw[0] = from_left(xw[n][t - 1][2][1]);
                    xsw[1] = xw[n][t - 1][2][0];
                    wa[0] = cne[t][0];
                    wa[1] = cne[t][1];
                    wb[0] = csw[t + 1];
                    wb[1] = cne[t + 1][0];
                }
                // x + b ((f + sum w x_nb) / D - x)
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    T sfv = __builtin_fmaf(we[cc], xe[cc], fw[n][t][cc]);
                    sfv = __builtin_fmaf(ww[cc], xwv[cc], sfv);
                    sfv = __builtin_fmaf(cwy[t][cc], xw[n][t - 1][0][cc], sfv);
                    sfv = __builtin_fmaf(cwy[t + 1][cc], xw[n][t - 1][2][cc], sfv);
                    if constexpr (GEN) {
                        sfv = __builtin_fmaf(wa[cc], xne[cc], sfv);
                        sfv = __builtin_fmaf(wb[cc], xsw[cc], sfv);
                    }
                    T val = __builtin_fmaf(bs[t - 1], __builtin_fmaf(sfv, cdi[t][cc], -mc[cc]), mc[cc]);
                    if (t >= 2) val = __builtin_fmaf(as[t - 1], mc[cc] - xw[n][t - 2][2][cc], val);
                    v[cc] = val;
                }
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    xw[n][t][2][cc] = xw[n][t][1][cc];
                    xw[n][t][1][cc] = xw[n][t][0][cc];
                    xw[n][t][0][cc] = v[cc];
                }
            }
        }
        {
            const int q = r - S;
            const bool st_row = q >= y0 && q < y0 + MSEG && q >= 1 && q <= g.m;  // uniform
            const unsigned so = 4u * (unsigned)(gx(max(q, 0)) * g.pitch + ORIGIN);
#pragma unroll
            for (int n = 0; n < NR; ++n) {
                bstore(xw[n][S][0][0], os, st_row ? so + n * pb + sa : kDropped);
                bstore(xw[n][S][0][1], os, st_row ? so + n * pb + sb : kDropped);
            }
        }
        if constexpr (!POST) {
            // residual at row r - S - 1 from x_S rows (r-S, r-S-1, r-S-2), in
            // the difference form (the restricted residual is small against
            // D x once the error is smooth); then the restriction to the
            // coarse node centred at (i0, r - S - 2).  An interior coarse
            // node's seven fine nodes are interior, so the residuals of
            // boundary and outside nodes (finite, not zero) never reach a
            // stored value
            const int q2 = r - S - 2;
            const bool rrow = ((q2 & 1) == 0) && q2 >= y0 && q2 < y0 + MSEG && (q2 >> 1) >= 1 && (q2 >> 1) <= gc.m;
            const unsigned sor = 4u * (unsigned)(gcx(max(q2, 0) >> 1) * gc.pitch + ORIGIN);
            const T ww0 = cww[S + 1];
#pragma unroll
            for (int n = 0; n < NR; ++n) {
                const T m0 = xw[n][S][1][0], m1 = xw[n][S][1][1];
                const T left = from_left(m1), right = from_right(m0);
                T ax0 = cwx[S + 1][0] * (m0 - m1) + ww0 * (m0 - left) + cwy[S + 1][0] * (m0 - xw[n][S][0][0]) +
                        cwys[0] * (m0 - xw[n][S][2][0]);
                T ax1 = cwx[S + 1][1] * (m1 - right) + cwx[S + 1][0] * (m1 - m0) +
                        cwy[S + 1][1] * (m1 - xw[n][S][0][1]) + cwys[1] * (m1 - xw[n][S][2][1]);
                if constexpr (GEN) {
                    // the diagonal couplings, and the rest of the diagonal
                    // (d minus the six weights) times x
                    const T ne0 = xw[n][S][0][1], ne1 = from_right(xw[n][S][0][0]);
                    const T sw0 = from_left(xw[n][S][2][1]), sw1 = xw[n][S][2][0];
                    const T wa0 = cne[S + 1][0], wa1 = cne[S + 1][1], wb0 = csws, wb1 = cnes[0];
                    ax0 += wa0 * (m0 - ne0) + wb0 * (m0 - sw0) +
                           (cdd[S + 1][0] - (cwx[S + 1][0] + ww0 + cwy[S + 1][0] + cwys[0] + wa0 + wb0)) * m0;
                    ax1 += wa1 * (m1 - ne1) + wb1 * (m1 - sw1) +
                           (cdd[S + 1][1] - (cwx[S + 1][1] + cwx[S + 1][0] + cwy[S + 1][1] + cwys[1] + wa1 + wb1)) *
                               m1;
                }
                T res0 = fw[n][S + 1][0] - ax0;
                T res1 = fw[n][S + 1][1] - ax1;
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    rw[n][2][cc] = rw[n][1][cc];
                    rw[n][1][cc] = rw[n][0][cc];
                }
                rw[n][0][0] = res0;
                rw[n][0][1] = res1;
                const T mid_left = from_left(rw[n][1][1]);  // (i0-1, q2)
                const T dn_left = from_left(rw[n][2][1]);   // (i0-1, q2-1)
                const T rv = rw[n][1][0] + T(0.5) * (rw[n][1][1] + mid_left + rw[n][0][0] + rw[n][2][0] +
                                                     rw[n][0][1] + dn_left);
                bstore(rv, rs, (rrow && rown) ? sor + n * cb + vr : kDropped);
            }
        }
    };

    Slot q[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) load(r_begin + p, q[p]);
    drain_vmem();
    constexpr int UNR = ew_unroll<S, PF>();
    const int iters = (r_end - r_begin + UNR) / UNR;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int r = r_begin + it * UNR + u;
            shift_in(q[u % PF], r);
            load(r + PF, q[u % PF]);
            advance(r);
        }
    }
}

// Workgroup slots of the whole device for a kernel (one wavefront each).
template <typename K>
int device_wave_slots(K kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    PASM_HIP(hipGetDevice(&dev));
    PASM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PASM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, NL, 0));
    return std::max(1, cus * per_cu);
}

// Rows per band.  A wavefront walks its band's rows plus `extra` rows of
// halo (rounded up to the unrolled body of `unr` rows), and the launch runs
// in rounds of `slots` resident wavefronts, the last one possibly partial:
// the band height is the one that minimises rounds x rows walked (taller
// bands walk fewer halo rows in total, shorter ones leave less of a last
// round idle).  rows > 0 fixes the height instead.
MarchShape march_shape(const Grid& g, int txo, int nrhs, int slots, int rows, int extra = 0, int unr = 1) {
    MarchShape sh{};
    sh.strips = (g.n + 1 + txo - 1) / txo;
    const long base = (long)sh.strips * nrhs;
    int mseg = rows;
    if (mseg <= 0) {
        double best = 0.0;
        for (int m = 16; m <= 512; m += 2) {
            const long segs = (g.n + 1 + m - 1) / m;
            const long rounds = (base * segs + slots - 1) / slots;
            const long walked = (m + extra + unr - 1) / unr * unr;
            const double cost = (double)rounds * walked;
            if (mseg <= 0 || cost < best) {
                best = cost;
                mseg = m;
            }
            if (m >= g.n + 1) break;
        }
    }
    sh.mseg = (mseg + 1) & ~1;
    sh.segs = (g.n + 1 + sh.mseg - 1) / sh.mseg;
    sh.nrhs = nrhs;
    sh.work = (int)((long)sh.strips * sh.segs * nrhs);
    sh.blocks = (sh.work + XCDS - 1) / XCDS * XCDS;
    return sh;
}

// Returns the wavefronts per right-hand side (MODE 3: pairs of sums in part).
template <typename T, int S, int MODE>
int march_launch(const Grid& g, T w0, const T* x0, const T* f, T* out, const T* ec, const Grid& gc, T* rc, T* rc2,
                 double* part, int nrhs, long sf, long sc, const SmoothSteps& ss, bool x_zero, int rows,
                 hipStream_t st) {
    constexpr int TXO = MW - 2 * march_halo(S);
    static const int slots = device_wave_slots(k_march<T, S, MODE, false>);
    constexpr int UNR = MODE == 4 ? lcm_(3, prefetch_rows<T>()) : march_unroll(S, prefetch_rows<T>());
    const MarchShape sh = march_shape(g, TXO, nrhs, slots, rows, 2 * S + 4, UNR);
    if constexpr (MODE == 1) {
        if (x_zero) {
            hipLaunchKernelGGL((k_march<T, S, MODE, true>), dim3(sh.blocks), dim3(NL), 0, st, g, w0, x0, f, out, ec,
                               gc, rc, rc2, part, sf, sc, ss, sh, ProlongSrc{});
            PASM_CHECK_LAUNCH();
            return sh.strips * sh.segs;
        }
    }
    hipLaunchKernelGGL((k_march<T, S, MODE, false>), dim3(sh.blocks), dim3(NL), 0, st, g, w0, x0, f, out, ec, gc, rc,
                       rc2, part, sf, sc, ss, sh, ProlongSrc{});
    PASM_CHECK_LAUNCH();
    return sh.strips * sh.segs;
}

// MODE 4 (FP64): the post-smoothing of one V-cycle, with its prolongation,
// and the next cycle's pre-smoothing, with its residual restriction, in one
// pass.  More registers per wavefront than one phase, so the bands are sized
// for a single round of resident wavefronts.
// Rows per band such that every wavefront of the launch is resident at once.
int one_round_rows(const Grid& g, int txo, int nrhs, int slots) {
    const long strips = (g.n + 1 + txo - 1) / txo;
    const long bands = std::max<long>(1, slots / (strips * nrhs));
    return std::max(16, (int)((g.n + 1 + bands - 1) / bands));
}

template <int S>
void march_pair_launch(const Grid& g, double w0, const double* x, const double* f, double* out, const double* ec,
                       const Grid& gc, double* rc, int nrhs, const SmoothSteps& ss, hipStream_t st) {
    constexpr int TXO = MW - 2 * march_halo(S);
    static const int slots = device_wave_slots(k_march<double, S, 4, false>);
    const MarchShape sh = march_shape(g, TXO, nrhs, slots, one_round_rows(g, TXO, nrhs, slots));
    hipLaunchKernelGGL((k_march<double, S, 4, false>), dim3(sh.blocks), dim3(NL), 0, st, g, w0, x, f, out, ec, gc,
                       rc, (double*)nullptr, (double*)nullptr, g.plane, gc.plane, ss, sh, ProlongSrc{});
    PASM_CHECK_LAUNCH();
}

// MODE 5 (FP64): the first pre-smoothing of a correction step with the
// previous step's prolongation and its right-hand side formed in the pass.
template <int S>
void march_prolong_launch(const Grid& g, double w0, const double* u, double* fout, double* out, const Grid& gc,
                          double* rc, const ProlongSrc& ps, int nrhs, const SmoothSteps& ss, hipStream_t st) {
    constexpr int TXO = MW - 2 * march_halo(S);
    static const int slots = device_wave_slots(k_march<double, S, 5, false>);
    const MarchShape sh = march_shape(g, TXO, nrhs, slots, one_round_rows(g, TXO, nrhs, slots));
    hipLaunchKernelGGL((k_march<double, S, 5, false>), dim3(sh.blocks), dim3(NL), 0, st, g, w0, u, fout, out,
                       (const double*)nullptr, gc, rc, (double*)nullptr, (double*)nullptr, g.plane, gc.plane, ss, sh,
                       ps);
    PASM_CHECK_LAUNCH();
}

template <typename T, int MODE>
int march_dispatch(const Grid& g, T w0, const T* x0, const T* f, T* out, const T* ec, const Grid& gc, T* rc,
                   T* rc2, double* part, int nrhs, long sf, long sc, const SmoothSteps& ss, bool x_zero, int rows,
                   hipStream_t st) {
    switch (ss.s) {
        case 1: return march_launch<T, 1, MODE>(g, w0, x0, f, out, ec, gc, rc, rc2, part, nrhs, sf, sc, ss, x_zero, rows, st);
        case 2: return march_launch<T, 2, MODE>(g, w0, x0, f, out, ec, gc, rc, rc2, part, nrhs, sf, sc, ss, x_zero, rows, st);
        case 3: return march_launch<T, 3, MODE>(g, w0, x0, f, out, ec, gc, rc, rc2, part, nrhs, sf, sc, ss, x_zero, rows, st);
        case 4: return march_launch<T, 4, MODE>(g, w0, x0, f, out, ec, gc, rc, rc2, part, nrhs, sf, sc, ss, x_zero, rows, st);
        default: throw Error(PASM_E_INVALID, "marching smoother supports 1..4 steps");
    }
}

// Edge-weight phases: NR right-hand sides per wavefront (a ragged last
// group is padded by right-hand sides whose accesses fall outside the
// buffers).
template <int S, int MODE, int NR, bool GEN>
void march_launch_ew(const Grid& g, const float* x0, const float* f, float* out, const float* ec, const Grid& gc,
                     float* rc, int nrhs, const SmoothSteps& ss, bool x_zero, const EdgeW<float>& ew,
                     hipStream_t st) {
    constexpr int TXO = MW - 2 * march_halo(S);
    constexpr int PF = 6 / NR > 2 ? 6 / NR : 3;
    static const int slots = device_wave_slots(k_march_ew<S, MODE, false, NR, GEN>);
    const int ngrp = (nrhs + NR - 1) / NR;
    MarchShape sh = march_shape(g, TXO, ngrp, slots, 0, 2 * S + 4, ew_unroll<S, PF>());
    sh.nrhs = nrhs;
    if (MODE == 1 && x_zero)
        hipLaunchKernelGGL((k_march_ew<S, MODE, true, NR, GEN>), dim3(sh.blocks), dim3(NL), 0, st, g, x0, f, out, ec,
                           gc, rc, g.plane, gc.plane, ss, sh, ew);
    else
        hipLaunchKernelGGL((k_march_ew<S, MODE, false, NR, GEN>), dim3(sh.blocks), dim3(NL), 0, st, g, x0, f, out, ec,
                           gc, rc, g.plane, gc.plane, ss, sh, ew);
    PASM_CHECK_LAUNCH();
}

template <int MODE, int NR, bool GEN>
void march_dispatch_ew_nr(const Grid& g, const float* x0, const float* f, float* out, const float* ec,
                          const Grid& gc, float* rc, int nrhs, const SmoothSteps& ss, bool x_zero,
                          const EdgeW<float>& ew, hipStream_t st) {
    switch (ss.s) {
        case 1: march_launch_ew<1, MODE, NR, GEN>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st); break;
        case 2: march_launch_ew<2, MODE, NR, GEN>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st); break;
        case 3: march_launch_ew<3, MODE, NR, GEN>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st); break;
        case 4: march_launch_ew<4, MODE, NR, GEN>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st); break;
        default: throw Error(PASM_E_INVALID, "marching smoother supports 1..4 steps");
    }
}

// Two right-hand sides per wavefront unless a pair could straddle two
// members of a batch (an odd number of right-hand sides per member).
template <int MODE>
void march_dispatch_ew(const Grid& g, const float* x0, const float* f, float* out, const float* ec, const Grid& gc,
                       float* rc, int nrhs, const SmoothSteps& ss, bool x_zero, const EdgeW<float>& ew,
                       hipStream_t st) {
    const bool per_member = ew.ms != 0 || ew.bsc;
    const bool pairs = nrhs >= 2 && (!per_member || ew.kpm % 2 == 0);
    if (ew.d) {
        if (pairs) march_dispatch_ew_nr<MODE, 2, true>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st);
        else march_dispatch_ew_nr<MODE, 1, true>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st);
    } else {
        if (pairs) march_dispatch_ew_nr<MODE, 2, false>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st);
        else march_dispatch_ew_nr<MODE, 1, false>(g, x0, f, out, ec, gc, rc, nrhs, ss, x_zero, ew, st);
    }
}

EdgeW<float> edge_weights_of(const Coef<float>& c) {
    EdgeW<float> ew{c.wx, c.wy};
    ew.d = c.d;
    ew.wne = c.wne;
    ew.ms = c.ms;
    ew.kpm = std::max(1, c.kpm);
    ew.bsc = c.bsc;
    return ew;
}

}  // namespace

// Levels with edge weights (per-element kappa) or the general 7-point
// operator (kappa and a potential), FP32 V-cycles: pre-smoothing with the
// residual restriction and post-smoothing with the prolongation as marching
// passes, as for constant coefficients.  Batches: every member's planes.
// (from 128 cells: with many right-hand sides the strips, bands and pairs
// still fill the machine; measured faster than the tile smoothers there)
bool march_ew_supported(const Grid& g, int steps) {
    return g.dim == 2 && steps >= 1 && steps <= 4 && g.n >= 128;
}

bool march_coef_supported(const Grid& g, const Coef<float>& c, int steps) {
    const int kind = coef_kind(c);
    return march_ew_supported(g, steps) && (kind == 1 || (kind == 2 && c.wne)) && c.wx && c.wy;
}

void launch_march_pre_ew(const Grid& g, const Coef<float>& c, const float* x0, const float* f, float* out,
                         const Grid& gc, float* rc, int nrhs, const SmoothSteps& ss, bool x_zero, hipStream_t st) {
    if (!march_coef_supported(g, c, ss.s) || gc.n * 2 != g.n)
        throw Error(PASM_E_INVALID, "coefficient marching: 2D, at least 128 cells, ratio 2, edge weights or 7 points");
    march_dispatch_ew<1>(g, x0, f, out, nullptr, gc, rc, nrhs, ss, x_zero, edge_weights_of(c), st);
}

void launch_march_post_ew(const Grid& g, const Coef<float>& c, const float* x, const float* f, float* out,
                          const Grid& gc, const float* ec, int nrhs, const SmoothSteps& ss, hipStream_t st) {
    if (!march_coef_supported(g, c, ss.s) || gc.n * 2 != g.n)
        throw Error(PASM_E_INVALID, "coefficient marching: 2D, at least 128 cells, ratio 2, edge weights or 7 points");
    march_dispatch_ew<2>(g, x, f, out, ec, gc, nullptr, nrhs, ss, false, edge_weights_of(c), st);
}

// Large 2D levels only: a wavefront walks 64 + 2(S+2) rows in sequence, which
// needs many strips and segments to fill the machine; smaller levels use the
// tile kernels.
bool march_supported(const Grid& g, bool const_coef, int steps) {
    return g.dim == 2 && const_coef && steps >= 1 && steps <= 4 && g.n >= 256;
}

bool march_pair_supported(const Grid& g, bool const_coef, int post, int pre) {
    return march_supported(g, const_coef, post) && march_supported(g, const_coef, pre) && post + pre <= 8;
}

void launch_march_post_pre(const Grid& g, double w0, const double* x, const double* f, double* out, const Grid& gc,
                           const double* ec, double* rc, int nrhs, const SmoothSteps& post, const SmoothSteps& pre,
                           hipStream_t st) {
    if (!march_pair_supported(g, true, post.s, pre.s) || gc.n * 2 != g.n)
        throw Error(PASM_E_INVALID, "paired marching phases: 2D, ratio 2, at most 8 steps");
    // the step sizes come scaled by 1 / (4 w0) (the diagonal), as the
    // one-phase kernels scale them, so that they stay in scalar registers
    const double invD = 1.0 / (4.0 * w0);
    SmoothSteps ss{};
    ss.s = post.s + pre.s;
    for (int t = 0; t < post.s; ++t) {
        ss.a[t] = post.a[t];
        ss.b[t] = post.b[t] * invD;
    }
    for (int t = 0; t < pre.s; ++t) {
        // the first pre-smoothing step starts a new recurrence: no momentum term
        ss.a[post.s + t] = t == 0 ? 0.0 : pre.a[t];
        ss.b[post.s + t] = pre.b[t] * invD;
    }
    switch (ss.s) {
        case 2: march_pair_launch<2>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
        case 3: march_pair_launch<3>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
        case 4: march_pair_launch<4>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
        case 5: march_pair_launch<5>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
        case 6: march_pair_launch<6>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
        case 7: march_pair_launch<7>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
        default: march_pair_launch<8>(g, w0, x, f, out, ec, gc, rc, nrhs, ss, st); break;
    }
}

int ratio_log2(const Grid& g, const Grid& gq) {
    if (gq.n <= 0 || g.n % gq.n != 0) return -1;
    const int r = g.n / gq.n;
    if (r < 2 || (r & (r - 1)) != 0) return -1;
    int lr = 0;
    while ((1 << lr) < r) ++lr;
    return lr;
}

bool march_prolong_supported(const Grid& g, bool const_coef, int pre, const Grid& gq) {
    return march_supported(g, const_coef, pre) && gq.dim == 2 && ratio_log2(g, gq) > 0;
}

void launch_march_pre_prolong(const Grid& g, double w0, const double* u, double* fout, double* out, const Grid& gc,
                              double* rc, const Grid& gq, const double* q, const double* beta, const double* lam,
                              int nrhs, const SmoothSteps& pre, hipStream_t st) {
    if (!march_prolong_supported(g, true, pre.s, gq) || gc.n * 2 != g.n)
        throw Error(PASM_E_INVALID, "prolonging pre-smoothing: 2D, power-of-two ratio to the coarse space");
    const ProlongSrc ps{gq, q, gq.plane, ratio_log2(g, gq), beta, lam, fout};
    switch (pre.s) {
        case 1: march_prolong_launch<1>(g, w0, u, fout, out, gc, rc, ps, nrhs, pre, st); break;
        case 2: march_prolong_launch<2>(g, w0, u, fout, out, gc, rc, ps, nrhs, pre, st); break;
        case 3: march_prolong_launch<3>(g, w0, u, fout, out, gc, rc, ps, nrhs, pre, st); break;
        default: march_prolong_launch<4>(g, w0, u, fout, out, gc, rc, ps, nrhs, pre, st); break;
    }
}

template <typename T>
void launch_march_pre(const Grid& g, T w0, const T* x0, const T* f, T* out, const Grid& gc, T* rc, int nrhs,
                      const SmoothSteps& ss, bool x_zero, hipStream_t st, int rows) {
    march_dispatch<T, 1>(g, w0, x0, f, out, (const T*)nullptr, gc, rc, (T*)nullptr, nullptr, nrhs, g.plane, gc.plane,
                         ss, x_zero, rows, st);
}

template <typename T>
void launch_march_post(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                       const SmoothSteps& ss, hipStream_t st, int rows) {
    march_dispatch<T, 2>(g, w0, x, f, out, ec, gc, (T*)nullptr, (T*)nullptr, nullptr, nrhs, g.plane, gc.plane, ss,
                         false, rows, st);
}

int launch_march_post_border(const Grid& g, double w0, const double* x, const double* f, double* out, const Grid& gc,
                             const double* ec, double* bc, double* cc, double* partial, int nrhs,
                             const SmoothSteps& ss, hipStream_t st, int rows) {
    if (g.dim != 2 || gc.n * 2 != g.n) throw Error(PASM_E_INVALID, "fused border restriction: 2D, ratio 2");
    return march_dispatch<double, 3>(g, w0, x, f, out, ec, gc, bc, cc, partial, nrhs, g.plane, gc.plane, ss, false,
                                     rows, st);
}

template void launch_march_pre<double>(const Grid&, double, const double*, const double*, double*, const Grid&,
                                       double*, int, const SmoothSteps&, bool, hipStream_t, int);
template void launch_march_pre<float>(const Grid&, float, const float*, const float*, float*, const Grid&, float*,
                                      int, const SmoothSteps&, bool, hipStream_t, int);
template void launch_march_post<double>(const Grid&, double, const double*, const double*, double*, const Grid&,
                                        const double*, int, const SmoothSteps&, hipStream_t, int);
template void launch_march_post<float>(const Grid&, float, const float*, const float*, float*, const Grid&,
                                       const float*, int, const SmoothSteps&, hipStream_t, int);

}  // namespace pasm

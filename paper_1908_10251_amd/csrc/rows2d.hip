// The borders after the last correction of a step (Algorithm 1, step 2: the
// coarse-space vectors built from A u~ and M u~, and the scalars u~.A u~,
// u~.M u~) as a row-marching FP64 pass, on 2D levels with edge weights
// (per-element kappa) of a single problem with many right-hand sides.
//
// One wavefront owns a strip of 64 consecutive columns of one right-hand side
// (one column per lane) and marches up a band of rows.  The last three rows
// of its fields and the next two rows in flight sit in a ring of five
// register slots; the loop over rows is unrolled by five, so each slot is a
// fixed set of registers and the only wait is for the oldest row in flight.
// East and west neighbours come from the adjacent lanes by DPP wavefront
// shifts; the strips overlap by four columns, whose lanes only supply
// neighbours, so every node is read about once (plus one row at each end of
// a band) and no halo is staged.  Pieces of work (strip, band, right-hand
// side), strip fastest, go to the dies in contiguous ranges: the strips of a
// band that share halo columns run on one die, and each die streams whole
// rows of one right-hand side at a time (the weights then come from the
// shared last-level cache; taking several right-hand sides of a strip
// together in a wavefront, or on a die at once, measured slower).
#include <algorithm>

#include "common.h"

namespace pasm {

namespace {

constexpr int RL = 64;   // lanes per wavefront
constexpr int RWG = 4;   // wavefronts per workgroup
constexpr int RXCD = 8;  // dies; workgroup b runs on die b % 8
constexpr int RNS = 5;   // register slots: rows j - 1, j, j + 1 and two in flight

// Value of lane l - 1 (lane 0 gets 0) and of lane l + 1 (lane 63 gets 0).
__device__ inline double lane_prev(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double lane_next(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

struct RowWork {
    int strips;  // strips per row
    int bands;   // bands per right-hand side
    int rows;    // coarse rows per band
    int work;    // strips x bands x right-hand sides
};

// ---------------------------------------------------------------------------
// Borders of un = u + e (e the FP32 correction, added in FP64), un written
// (E0: un = (u + e0) + e, the corrections of two cycles in their order):
// A un and M un at every fine node, bc = P^T A un and cc = P^T M un on the
// next coarser grid gc (centre 1, the six neighbours of the "/" mesh 1/2),
// and the sums un.A un, un.M un over the piece's own fine nodes (one pair per
// piece).  Lanes 1 .. 60 own their fine columns; the coarse nodes sit at the
// even lanes 2 .. 60 and gather from lanes 1 .. 61, whose A un needs lane 62.
// A band is a range of coarse rows J0 .. J1 - 1 and owns the fine rows
// 2 J0 - 1 .. 2 J1 - 2 (the last band up to m); it forms A un on the fine
// rows 2 J0 - 1 .. 2 J1 - 1.
// ---------------------------------------------------------------------------
constexpr int BOWN = RL - 4;

template <bool E0>
__global__ __launch_bounds__(RL* RWG) void k_border_rows(Grid g, const double* __restrict__ wx,
                                                         const double* __restrict__ wy, const double* __restrict__ u,
                                                         const float* __restrict__ e, const float* __restrict__ e0,
                                                         double* __restrict__ un,
                                                         Grid gc, double* __restrict__ bc, double* __restrict__ cc,
                                                         double* __restrict__ partial, long stride, long sc,
                                                         RowWork rw) {
    const int per = gridDim.x / RXCD;
    const int wg = (blockIdx.x % RXCD) * per + blockIdx.x / RXCD;
    // the wavefront's piece, as a uniform value
    const int w = wg * RWG + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RL));
    if (w >= rw.work) return;
    const int strip = w % rw.strips;
    const int band = (w / rw.strips) % rw.bands;
    const int z = w / (rw.strips * rw.bands);
    const int lane = threadIdx.x % RL;
    const int i = strip * BOWN + lane;
    const long col = ORIGIN + min(i, g.n);  // lanes past the boundary read the boundary (zero)
    const bool own = lane >= 1 && lane <= BOWN && i <= g.m;
    const bool cown = own && (lane % 2) == 0;  // coarse node I = i / 2 (i <= m, even: I <= gc.m)
    const long ccol = ORIGIN + (own ? i / 2 : 1);
    const int J0 = 1 + band * rw.rows, J1 = min(J0 + rw.rows, gc.n);
    const int ja = 2 * J0 - 1, jb1 = 2 * J1 - 1;  // fine rows with A un: ja .. jb1
    const int jo = J1 == gc.n ? g.m : 2 * J1 - 2;  // last owned fine row
    const long p = g.pitch, pc = gc.pitch;
    const long zo = (long)z * stride, zq = (long)z * sc;
    const double h2 = g.h * g.h;
    double su[RNS], swx[RNS], swy[RNS];
    float se[RNS], s0[RNS];
    auto load = [&](int s, int jj) {
        const long o = (long)jj * p + col;
        swx[s] = wx[o];
        swy[s] = wy[o];
        su[s] = u[zo + o];
        se[s] = e[zo + o];
        if (E0) s0[s] = e0[zo + o];
    };
    auto xsum = [&](int s) { return E0 ? (su[s] + (double)s0[s]) + (double)se[s] : su[s] + (double)se[s]; };
#pragma unroll
    for (int s = 0; s < RNS - 1; ++s) load(s, min(ja - 1 + s, jb1 + 1));  // rows ja - 1 .. ja + 2
    // restriction state: of A un and M un, the sum of S and SW of the coarse
    // row being formed (from its odd row below), and its centre C and the sum
    // of W and E (from its even row)
    double aS = 0.0, aC = 0.0, aWE = 0.0, mS = 0.0, mC = 0.0, mWE = 0.0, ua = 0.0, um = 0.0;
    // one row: q the row's place in the unrolled body of RNS rows
    auto step = [&](const int q, const int j) {
        const int S = q % RNS, C = (q + 1) % RNS, N = (q + 2) % RNS, P = (q + 4) % RNS;
        load(P, min(j + 3, jb1 + 1));  // row j + 3 into the free slot (the last rows load row jb1 + 1 again)
        const double we = swx[C], ww = lane_prev(we), wn = swy[C], ws = swy[S];
        const double x0 = xsum(C);
        const double xn = xsum(N), xs = xsum(S);
        const double xe = lane_next(x0), xw = lane_prev(x0);
        const double xne = lane_next(xn), xsw = lane_prev(xs);
        const double Ax = (we + ww + wn + ws) * x0 - we * xe - ww * xw - wn * xn - ws * xs;
        const double Mx = h2 * (0.5 * x0 + (xe + xw + xn + xs + xne + xsw) * (1.0 / 12.0));
        if (own && j <= jo) {
            un[zo + (long)j * p + col] = x0;
            ua += x0 * Ax;
            um += x0 * Mx;
        }
        // A un, M un one lane to each side (the coarse node's W, SW and E, NE)
        const double aP = lane_prev(Ax), aX = lane_next(Ax), mP = lane_prev(Mx), mX = lane_next(Mx);
        const bool odd = (j & 1) != 0;
        const int Jd = (j - 1) / 2;  // an odd row 2 J - 1 completes coarse row J - 1
        if (odd && Jd >= J0 && cown) {
            const long cid = zq + (long)Jd * pc + ccol;
            bc[cid] = aC + 0.5 * (aWE + aS + (Ax + aX));
            cc[cid] = mC + 0.5 * (mWE + mS + (Mx + mX));
        }
        // selects, not branches: the state stays in registers
        aS = odd ? Ax + aP : aS;
        mS = odd ? Mx + mP : mS;
        aC = odd ? aC : Ax;
        mC = odd ? mC : Mx;
        aWE = odd ? aWE : aP + aX;
        mWE = odd ? mWE : mP + mX;
    };
    // whole bodies of RNS rows, then the remaining rows (the loop carries no
    // early exit, so no wait drains the rows in flight)
    int jb = ja;
    for (; jb + RNS <= jb1 + 1; jb += RNS) {
#pragma unroll
        for (int q = 0; q < RNS; ++q) step(q, jb + q);
    }
#pragma unroll
    for (int q = 0; q < RNS - 1; ++q)
        if (jb + q < jb1 + 1) step(q, jb + q);
    for (int o = RL / 2; o > 0; o /= 2) {
        ua += __shfl_down(ua, o, RL);
        um += __shfl_down(um, o, RL);
    }
    if (lane == 0) {
        const long b = ((long)z * rw.bands + band) * rw.strips + strip;
        partial[2 * b] = ua;
        partial[2 * b + 1] = um;
    }
}

int row_slots() {
    int dev = 0, cus = 0, per_cu = 0;
    PASM_HIP(hipGetDevice(&dev));
    PASM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PASM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_border_rows<false>, RL * RWG, 0));
    return std::max(1, cus * per_cu * RWG);
}

// Bands over `units` coarse rows: the height that minimises rounds of
// resident wavefronts x rows walked (each band walks one coarse row more than
// it owns), with at most `maxbands` bands and at least 8 rows each.
RowWork row_shape(int strips, int units, int nrhs, int slots, int maxbands) {
    RowWork rw{};
    rw.strips = strips;
    double best = -1.0;
    for (int b = 1; b <= std::max(1, maxbands); ++b) {
        const int rows = (units + b - 1) / b;
        if (b > 1 && rows < 8) break;
        const int bands = (units + rows - 1) / rows;
        const long pieces = (long)strips * bands * nrhs;
        const long rounds = (pieces + slots - 1) / slots;
        const double cost = (double)rounds * (rows + 1);
        if (best < 0.0 || cost < best) {
            best = cost;
            rw.rows = rows;
            rw.bands = bands;
        }
    }
    rw.work = strips * rw.bands * nrhs;
    return rw;
}

}  // namespace

bool rows_supported(const Grid& g, const Coef<double>& c) {
    return g.dim == 2 && coef_kind(c) == 1 && c.kpm <= 1 && c.ms == 0 && g.n >= 4;
}

int launch_border_rows(const Grid& g, const Coef<double>& c, const double* u, const float* e, double* un,
                       const Grid& gc, double* bc, double* cc, double* partial, int nrhs, long stride, long sc,
                       long max_blocks, hipStream_t st, const float* e0) {
    if (!rows_supported(g, c) || gc.n * 2 != g.n || un == u)
        throw Error(PASM_E_INVALID, "row-marching borders: 2D edge weights, ratio 2, separate output");
    static const int slots = row_slots();
    const int strips = (g.m + BOWN - 1) / BOWN;
    const int maxb = (int)std::max<long>(1, max_blocks / strips);
    const RowWork rw = row_shape(strips, gc.m, nrhs, slots, maxb);
    if ((long)strips * rw.bands > max_blocks) throw Error(PASM_E_INVALID, "row-marching borders: partial sums");
    const int wgs = (rw.work + RWG - 1) / RWG;
    const dim3 grid((wgs + RXCD - 1) / RXCD * RXCD), blk(RL * RWG);
    if (e0)
        hipLaunchKernelGGL(k_border_rows<true>, grid, blk, 0, st, g, c.wx, c.wy, u, e, e0, un, gc, bc, cc, partial,
                           stride, sc, rw);
    else
        hipLaunchKernelGGL(k_border_rows<false>, grid, blk, 0, st, g, c.wx, c.wy, u, e, (const float*)nullptr, un, gc,
                           bc, cc, partial, stride, sc, rw);
    PASM_CHECK_LAUNCH();
    return strips * rw.bands;
}

}  // namespace pasm

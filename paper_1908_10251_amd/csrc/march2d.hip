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
//         x_0 = x + P e_c.
// Steps follow x_{t+1} = x_t + a_t (x_t - x_{t-1}) + b_t D^{-1} (f - A x_t)
// with a_0 = 0 (a phase starts fresh).
#include "common.h"

namespace pasm {

namespace {

constexpr int NL = 64;      // lanes per wavefront
constexpr int MW = 2 * NL;  // strip width: each lane owns two adjacent columns
constexpr int MSEG = 64;    // rows owned by one wavefront (even)
constexpr int MWAVES = 4;   // wavefronts per workgroup (consecutive segments)
constexpr int PF = 3;       // rows loaded ahead of the one being processed

// Cross-lane moves of a double by one lane (DPP wave shifts; the lane at the
// wavefront edge receives 0, which only ever reaches halo columns).
__device__ inline double from_left(double v) {  // value of lane l - 1
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double from_right(double v) {  // value of lane l + 1
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ inline float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

template <typename T, int S, int MODE>
__global__ __launch_bounds__(NL* MWAVES) void k_march(Grid g, T w0, const T* __restrict__ x0,
                                                      const T* __restrict__ f, T* __restrict__ out,
                                                      const T* __restrict__ ec, Grid gc, T* __restrict__ rc, long sf,
                                                      long sc, SmoothSteps st, int x_zero) {
    constexpr int HX = S + 2;
    constexpr int TXO = MW - 2 * HX;
    const int lane = threadIdx.x;
    const int y0 = (blockIdx.y * MWAVES + threadIdx.y) * MSEG;
    if (y0 > g.n) return;  // uniform per wavefront
    const int c0 = 2 * lane;                      // strip column of the lane's first column
    const int i0 = blockIdx.x * TXO - HX + c0;    // global column (even)
    bool inner[2], owned[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        inner[cc] = (i0 + cc) >= 1 && (i0 + cc) <= g.m;
        owned[cc] = (c0 + cc) >= HX && (c0 + cc) < MW - HX;
    }
    const long off = (long)blockIdx.z * sf;
    const T* xr = x0 + off;
    const T* fr = f + off;
    T* outr = out + off;
    const T* ecr = ec + (long)blockIdx.z * sc;
    const T invD = T(1) / (T(4) * w0);
    T bs[S], as[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        bs[t] = (T)st.b[t] * invD;
        as[t] = (T)st.a[t];
    }

    T xw[S + 1][3][2];
    T fw[S + 2][2];
    T rw[3][2];
#pragma unroll
    for (int t = 0; t <= S; ++t)
#pragma unroll
        for (int k = 0; k < 3; ++k) xw[t][k][0] = xw[t][k][1] = T(0);
#pragma unroll
    for (int j = 0; j < S + 2; ++j) fw[j][0] = fw[j][1] = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) rw[k][0] = rw[k][1] = T(0);

    const int r_begin = y0 - 2 - S;
    const int r_end = y0 + MSEG + S;

    // Loads are branch-free so that rows requested PF steps ahead stay in
    // flight: positions outside the grid are clamped onto the boundary ring,
    // whose stored values are zero (the Dirichlet data), which is exactly the
    // value such positions must have.
    const int ia = min(max(i0, 0), g.n), ib = min(max(i0 + 1, 0), g.n);
    auto prolong_at = [&](int i, int r) -> T {
        // nodal interpolation of the coarse correction at fine node (i, r):
        // the mean of coarse nodes (I, J) and (I + a, J + b); for a = b = 0 both
        // reads are the same node and the mean is exact, so there is no branch
        const int a = i & 1, b = r & 1;
        const long cid = gc.idx(i >> 1, r >> 1);
        return T(0.5) * (ecr[cid] + ecr[cid + a + (long)b * gc.pitch]);
    };
    auto load = [&](int r, T* xv, T* fv) {
        const int rr = min(max(r, 0), g.n);
        const long row = (long)rr * g.pitch + ORIGIN;
        fv[0] = fr[row + ia];
        fv[1] = fr[row + ib];
        if (MODE == 2) {
            xv[0] = xr[row + ia] + prolong_at(ia, rr);
            xv[1] = xr[row + ib] + prolong_at(ib, rr);
        } else if (!x_zero) {
            xv[0] = xr[row + ia];
            xv[1] = xr[row + ib];
        } else {
            xv[0] = xv[1] = T(0);
        }
    };

    T qx[PF][2], qf[PF][2];
#pragma unroll
    for (int p = 0; p < PF; ++p) load(r_begin + p, qx[p], qf[p]);

    for (int r = r_begin; r <= r_end; ++r) {
        T cx[2] = {qx[0][0], qx[0][1]}, cf[2] = {qf[0][0], qf[0][1]};
#pragma unroll
        for (int p = 0; p < PF - 1; ++p) {
            qx[p][0] = qx[p + 1][0];
            qx[p][1] = qx[p + 1][1];
            qf[p][0] = qf[p + 1][0];
            qf[p][1] = qf[p + 1][1];
        }
        load(r + PF, qx[PF - 1], qf[PF - 1]);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
#pragma unroll
            for (int j = S + 1; j > 0; --j) fw[j][cc] = fw[j - 1][cc];
            fw[0][cc] = cf[cc];
            xw[0][2][cc] = xw[0][1][cc];
            xw[0][1][cc] = xw[0][0][cc];
            xw[0][0][cc] = cx[cc];
        }
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
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const T Ax = w0 * (T(4) * mc[cc] - nb[cc]);
                T val = mc[cc] + bs[t - 1] * (fw[t][cc] - Ax);
                if (t >= 2) val += as[t - 1] * (mc[cc] - xw[t - 2][2][cc]);
                v[cc] = (row_in && inner[cc]) ? val : T(0);
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
                const long id = g.idx(i0, q);
#pragma unroll
                for (int cc = 0; cc < 2; ++cc)
                    if (owned[cc] && inner[cc]) outr[id + cc] = xw[S][0][cc];
            }
        }
        if (MODE == 1) {
            // residual at row r - S - 1 from x_S rows (r-S, r-S-1, r-S-2)
            const int q1 = r - S - 1;
            const bool row_in = q1 >= 1 && q1 <= g.m;
            const T m0 = xw[S][1][0], m1 = xw[S][1][1];
            const T left = from_left(m1), right = from_right(m0);
            const T nb0 = left + m1 + xw[S][0][0] + xw[S][2][0];
            const T nb1 = m0 + right + xw[S][0][1] + xw[S][2][1];
            T res0 = fw[S + 1][0] - w0 * (T(4) * m0 - nb0);
            T res1 = fw[S + 1][1] - w0 * (T(4) * m1 - nb1);
            res0 = (row_in && inner[0]) ? res0 : T(0);
            res1 = (row_in && inner[1]) ? res1 : T(0);
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
                    rc[(long)blockIdx.z * sc + gc.idx(I, J)] =
                        rw[1][0] + T(0.5) * (rw[1][1] + mid_left + rw[0][0] + rw[2][0] + rw[0][1] + dn_left);
            }
        }
    }
}

template <typename T, int S, int MODE>
void march_launch(const Grid& g, T w0, const T* x0, const T* f, T* out, const T* ec, const Grid& gc, T* rc,
                  int nrhs, long sf, long sc, const SmoothSteps& ss, bool x_zero, hipStream_t st) {
    constexpr int TXO = MW - 2 * (S + 2);
    const int strips = (g.n + 1 + TXO - 1) / TXO;
    const int segs = (g.n + 1 + MSEG - 1) / MSEG;
    dim3 grid(strips, (segs + MWAVES - 1) / MWAVES, nrhs);
    hipLaunchKernelGGL((k_march<T, S, MODE>), grid, dim3(NL, MWAVES), 0, st, g, w0, x0, f, out, ec, gc, rc, sf, sc,
                       ss, (int)x_zero);
    PASM_CHECK_LAUNCH();
}

template <typename T, int MODE>
void march_dispatch(const Grid& g, T w0, const T* x0, const T* f, T* out, const T* ec, const Grid& gc, T* rc,
                    int nrhs, long sf, long sc, const SmoothSteps& ss, bool x_zero, hipStream_t st) {
    switch (ss.s) {
        case 1: march_launch<T, 1, MODE>(g, w0, x0, f, out, ec, gc, rc, nrhs, sf, sc, ss, x_zero, st); break;
        case 2: march_launch<T, 2, MODE>(g, w0, x0, f, out, ec, gc, rc, nrhs, sf, sc, ss, x_zero, st); break;
        case 3: march_launch<T, 3, MODE>(g, w0, x0, f, out, ec, gc, rc, nrhs, sf, sc, ss, x_zero, st); break;
        case 4: march_launch<T, 4, MODE>(g, w0, x0, f, out, ec, gc, rc, nrhs, sf, sc, ss, x_zero, st); break;
        default: throw Error(PASM_E_INVALID, "marching smoother supports 1..4 steps");
    }
}

}  // namespace

// Large 2D levels only: a wavefront walks 64 + 2(S+2) rows in sequence, which
// needs many strips and segments to fill the machine; smaller levels use the
// tile kernels.
bool march_supported(const Grid& g, bool const_coef, int steps) {
    return g.dim == 2 && const_coef && steps >= 1 && steps <= 4 && g.n >= 512;
}

template <typename T>
void launch_march_pre(const Grid& g, T w0, const T* x0, const T* f, T* out, const Grid& gc, T* rc, int nrhs,
                      const SmoothSteps& ss, bool x_zero, hipStream_t st) {
    march_dispatch<T, 1>(g, w0, x0, f, out, (const T*)nullptr, gc, rc, nrhs, g.plane, gc.plane, ss, x_zero, st);
}

template <typename T>
void launch_march_post(const Grid& g, T w0, const T* x, const T* f, T* out, const Grid& gc, const T* ec, int nrhs,
                       const SmoothSteps& ss, hipStream_t st) {
    march_dispatch<T, 2>(g, w0, x, f, out, ec, gc, (T*)nullptr, nrhs, g.plane, gc.plane, ss, false, st);
}

template void launch_march_pre<double>(const Grid&, double, const double*, const double*, double*, const Grid&,
                                       double*, int, const SmoothSteps&, bool, hipStream_t);
template void launch_march_pre<float>(const Grid&, float, const float*, const float*, float*, const Grid&, float*,
                                      int, const SmoothSteps&, bool, hipStream_t);
template void launch_march_post<double>(const Grid&, double, const double*, const double*, double*, const Grid&,
                                        const double*, int, const SmoothSteps&, hipStream_t);
template void launch_march_post<float>(const Grid&, float, const float*, const float*, float*, const Grid&,
                                       const float*, int, const SmoothSteps&, hipStream_t);

}  // namespace pasm

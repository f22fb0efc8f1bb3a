// Moment observables of a field (Sec. 5): centre of mass (eq. CoM), RMS
// radius (eq. RMS radius), the inertia tensors U, V, W (eqs. U, V, W inertia
// tensor), the isospin-0 quadrupole (eq. Q tensor) and the D-term (eq. D-term
// with the static stress tensor of eq. Stress tensor).
//
// Two passes over the interior I, one thread per site, FP64 arithmetic from
// the stored field: pass 1 sums the charge density b and its first moments and
// fixes the centre X_c on the device; pass 2 sums the tensor densities in the
// frame r = x - X_c.  Per-block partial sums are reduced in a fixed order, so
// the result is deterministic.
//
// The traces of the printed formulas are evaluated in the vector form of
// su(2): with X = x0 + i x.tau, Tr(XY) = 2 (x0 y0 - x.y) and a commutator
// [X, Y] = i (-2 x cross y).tau, so Tr([X, Z][Y, W]) = -8 (x cross z).(y cross w).
// L_k = U^dagger d_k U has scalar part s_k = phi . a_k and vector part
// l_k = phi0 a_k - a_k^0 phi + phi cross a_k (3-vector parts); T_j =
// (i/2) U^dagger [tau^j, U] is pure with vector t_j = -phi0 (e_j cross phi)
// - |phi|^2 e_j + phi_j phi.  With the Gram matrices G = (l_m . l_p), S = tr G,
// Mx = (l_k . t_i) the densities are
//   U_ij: 2 (1 + S) t_i.t_j - 2 (Mx^T Mx)_ij
//   K    = 2 (G - s s^T) + 2 (S G - G^2)   (the stress tensor without its delta_ij part)
//   V   = R K R^T, R v = r cross v
//   W_ij: -2 (R N)_ji, N = (1 + S) Mx - G Mx
//   D   : r.K.r - |r|^2 tr K / 3
// Quantities use the printed (un-halved) normalisation of the Lagrangian.
#pragma once

#include <hip/hip_runtime.h>

namespace skyr {

constexpr int MOM_THREADS = 256;
constexpr int MOM_MAX_BLOCKS = 1024;
constexpr int MOM_NACC = 32;  // partial-sum slots per block (pass 2 uses 28)
constexpr int MOM_PASS_CENTRE = 1;
constexpr int MOM_PASS_TENSORS = 2;

// device result record: {B, E, X[3], R, U[9], V[9], W[9], Q[9], D}
constexpr int MOM_OUT_DOUBLES = 43;

struct MomArgs {
    const void* phi;
    int n0, n1, n2;
    double h;
    double* partials;      // [gridDim.x][MOM_NACC]
    double* centre;        // 4 doubles: sum b, X_c (written by pass 1, read by pass 2)
    const double* obs;     // library observables; obs[0] = E (halved normalisation)
    double* out;           // MOM_OUT_DOUBLES
};

template <int PASS> struct MomAcc {
    static constexpr int N = PASS == MOM_PASS_CENTRE ? 4 : 28;
};

template <typename T, int PASS>
__global__ __launch_bounds__(MOM_THREADS) void moments_kernel(MomArgs a)
{
    constexpr int NA = MomAcc<PASS>::N;
    const T* __restrict__ phi = (const T*)a.phi;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const size_t sy = (size_t)n2, sx = (size_t)n1 * n2, N3 = (size_t)n0 * sx;
    const int ni1 = n1 - 4, ni2 = n2 - 4;
    const long long nI = (long long)(n0 - 4) * ni1 * ni2;
    const double h = a.h, inv12h = 1.0 / (12.0 * h);
    const double cb0 = 0.5 * (n0 - 1), cb1 = 0.5 * (n1 - 1), cb2 = 0.5 * (n2 - 1);
    double Xc0 = 0.0, Xc1 = 0.0, Xc2 = 0.0;
    if constexpr (PASS == MOM_PASS_TENSORS) {
        Xc0 = a.centre[1];
        Xc1 = a.centre[2];
        Xc2 = a.centre[3];
    }
    double acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;

    for (long long q = (long long)blockIdx.x * MOM_THREADS + threadIdx.x; q < nI;
         q += (long long)gridDim.x * MOM_THREADS) {
        const int z = 2 + (int)(q % ni2);
        const long long yx = q / ni2;
        const int y = 2 + (int)(yx % ni1);
        const int x = 2 + (int)(yx / ni1);
        const size_t s = (size_t)x * sx + (size_t)y * sy + (size_t)z;
        double p[4], d[3][4];
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            const T* c = phi + (size_t)A * N3 + s;
            p[A] = (double)c[0];
            // fourth-order first difference (Sec. 3): (f(-2) - 8 f(-1) + 8 f(+1) - f(+2)) / 12h
            d[0][A] = ((double)c[-2 * (long long)sx] - 8.0 * (double)c[-(long long)sx] + 8.0 * (double)c[sx] -
                       (double)c[2 * sx]) * inv12h;
            d[1][A] = ((double)c[-2 * (long long)sy] - 8.0 * (double)c[-(long long)sy] + 8.0 * (double)c[sy] -
                       (double)c[2 * sy]) * inv12h;
            d[2][A] = ((double)c[-2] - 8.0 * (double)c[-1] + 8.0 * (double)c[1] - (double)c[2]) * inv12h;
        }
        const double b = -det4(p, d[0], d[1], d[2]) * (1.0 / (2.0 * M_PI * M_PI));
        const double X0 = (x - cb0) * h, X1 = (y - cb1) * h, X2 = (z - cb2) * h;
        if constexpr (PASS == MOM_PASS_CENTRE) {
            acc[0] += b;
            acc[1] += X0 * b;
            acc[2] += X1 * b;
            acc[3] += X2 * b;
        } else {
            const double r[3] = {X0 - Xc0, X1 - Xc1, X2 - Xc2};
            // charge moments: xx yy zz xy xz yz
            acc[0] += r[0] * r[0] * b;
            acc[1] += r[1] * r[1] * b;
            acc[2] += r[2] * r[2] * b;
            acc[3] += r[0] * r[1] * b;
            acc[4] += r[0] * r[2] * b;
            acc[5] += r[1] * r[2] * b;
            // currents
            const double p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
            double sk[3], l[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double* e = d[k];
                sk[k] = p0 * e[0] + p1 * e[1] + p2 * e[2] + p3 * e[3];
                l[k][0] = p0 * e[1] - e[0] * p1 + (p2 * e[3] - p3 * e[2]);
                l[k][1] = p0 * e[2] - e[0] * p2 + (p3 * e[1] - p1 * e[3]);
                l[k][2] = p0 * e[3] - e[0] * p3 + (p1 * e[2] - p2 * e[1]);
            }
            const double pv2 = p1 * p1 + p2 * p2 + p3 * p3;
            const double t[3][3] = {{p1 * p1 - pv2, p0 * p3 + p1 * p2, p1 * p3 - p0 * p2},
                                    {p1 * p2 - p0 * p3, p2 * p2 - pv2, p0 * p1 + p2 * p3},
                                    {p0 * p2 + p1 * p3, p2 * p3 - p0 * p1, p3 * p3 - pv2}};
            double G[3][3], Mx[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    G[i][j] = l[i][0] * l[j][0] + l[i][1] * l[j][1] + l[i][2] * l[j][2];
                    Mx[i][j] = l[i][0] * t[j][0] + l[i][1] * t[j][1] + l[i][2] * t[j][2];
                }
            const double S = G[0][0] + G[1][1] + G[2][2];
            // U (symmetric): xx yy zz xy xz yz
            const int iu[6] = {0, 1, 2, 0, 0, 1}, ju[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int i = iu[e], j = ju[e];
                const double tt = t[i][0] * t[j][0] + t[i][1] * t[j][1] + t[i][2] * t[j][2];
                const double mm = Mx[0][i] * Mx[0][j] + Mx[1][i] * Mx[1][j] + Mx[2][i] * Mx[2][j];
                acc[6 + e] += 2.0 * (1.0 + S) * tt - 2.0 * mm;
            }
            // K = 2 (G - s s^T) + 2 (S G - G^2)
            double K[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double gg = G[i][0] * G[0][j] + G[i][1] * G[1][j] + G[i][2] * G[2][j];
                    K[i][j] = 2.0 * (G[i][j] - sk[i] * sk[j]) + 2.0 * (S * G[i][j] - gg);
                }
            // R v = r cross v
            const double R[3][3] = {{0.0, -r[2], r[1]}, {r[2], 0.0, -r[0]}, {-r[1], r[0], 0.0}};
            double RK[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) RK[i][j] = R[i][0] * K[0][j] + R[i][1] * K[1][j] + R[i][2] * K[2][j];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int i = iu[e], j = ju[e];
                acc[12 + e] += RK[i][0] * R[j][0] + RK[i][1] * R[j][1] + RK[i][2] * R[j][2];
            }
            // N = (1 + S) Mx - G Mx; W_ij = -2 sum_m R_jm N_mi
            double N[3][3];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    N[m][i] = (1.0 + S) * Mx[m][i] - (G[m][0] * Mx[0][i] + G[m][1] * Mx[1][i] + G[m][2] * Mx[2][i]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    acc[18 + 3 * i + j] += -2.0 * (R[j][0] * N[0][i] + R[j][1] * N[1][i] + R[j][2] * N[2][i]);
            // D-term moment: r.K.r - |r|^2 tr K / 3
            double rKr = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) rKr += r[i] * (K[i][0] * r[0] + K[i][1] * r[1] + K[i][2] * r[2]);
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            acc[27] += rKr - r2 * (K[0][0] + K[1][1] + K[2][2]) * (1.0 / 3.0);
        }
    }

    // fixed-order block reduction: wave shuffles, then the four waves in order
    __shared__ double red[MOM_THREADS / 64][NA];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NA) {
        const int k = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < MOM_THREADS / 64; ++w) v += red[w][k];
        a.partials[(size_t)blockIdx.x * MOM_NACC + k] = v;
    }
}

// sum of slot k over nblocks records, thread t taking blocks t, t + 256, ...
// then a fixed tree; every thread returns the total
__device__ static double mom_reduce_slot(const double* __restrict__ part, int nblocks, int k, double* red)
{
    const int t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblocks; b += MOM_THREADS) s += part[(size_t)b * MOM_NACC + k];
    red[t] = s;
    __syncthreads();
    for (int w = MOM_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double total = red[0];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(MOM_THREADS) void moments_centre_kernel(MomArgs a, int nblocks)
{
    __shared__ double red[MOM_THREADS];
    double s[4];
    for (int k = 0; k < 4; ++k) s[k] = mom_reduce_slot(a.partials, nblocks, k, red);
    if (threadIdx.x == 0) {
        a.centre[0] = s[0];
        a.centre[1] = s[1] / s[0];
        a.centre[2] = s[2] / s[0];
        a.centre[3] = s[3] / s[0];
    }
}

__global__ __launch_bounds__(MOM_THREADS) void moments_finish_kernel(MomArgs a, int nblocks)
{
    __shared__ double red[MOM_THREADS];
    double s[28];
    for (int k = 0; k < 28; ++k) s[k] = mom_reduce_slot(a.partials, nblocks, k, red);
    if (threadIdx.x != 0) return;
    const double h3 = a.h * a.h * a.h;
    const double B = h3 * a.centre[0];
    const double E = 2.0 * a.obs[0];  // printed normalisation
    double* o = a.out;
    o[0] = B;
    o[1] = E;
    o[2] = a.centre[1];
    o[3] = a.centre[2];
    o[4] = a.centre[3];
    const int iu[6] = {0, 1, 2, 0, 0, 1}, ju[6] = {0, 1, 2, 1, 2, 2};
    double Mom[3][3];
    for (int e = 0; e < 6; ++e) Mom[iu[e]][ju[e]] = Mom[ju[e]][iu[e]] = h3 * s[e];
    const double trM = Mom[0][0] + Mom[1][1] + Mom[2][2];
    o[5] = sqrt(trM / B);
    double* U = o + 6;
    double* V = o + 15;
    double* W = o + 24;
    double* Q = o + 33;
    for (int e = 0; e < 6; ++e) {
        const int i = iu[e], j = ju[e];
        U[3 * i + j] = U[3 * j + i] = h3 * s[6 + e];
        V[3 * i + j] = V[3 * j + i] = h3 * s[12 + e];
    }
    for (int e = 0; e < 9; ++e) W[e] = h3 * s[18 + e];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q[3 * i + j] = 0.5 * (3.0 * Mom[i][j] - (i == j ? trM : 0.0));
    o[42] = -(2.0 * E / 5.0) * h3 * s[27];
}

// kinetic energy: per-block sums of |v|^2 over I (slot 0 of the partial records)
template <typename T>
__global__ __launch_bounds__(MOM_THREADS) void kinetic_kernel(const T* __restrict__ vel, int n0, int n1, int n2,
                                                              double* __restrict__ partials)
{
    const size_t sy = (size_t)n2, sx = (size_t)n1 * n2, N3 = (size_t)n0 * sx;
    const int ni1 = n1 - 4, ni2 = n2 - 4;
    const long long nI = (long long)(n0 - 4) * ni1 * ni2;
    double acc = 0.0;
    for (long long q = (long long)blockIdx.x * MOM_THREADS + threadIdx.x; q < nI;
         q += (long long)gridDim.x * MOM_THREADS) {
        const int z = 2 + (int)(q % ni2);
        const long long yx = q / ni2;
        const int y = 2 + (int)(yx % ni1);
        const int x = 2 + (int)(yx / ni1);
        const size_t s = (size_t)x * sx + (size_t)y * sy + (size_t)z;
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            const double v = (double)vel[(size_t)A * N3 + s];
            acc += v * v;
        }
    }
    __shared__ double red[MOM_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < MOM_THREADS / 64; ++w) v += red[w];
        partials[(size_t)blockIdx.x * MOM_NACC] = v;
    }
}

__global__ __launch_bounds__(MOM_THREADS) void kinetic_finish_kernel(const double* __restrict__ partials, int nblocks,
                                                                     double h, double* __restrict__ out)
{
    __shared__ double red[MOM_THREADS];
    const double s = mom_reduce_slot(partials, nblocks, 0, red);
    if (threadIdx.x == 0) out[0] = 0.5 * h * h * h * s;
}

}  // namespace skyr

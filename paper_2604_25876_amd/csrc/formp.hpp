// Printed-form flow sweep: the force from the paper's Euler-Lagrange
// expression (Sec. 3, eq. Sigma model EL equations, halved to this library's
// energy normalisation) instead of the exact derivative of the discrete energy:
//   g = -{ (1 + S) Lap phi + sum_i c_i a_i - sum_ij G_ij D_i D_j phi } + V'(phi0) e_0,
//   a_i = D_i phi, G_ij = a_i . a_j, S = tr G, Lap = sum_i D_ii phi,
//   c_i = sum_j (D_i D_j phi) . a_j - Lap . a_i,
// with the five-point second difference D_ii and the mixed derivative D_i D_j
// as the product of two first-difference stencils (radius 2 in each of its
// two directions).  The stencil is one-stage: g at a site depends on phi
// within the 5 x 5 x 5 box around it, so there is no flux pass.  Everything
// else (energy density for the arrest test, projection, kick-drift update,
// renormalisation, partial sums) is that of the exact-gradient sweep.
//
// 2.5D march: a block owns a 16 x 16 (y, z) tile and a slab of x; a ring of
// five phi planes with a two-site halo lives in LDS (plane x + 2 replaces
// plane x - 3), one thread per (y, z) column, two barriers per plane.
#pragma once

#include "sweep.hpp"

namespace skyr {

constexpr int FP_TY = 16, FP_TZ = 16, FP_THREADS = FP_TY * FP_TZ;
constexpr int FP_H = FP_TY + 4, FP_W = FP_TZ + 4;
constexpr int FP_XCHUNK = 32;  // planes per slab

__host__ __device__ inline int formp_tiles(int n1, int n2) { return ((n1 - 4 + FP_TY - 1) / FP_TY) * ((n2 - 4 + FP_TZ - 1) / FP_TZ); }
__host__ __device__ inline int formp_blocks(int n0, int n1, int n2)
{
    return formp_tiles(n1, n2) * ((n0 - 4 + FP_XCHUNK - 1) / FP_XCHUNK);
}

template <typename T> struct FormPSmem {
    T phi[5][4][FP_H][FP_W];
    double red[FP_THREADS / 64][7];
};

template <typename T, int MODE, bool EXT>
__global__ __launch_bounds__(FP_THREADS) void formp_kernel(SweepArgs a)
{
    __shared__ FormPSmem<T> sm;
    const Ctl* ctl = a.ctl;
    int cur = 0;
    bool redo = false, renorm64 = false;
    if constexpr (MODE == MODE_STEP) {
        if (ctl->done) return;  // uniform
        cur = ctl->cur;
        redo = ctl->redo != 0;
        const int kr = ctl->renorm64_every;
        renorm64 = (kr > 0) && (((ctl->steps + 1) % kr) == 0);
    }
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const size_t N3 = (size_t)n0 * n1 * n2, plane = (size_t)n1 * n2;
    const T* __restrict__ pin = (const T*)(MODE == MODE_STEP && cur ? (const void*)a.phi1 : a.phi0);
    T* __restrict__ pout = (T*)(MODE == MODE_STEP ? (cur ? (void*)a.phi0 : a.phi1) : nullptr);
    T* __restrict__ vel = (T*)a.vel;
    T* __restrict__ gout = (T*)a.grad;

    const int tz_tiles = (n2 - 4 + FP_TZ - 1) / FP_TZ;
    const int tiles = formp_tiles(n1, n2);
    const int slab = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int y0 = 2 + (tile / tz_tiles) * FP_TY, z0 = 2 + (tile % tz_tiles) * FP_TZ;
    const int xb = 2 + slab * a.xchunk, xe = min(n0 - 2, xb + a.xchunk);
    const int tid = threadIdx.x, ly = tid / FP_TZ, lz = tid % FP_TZ;
    const int y = y0 + ly, z = z0 + lz;
    const bool out = (y <= n1 - 3) && (z <= n2 - 3);

    const T c1h = T(Coef<double>::c1 / a.h), c2h = T(Coef<double>::c2 / a.h);
    const T d1h = T(Coef<double>::d1 / (a.h * a.h)), d2h = T(Coef<double>::d2 / (a.h * a.h));
    const T c1 = Coef<T>::c1, c2 = Coef<T>::c2;
    const T ih2 = T(1.0 / (a.h * a.h));
    const T dt = T(a.dt);
    const T m2 = T(a.m * a.m), my2 = T(a.m_y * a.m_y), mz2 = T(a.m_z * a.m_z), mw2 = T(a.m_w * a.m_w);
    const bool grad_flow = MODE == MODE_STEP && a.gradient_flow != 0;
    const bool has_grad = gout != nullptr, projected = a.projected != 0, baryon = a.baryon != 0;

    double pe2 = 0.0, pe4 = 0.0, pe0 = 0.0, pb = 0.0, pp = 0.0;
    T pf2 = T(0);

    // the plane-load pattern is the same for every plane: thread tid moves elements
    // tid + 256 k of the 4 x FP_H x FP_W halo tile; its source offsets within a plane
    // (component, clamped y and z) and LDS positions are fixed up front
    constexpr int NE = 4 * FP_H * FP_W, NK = (NE + FP_THREADS - 1) / FP_THREADS;
    unsigned goff[NK];
    int loff[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int e = min(tid + k * FP_THREADS, NE - 1);
        const int A = e / (FP_H * FP_W), rem = e % (FP_H * FP_W);
        const int ry = rem / FP_W, rz = rem % FP_W;
        const int gy = clampi(y0 - 2 + ry, 0, n1 - 1), gz = clampi(z0 - 2 + rz, 0, n2 - 1);
        goff[k] = (unsigned)(A * N3) + (unsigned)(gy * n2 + gz);
        loff[k] = e;
    }
    auto load_plane = [&](int x) {
        T* dst = &sm.phi[x % 5][0][0][0];  // x >= 0
        const T* src = pin + (size_t)clampi(x, 0, n0 - 1) * plane;
#pragma unroll
        for (int k = 0; k < NK; ++k)
            if (k < NK - 1 || tid + k * FP_THREADS < NE) dst[loff[k]] = src[goff[k]];
    };

    if (xb < xe) {
        for (int x = xb - 2; x <= xb + 1; ++x) load_plane(x);
        for (int x = xb; x < xe; ++x) {
            load_plane(x + 2);
            __syncthreads();
            if (out) {
                const int sm2 = (x - 2) % 5, sm1 = (x - 1) % 5, s0 = x % 5, sp1 = (x + 1) % 5, sp2 = (x + 2) % 5;
                const int r = ly + 2, q = lz + 2;
                // pass 1: centre values and first derivatives, then the Gram matrix
                T c[4], ax[4], ay[4], az[4];
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    const T(*P0)[FP_W] = sm.phi[s0][A];
                    c[A] = P0[r][q];
                    ax[A] = c1h * (sm.phi[sp1][A][r][q] - sm.phi[sm1][A][r][q]) +
                            c2h * (sm.phi[sp2][A][r][q] - sm.phi[sm2][A][r][q]);
                    ay[A] = c1h * (P0[r + 1][q] - P0[r - 1][q]) + c2h * (P0[r + 2][q] - P0[r - 2][q]);
                    az[A] = c1h * (P0[r][q + 1] - P0[r][q - 1]) + c2h * (P0[r][q + 2] - P0[r][q - 2]);
                }
                const T gxx = dot4(ax, ax), gyy = dot4(ay, ay), gzz = dot4(az, az);
                const T gxy = dot4(ax, ay), gxz = dot4(ax, az), gyz = dot4(ay, az);
                const T S = gxx + gyy + gzz;
                // pass 2, one component at a time: the second derivatives of component A give
                //   u_A = (1 + S) Lap_A - sum_ij G_ij (D_i D_j phi)_A,  lap_A,
                // and their contributions to c_i = sum_j (D_i D_j phi) . a_j - Lap . a_i
                T uu[4], lap[4];
                T cx = T(0), cy = T(0), cz = T(0);
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    const T(*P0)[FP_W] = sm.phi[s0][A];
                    const T cc = c[A];
                    auto second = [&](T m2v, T m1v, T p1v, T p2v) {
                        return d1h * ((p1v - cc) + (m1v - cc)) + d2h * ((p2v - cc) + (m2v - cc));
                    };
                    const T dxx = second(sm.phi[sm2][A][r][q], sm.phi[sm1][A][r][q], sm.phi[sp1][A][r][q],
                                         sm.phi[sp2][A][r][q]);
                    const T dyy = second(P0[r - 2][q], P0[r - 1][q], P0[r + 1][q], P0[r + 2][q]);
                    const T dzz = second(P0[r][q - 2], P0[r][q - 1], P0[r][q + 1], P0[r][q + 2]);
                    // D_x D_y: the y-difference on the four x-neighbour planes, then the x-difference
                    auto dy_on = [&](int sl) {
                        const T(*Pl)[FP_W] = sm.phi[sl][A];
                        return c1 * (Pl[r + 1][q] - Pl[r - 1][q]) + c2 * (Pl[r + 2][q] - Pl[r - 2][q]);
                    };
                    auto dz_on = [&](int sl, int rr) {
                        const T* row = sm.phi[sl][A][rr];
                        return c1 * (row[q + 1] - row[q - 1]) + c2 * (row[q + 2] - row[q - 2]);
                    };
                    const T dxy = ih2 * (c1 * (dy_on(sp1) - dy_on(sm1)) + c2 * (dy_on(sp2) - dy_on(sm2)));
                    const T dxz = ih2 * (c1 * (dz_on(sp1, r) - dz_on(sm1, r)) + c2 * (dz_on(sp2, r) - dz_on(sm2, r)));
                    const T dyz =
                        ih2 * (c1 * (dz_on(s0, r + 1) - dz_on(s0, r - 1)) + c2 * (dz_on(s0, r + 2) - dz_on(s0, r - 2)));
                    const T la = dxx + dyy + dzz;
                    lap[A] = la;
                    uu[A] = (T(1) + S) * la - (gxx * dxx + gyy * dyy + gzz * dzz +
                                               T(2) * (gxy * dxy + gxz * dxz + gyz * dyz));
                    cx += dxx * ax[A] + dxy * ay[A] + dxz * az[A] - la * ax[A];
                    cy += dxy * ax[A] + dyy * ay[A] + dyz * az[A] - la * ay[A];
                    cz += dxz * ax[A] + dyz * ay[A] + dzz * az[A] - la * az[A];
                }
                const T u = T(1) - c[0];
                T vslope = -m2, vpot = m2 * u;
                if constexpr (EXT) {
                    vslope -= my2 * c[0] + mz2 * u + mw2 * u * u * u;
                    vpot += T(0.5) * my2 * (T(1) - c[0] * c[0]) + T(0.5) * mz2 * u * u + T(0.25) * mw2 * (u * u) * (u * u);
                }
                T g[4];
#pragma unroll
                for (int A = 0; A < 4; ++A) g[A] = -(uu[A] + (cx * ax[A] + cy * ay[A] + cz * az[A]));
                g[0] += vslope;
                // energy density of the discrete energy (the arrest test and the observables)
                const T e2 = T(-0.5) * dot4(c, lap);
                const T e4 = T(0.5) * (gxx * gyy + gxx * gzz + gyy * gzz - gxy * gxy - gxz * gxz - gyz * gyz);
                if constexpr (MODE == MODE_STEP) {
                    pe2 += (double)(e2 + e4 + vpot);
                } else {
                    pe2 += (double)e2;
                    pe4 += (double)e4;
                    pe0 += (double)vpot;
                    if (baryon) pb += (double)det4(c, ax, ay, az);
                }
                const T gp = dot4(g, c);
                T f[4];
#pragma unroll
                for (int A = 0; A < 4; ++A) f[A] = gp * c[A] - g[A];
                pf2 = fmax_nonneg(pf2, dot4(f, f));
                const size_t s = (size_t)x * plane + (size_t)y * n2 + z;
                if constexpr (MODE == MODE_STEP) {
                    T vc[4], v[4], qv[4];
#pragma unroll
                    for (int A = 0; A < 4; ++A) vc[A] = redo ? T(0) : vel[(size_t)A * N3 + s];
                    pp += (double)dot4(f, vc);
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        v[A] = grad_flow ? T(0) : vc[A] + dt * f[A];
                        qv[A] = c[A] + dt * (grad_flow ? f[A] : v[A]);
                    }
                    if (renorm64) {
                        const double s2 = (double)qv[0] * qv[0] + (double)qv[1] * qv[1] + (double)qv[2] * qv[2] +
                                          (double)qv[3] * qv[3];
                        const double inv = 1.0 / sqrt(s2);
#pragma unroll
                        for (int A = 0; A < 4; ++A) qv[A] = T((double)qv[A] * inv);
                    } else {
                        const T inv = rnorm(dot4(qv, qv));
#pragma unroll
                        for (int A = 0; A < 4; ++A) qv[A] *= inv;
                    }
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        pout[(size_t)A * N3 + s] = qv[A];
                        vel[(size_t)A * N3 + s] = v[A];
                    }
                } else if (has_grad) {
#pragma unroll
                    for (int A = 0; A < 4; ++A) gout[(size_t)A * N3 + s] = projected ? -f[A] : g[A];
                }
            }
            __syncthreads();
        }
    }

    // block reduction of the partial sums (fixed order), the layout of the exact-gradient sweep
    double vals[7] = {pe2, pe4, pe0, pb, (double)pf2, pp, 0.0};
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        double v = vals[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = (i == P_F2) ? fmax(v, o) : v + o;
        }
        if (lane == 0) sm.red[wave][i] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double* o = a.partials + (size_t)blockIdx.x * NPART;
        for (int i = 0; i < 7; ++i) {
            double sum = 0.0;
            for (int w = 0; w < FP_THREADS / 64; ++w) sum = (i == P_F2) ? fmax(sum, sm.red[w][i]) : sum + sm.red[w][i];
            o[i] = sum;
        }
    }
}

}  // namespace skyr

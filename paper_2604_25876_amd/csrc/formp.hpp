// Printed-form flow sweep: the force from the paper's Euler-Lagrange
// expression (Sec. 3, eq. Sigma model EL equations, halved to this library's
// energy normalisation) instead of the exact derivative of the discrete energy:
//   g = -{ (1 + S) Lap phi + sum_i c_i a_i - sum_ij G_ij D_i D_j phi } + V'(phi0) e_0,
//   a_i = D_i phi, G_ij = a_i . a_j, S = tr G, Lap = sum_i D_ii phi,
//   c_i = sum_j (D_i D_j phi) . a_j - Lap . a_i,
// with the five-point second difference D_ii and the mixed derivative D_i D_j
// as the product of two first-difference stencils (radius 2 in each of its
// two directions).  The stencil is one-stage: g at a site depends on phi
// within the 5 x 5 x 5 box around it, so there is no flux pass and no tile
// overlap.  Everything else (energy density for the arrest test, projection,
// kick-drift update, renormalisation, partial sums) is that of the
// exact-gradient sweep.
//
// 2.5D march: a block owns a 16 x 32 (y, z) tile (one thread per column) and
// a slab of x.  Each thread keeps, for planes x-2 .. x+2 of its column, phi,
// D_y phi and D_z phi in register rings: the x-derivatives and D_x D_y, D_x D_z
// come from registers.  phi planes with a two-site halo pass through a ring of
// four LDS slots: at plane x the block stages plane x+2 (from a register
// prefetch), and after one barrier each thread takes D_y, D_z of plane x+2 and
// the y/z second derivatives and D_y D_z of plane x from LDS.  Plane x+2 goes
// to the slot of x-2, whose last reads came before the previous barrier.
#pragma once

#include "sweep.hpp"

namespace skyr {

constexpr int FP_LW = 32, FP_ROWS = 16, FP_THREADS = FP_LW * FP_ROWS;
constexpr int FP_H = FP_ROWS + 4, FP_W = FP_LW + 4;
constexpr int FP_NH = FP_H * FP_W - FP_ROWS * FP_LW;  // halo sites of a plane

__host__ __device__ inline int formp_tiles(int n1, int n2)
{
    return ((n1 - 4 + FP_ROWS - 1) / FP_ROWS) * ((n2 - 4 + FP_LW - 1) / FP_LW);
}
// planes per slab: the even split of x into the most slabs (of at least 16
// planes) whose blocks fit one round of the chip, two blocks per CU in float
// and one in double (the LDS ring of four planes)
__host__ __device__ inline int formp_chunk(int n0, int n1, int n2, bool dbl)
{
    const int nx = n0 - 4, tiles = formp_tiles(n1, n2);
    const int target = dbl ? 256 : 512;
    int slabs = target / (tiles > 0 ? tiles : 1);
    const int most = nx / 16 > 1 ? nx / 16 : 1;
    slabs = slabs < 1 ? 1 : (slabs > most ? most : slabs);
    const int xc = (nx + slabs - 1) / slabs;
    return xc < 16 ? 16 : xc;
}
__host__ __device__ inline int formp_blocks(int n0, int n1, int n2, bool dbl)
{
    const int xc = formp_chunk(n0, n1, n2, dbl);
    return formp_tiles(n1, n2) * ((n0 - 4 + xc - 1) / xc);
}

template <typename T> struct FormPSmem {
    T phi[4][4][FP_H][FP_W];  // [slot][component][row][column]
    double red[FP_THREADS / 64][7];
};

// float: at most 128 VGPRs, so that two blocks (16 waves) share a CU
template <typename T, int MODE, bool EXT>
__global__ __launch_bounds__(FP_THREADS, sizeof(T) == 4 ? 4 : 1) void formp_kernel(SweepArgs a)
{
    __shared__ FormPSmem<T> sm;
    const Ctl* ctl = a.ctl;
    int cur = 0;
    bool redo = false, renorm64 = false;
    int restore = RESTORE_NONE;
    if constexpr (MODE == MODE_STEP) {
        restore = ctl->restore;
        if (ctl->done && !restore) return;  // uniform
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

    const int tz_tiles = (n2 - 4 + FP_LW - 1) / FP_LW;
    const int tiles = formp_tiles(n1, n2);
    const int slab = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int y0 = 2 + (tile / tz_tiles) * FP_ROWS, z0 = 2 + (tile % tz_tiles) * FP_LW;
    const int xb = 2 + slab * a.xchunk, xe = min(n0 - 2, xb + a.xchunk);
    const int tid = threadIdx.x, ly = tid / FP_LW, lz = tid % FP_LW;
    const int y = y0 + ly, z = z0 + lz;
    const bool out = (y <= n1 - 3) && (z <= n2 - 3);
    const int r = ly + 2, q = lz + 2;  // LDS position of the own column
    // own column and, for the first FP_NH threads, one halo site of the tile
    const size_t own = (size_t)clampi(y, 0, n1 - 1) * n2 + clampi(z, 0, n2 - 1);
    const bool halo_loader = tid < FP_NH;
    int hr = 0, hq = 0;
    {
        // halo sites: rows 0, 1, FP_H-2, FP_H-1 (all columns), then columns 0, 1,
        // FP_W-2, FP_W-1 of the other rows
        const int u = min(tid, FP_NH - 1);
        if (u < 4 * FP_W) {
            const int k = u / FP_W;
            hr = k < 2 ? k : FP_ROWS + k;
            hq = u % FP_W;
        } else {
            const int v = u - 4 * FP_W, k = v & 3;
            hr = 2 + (v >> 2);
            hq = k < 2 ? k : FP_LW + k;
        }
    }
    const size_t hoff = (size_t)clampi(y0 - 2 + hr, 0, n1 - 1) * n2 + clampi(z0 - 2 + hq, 0, n2 - 1);

    const T c1h = T(Coef<double>::c1 / a.h), c2h = T(Coef<double>::c2 / a.h);
    const T d1h = T(Coef<double>::d1 / (a.h * a.h)), d2h = T(Coef<double>::d2 / (a.h * a.h));
    const T dt = T(a.dt);
    const T m2 = T(a.m * a.m), my2 = T(a.m_y * a.m_y), mz2 = T(a.m_z * a.m_z), mw2 = T(a.m_w * a.m_w);
    const bool grad_flow = MODE == MODE_STEP && a.gradient_flow != 0;
    const bool has_grad = gout != nullptr, projected = a.projected != 0, baryon = a.baryon != 0;

    double pe2 = 0.0, pe4 = 0.0, pe0 = 0.0, pb = 0.0, pp = 0.0;
    T pf2 = T(0);

    // register rings over planes x-2 .. x+2 (slots 0 .. 4) of the own column
    T rphi[5][4], rdy[5][4], rdz[5][4];
    T nxt[4], hnxt[4];  // prefetch of the next plane to stage: own column and halo site

    auto prefetch = [&](int x) {
        const size_t xo = (size_t)clampi(x, 0, n0 - 1) * plane;
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            nxt[A] = pin[(size_t)A * N3 + xo + own];
            if (halo_loader) hnxt[A] = pin[(size_t)A * N3 + xo + hoff];
        }
    };
    auto stage = [&](int x) {  // the prefetched plane x into its LDS slot
        const int sl = x & 3;
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            sm.phi[sl][A][r][q] = nxt[A];
            if (halo_loader) sm.phi[sl][A][hr][hq] = hnxt[A];
        }
    };
    auto take = [&](int x) {  // phi, D_y phi, D_z phi of the staged plane x into ring slot 4
        const int sl = x & 3;
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            const T(*P)[FP_W] = sm.phi[sl][A];
            rphi[4][A] = P[r][q];
            rdy[4][A] = c1h * (P[r + 1][q] - P[r - 1][q]) + c2h * (P[r + 2][q] - P[r - 2][q]);
            rdz[4][A] = c1h * (P[r][q + 1] - P[r][q - 1]) + c2h * (P[r][q + 2] - P[r][q - 2]);
        }
    };
    auto shift = [&]() {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                rphi[s][A] = rphi[s + 1][A];
                rdy[s][A] = rdy[s + 1][A];
                rdz[s][A] = rdz[s + 1][A];
            }
    };

    if (xb < xe) {
        // prologue: planes xb-2 .. xb+1 into ring slots 1 .. 4
        prefetch(xb - 2);
        for (int x = xb - 2; x <= xb + 1; ++x) {
            stage(x);
            prefetch(x + 1);
            __syncthreads();
            shift();
            take(x);
        }
        for (int x = xb; x < xe; ++x) {
            // stage plane x+2 into the slot of plane x-2 (last read before the previous barrier)
            stage(x + 2);
            prefetch(x + 3);
            const size_t s = (size_t)x * plane + own;
            T vc[4];
            if constexpr (MODE == MODE_STEP) {
#pragma unroll
                for (int A = 0; A < 4; ++A) vc[A] = (redo || !out) ? T(0) : vel[(size_t)A * N3 + s];
            }
            __syncthreads();
            shift();  // slots 0 .. 3 now hold planes x-2 .. x+1
            take(x + 2);
            if (out) {
                const int sl = x & 3;  // LDS slot of plane x (ring slot 2)
                T c[4], ax[4], ay[4], az[4];
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    c[A] = rphi[2][A];
                    ax[A] = c1h * (rphi[3][A] - rphi[1][A]) + c2h * (rphi[4][A] - rphi[0][A]);
                    ay[A] = rdy[2][A];
                    az[A] = rdz[2][A];
                }
                const T gxx = dot4(ax, ax), gyy = dot4(ay, ay), gzz = dot4(az, az);
                const T gxy = dot4(ax, ay), gxz = dot4(ax, az), gyz = dot4(ay, az);
                const T S = gxx + gyy + gzz;
                // per component: u_A = (1 + S) Lap_A - sum_ij G_ij (D_i D_j phi)_A, Lap_A, and the
                // contributions to c_i = sum_j (D_i D_j phi) . a_j - Lap . a_i
                T uu[4], lap[4];
                T cx = T(0), cy = T(0), cz = T(0);
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    const T(*P)[FP_W] = sm.phi[sl][A];
                    const T cc = c[A];
                    // five-point second differences from the centre (weights sum to zero)
                    const T dxx = d1h * ((rphi[3][A] - cc) + (rphi[1][A] - cc)) +
                                  d2h * ((rphi[4][A] - cc) + (rphi[0][A] - cc));
                    const T dyy = d1h * ((P[r + 1][q] - cc) + (P[r - 1][q] - cc)) +
                                  d2h * ((P[r + 2][q] - cc) + (P[r - 2][q] - cc));
                    const T dzz = d1h * ((P[r][q + 1] - cc) + (P[r][q - 1] - cc)) +
                                  d2h * ((P[r][q + 2] - cc) + (P[r][q - 2] - cc));
                    // D_x D_y and D_x D_z from the rings, D_y D_z from the LDS plane
                    const T dxy = c1h * (rdy[3][A] - rdy[1][A]) + c2h * (rdy[4][A] - rdy[0][A]);
                    const T dxz = c1h * (rdz[3][A] - rdz[1][A]) + c2h * (rdz[4][A] - rdz[0][A]);
                    auto dz_row = [&](int rr) {
                        return c1h * (P[rr][q + 1] - P[rr][q - 1]) + c2h * (P[rr][q + 2] - P[rr][q - 2]);
                    };
                    const T dyz = c1h * (dz_row(r + 1) - dz_row(r - 1)) + c2h * (dz_row(r + 2) - dz_row(r - 2));
                    const T la = dxx + dyy + dzz;
                    lap[A] = la;
                    uu[A] = (T(1) + S) * la -
                            (gxx * dxx + gyy * dyy + gzz * dzz + T(2) * (gxy * dxy + gxz * dxz + gyz * dyz));
                    cx += dxx * ax[A] + dxy * ay[A] + dxz * az[A] - la * ax[A];
                    cy += dxy * ax[A] + dyy * ay[A] + dyz * az[A] - la * ay[A];
                    cz += dxz * ax[A] + dyz * ay[A] + dzz * az[A] - la * az[A];
                }
                const T u = T(1) - c[0];
                T vslope = -m2, vpot = m2 * u;
                if constexpr (EXT) {
                    vslope -= my2 * c[0] + mz2 * u + mw2 * u * u * u;
                    vpot += T(0.5) * my2 * (T(1) - c[0] * c[0]) + T(0.5) * mz2 * u * u +
                            T(0.25) * mw2 * (u * u) * (u * u);
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
                if constexpr (MODE == MODE_STEP) {
                    T v[4], qv[4];
                    pp += (double)f[0] * vc[0] + (double)f[1] * vc[1] + (double)f[2] * vc[2] + (double)f[3] * vc[3];
                    if (restore) {
#pragma unroll
                        for (int A = 0; A < 4; ++A)
                            vel[(size_t)A * N3 + s] = restore == RESTORE_ZERO ? T(0) : vc[A] - dt * f[A];
                        continue;
                    }
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

// formp.hpp -- printed-form flow sweep for gfx950: the force from the paper's
// Euler-Lagrange expression (Sec. 3, eq. Sigma model EL equations, halved to this
// library's energy normalisation) instead of the exact derivative of the discrete energy:
//   g = -{ (1 + S) Lap phi + sum_i c_i a_i - sum_ij G_ij D_i D_j phi } + V'(phi0) e_0,
//   a_i = D_i phi, G_ij = a_i . a_j, S = tr G, Lap = sum_i D_ii phi,
//   c_i = sum_j (D_i D_j phi) . a_j - Lap . a_i,
// with the five-point second difference D_ii and the mixed derivative D_i D_j as the
// product of two first-difference stencils.  g at a site depends on phi within two
// sites along every axis and on the (+-1, +-2) x (+-1, +-2) squares of each pair of
// axes: one stencil stage, no flux pass and no overlap between tiles.  The energy
// density (for the arrest test and the observables), projection, kick-drift update,
// renormalisation, partial sums and the flow's decision are those of the exact sweep.
//
// Work decomposition (2.5D march along x, one output site per lane):
//   * a tile is OY rows x OZ columns; every lane owns one output column, and the
//     first lanes of the block also load one site each of the two-site frame around
//     the tile;
//   * phi planes with their frame pass through a ring of four LDS buffers: at step s
//     the block stages plane s; after one barrier each lane takes D_y phi and D_z phi
//     of its column in plane s, pushes their x-differences into register rings of five
//     accumulators (D_x D_y phi and D_x D_z phi of planes s-2 .. s+2) and writes D_z phi
//     to a ring of three LDS planes (the lanes of the frame rows add it for the two rows
//     above and below the tile); it then finishes output plane s-2 from its buffer (the
//     y/z second differences), the y-difference of its D_z phi plane (D_y D_z phi), the
//     phi ring of its column (the x-differences) and the accumulators, complete by then;
//   * x is cut into slabs and a launch has one block per (slab, tile) item, as in the
//     exact sweep; the velocity read and the outputs are streamed past L2.
// Stencils are evaluated in scaled form: 12 h D_i, and 144 h^2 for every second
// difference (pure and mixed); the constant factors are folded into the weights.
#pragma once

#include "sweep.hpp"

namespace skyr {

// Tile geometry: NW waves of 64 lanes, one output site each, OZ columns.
template <int NW_, int OZ_> struct FpGeo {
    static constexpr int NW = NW_, OZ = OZ_;
    static constexpr int THREADS = NW * 64;
    static constexpr int OY = THREADS / OZ;
    static constexpr int PW = OZ + 4, PH = OY + 4;  // a phi plane: rows -2 .. OY+1, columns -2 .. OZ+1
    static constexpr int PPLANE = PW * PH;
    static constexpr int NFRAME = 4 * PW + 4 * OY;  // two rows above and below, two columns left and right
    static constexpr int ZPLANE = PH * OZ;          // D_z phi plane: rows -2 .. OY+1, the tile's columns
    static_assert(THREADS % OZ == 0, "whole rows per block");
    static_assert(NFRAME <= THREADS, "one frame site per lane at most");
};
// float: 16 x 32 tiles (at 256^3: 16 x 8 tiles of two 126-plane slabs, one round of the
// chip); double: 8 x 32 tiles of four waves, one per SIMD, so that the registers the
// double rings need come from the whole register file of the SIMD
using FpGeoF32 = FpGeo<8, 32>;
using FpGeoF64 = FpGeo<4, 32>;
template <typename T> using FpGeoOf = std::conditional_t<sizeof(T) == 4, FpGeoF32, FpGeoF64>;

template <typename T, class G> struct FormPSmem {
    Site4<T> phi[4][G::PPLANE];  // [plane mod 4][site]
    Site4<T> dz[3][G::ZPLANE];   // 12 h D_z phi, [plane mod 3][site]
    double red[G::NW][NPART];
    int last;  // this block is the last of the sweep to finish
};

// Per-launch constants.  With a^ = 12 h a, every second difference D~ = 144 h^2 D, K2 = 144 h^2
// and K = K2^2, the scaled force is g^ = K g = -((K2 + S^) L~ + sum_i c^_i a^_i - sum_ij G^_ij D~_ij)
// + K V'(phi0) e_0 with G^ = a^.a^, S^ = tr G^, L~ = sum_i D~_ii, c^_i = sum_j D~_ij . a^_j - L~ . a^_i.
template <typename T> struct FormPConst {
    T K2;
    T ke2, ke4;  // e2 = ke2 phi.L~, e4 = ke4 (G^ quadratic form)
    T dt, dtK, invK;
    T m2, my2, mz2, mw2;
    T m2K, my2K, mz2K, mw2K;
    double dinvK, dinvK2, dinv12h3;
    bool more_pot, grad_flow;

    __device__ __forceinline__ void init(const SweepArgs& a, bool step_mode)
    {
        const double h = a.h, k2 = 144.0 * h * h, K = k2 * k2;
        K2 = T(k2);
        ke2 = T(-0.5 / k2);
        ke4 = T(0.5 / K);
        dt = T(a.dt);
        dtK = T(a.dt / K);
        invK = T(1.0 / K);
        m2 = T(a.m * a.m);
        my2 = T(a.m_y * a.m_y);
        mz2 = T(a.m_z * a.m_z);
        mw2 = T(a.m_w * a.m_w);
        m2K = T(K * a.m * a.m);
        my2K = T(K * a.m_y * a.m_y);
        mz2K = T(K * a.m_z * a.m_z);
        mw2K = T(K * a.m_w * a.m_w);
        dinvK = 1.0 / K;
        dinvK2 = 1.0 / (K * K);
        dinv12h3 = 1.0 / (1728.0 * h * h * h);
        more_pot = a.m_y != 0.0 || a.m_z != 0.0 || a.m_w != 0.0;
        grad_flow = step_mode && a.gradient_flow != 0;
    }
};

// 8 (f[+1] - f[-1]) - (f[+2] - f[-2]): 12 h times the first difference
template <typename T> __device__ __forceinline__ T d1s(T m2, T m1, T p1, T p2) { return fmaT(T(8), p1 - m1, m2 - p2); }
// 12 (16 ((f[+1] - f) + (f[-1] - f)) - ((f[+2] - f) + (f[-2] - f))): 144 h^2 times the five-point
// second difference, from differences with the centre (no cancellation of O(1) terms)
template <typename T> __device__ __forceinline__ T d2s(T m2, T m1, T c, T p1, T p2)
{
    return T(12) * fmaT(T(16), (p1 - c) + (m1 - c), -((p2 - c) + (m2 - c)));
}

template <typename T, int MODE, bool EXT> struct FormP {
    using G = FpGeoOf<T>;
    using Smem = FormPSmem<T, G>;
    Smem& sm;
    const FormPConst<T>& k;
    const SweepCommon<T, false>& cm;
    int row, col, pidx;
    unsigned off;       // byte offset of the own site within a plane
    bool out;           // the own column is in the output region (y, z)
    bool floader;       // this lane also loads a frame site
    bool fdz;           // ... in the rows above or below the tile, whose D_z phi it supplies
    int frow, fcol;     // its tile-relative row and column
    int fidx;           // its LDS index
    int zidx, fzidx;    // LDS index of the own and the frame site in a D_z phi plane
    unsigned foff;      // its byte offset within a plane
    int xa, xe;
    T ring[5][4];       // phi of planes s-4 .. s (slot = plane offset mod 5)
    T axy[5][4];        // D~_xy of planes s-2 .. s+2 (same slots)
    T axz[5][4];        // D~_xz
    T nxt[4], fnxt[4];  // prefetched own and frame sites of plane s+1
    T vnxt[4];          // prefetched velocity of plane s-1

    double pe2 = 0.0, pe4 = 0.0, pe0 = 0.0, pb_sum = 0.0, pp = 0.0;
    T pf2 = T(0);

    __device__ __forceinline__ FormP(Smem& s, const FormPConst<T>& kk, const SweepCommon<T, false>& c, int tid)
        : sm(s), k(kk), cm(c)
    {
        row = tid / G::OZ;
        col = tid - row * G::OZ;
        pidx = (row + 2) * G::PW + col + 2;
        floader = tid < G::NFRAME;
        const int f = floader ? tid : 0;
        if (f < 4 * G::PW) {  // rows -2, -1, OY, OY+1 over all columns
            const int q = f / G::PW;
            frow = q < 2 ? q - 2 : G::OY + q - 2;
            fcol = f - q * G::PW - 2;
        } else {  // columns -2, -1, OZ, OZ+1 of the tile's rows
            const int g = f - 4 * G::PW, q = g & 3;
            frow = g >> 2;
            fcol = q < 2 ? q - 2 : G::OZ + q - 2;
        }
        fidx = (frow + 2) * G::PW + fcol + 2;
        fdz = floader && f < 4 * G::PW && fcol >= 0 && fcol < G::OZ;
        zidx = (row + 2) * G::OZ + col;
        fzidx = fdz ? (frow + 2) * G::OZ + fcol : 0;
    }

    __device__ __forceinline__ void setup(const Segment& s, int tiles_z_start)
    {
        const int y0 = cm.olo1 + s.ty * G::OY, z0 = tiles_z_start + s.tz * G::OZ;
        const int y = y0 + row, z = z0 + col;
        out = (y <= cm.ohi1) && (z >= cm.olo2) && (z <= cm.ohi2);
        off = cm.site_off(y, z);
        foff = cm.site_off(y0 + frow, z0 + fcol);
        xa = s.xa;
        xe = s.xe;
    }

    __device__ __forceinline__ T slopeK(T p0) const
    {
        const T u = T(1) - p0;
        T d = -k.m2K;
        if constexpr (EXT) {
            if (k.more_pot) d -= k.my2K * p0 + k.mz2K * u + k.mw2K * u * u * u;
        }
        return d;
    }
    __device__ __forceinline__ T potential(T p0) const
    {
        const T u = T(1) - p0;
        T v = k.m2 * u;
        if constexpr (EXT) {
            if (k.more_pot)
                v += T(0.5) * k.my2 * (T(1) - p0 * p0) + T(0.5) * k.mz2 * u * u + T(0.25) * k.mw2 * (u * u) * (u * u);
        }
        return v;
    }

    // step s of the march: stage plane s, push D_x of its D_y phi and D_z phi, finish plane s-2
    template <int U> __device__ __forceinline__ void step(int s)
    {
        // slots of planes s-4, s-3, s-2, s-1, s (and of s+1 = s-4 + 5, s+2 = s-3 + 5)
        constexpr int Q4 = (U + 1) % 5, Q3 = (U + 2) % 5, Q2 = (U + 3) % 5, Q1 = (U + 4) % 5, Q0 = U % 5;
        // opaque to the optimiser from here on: the LDS and global addresses of this plane
        // are formed within it, not carried over from an earlier plane across the barriers
        asm volatile("" : "+v"(pidx), "+v"(off), "+v"(fidx), "+v"(foff), "+v"(zidx), "+v"(fzidx));
#pragma unroll
        for (int sl = 0; sl < 5; ++sl) {
            asm volatile("" : "+v"(ring[sl][0]), "+v"(ring[sl][1]), "+v"(ring[sl][2]), "+v"(ring[sl][3]));
            asm volatile("" : "+v"(axy[sl][0]), "+v"(axy[sl][1]), "+v"(axy[sl][2]), "+v"(axy[sl][3]));
            asm volatile("" : "+v"(axz[sl][0]), "+v"(axz[sl][1]), "+v"(axz[sl][2]), "+v"(axz[sl][3]));
        }
        // stage plane s into the buffer of plane s-4 (its last reads came before the last barrier)
        Site4<T>* B = sm.phi[s & 3];
        st4(B + pidx, nxt);
        if (floader) st4(B + fidx, fnxt);
#pragma unroll
        for (int A = 0; A < 4; ++A) ring[Q0][A] = nxt[A];
        // the velocity of output plane s-2 was prefetched one step earlier; plane s-1's now
        T vcur[4];
        if constexpr (MODE == MODE_STEP) {
            const unsigned vb = (unsigned)clampi(s - 1, 0, cm.n0 - 1) * cm.plane_b;
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                vcur[A] = vnxt[A];
                vnxt[A] = ldb_nt((gptr<const T>)cm.vel[A], vb + off);
            }
            if (cm.redo) {  // a redo sweep starts from zero velocity
#pragma unroll
                for (int A = 0; A < 4; ++A) vcur[A] = T(0);
            }
        }
        cm.load(off, s + 1, nxt);
        if (floader) cm.load(foff, s + 1, fnxt);
        __syncthreads();

        // D_y phi and D_z phi of the own column in plane s, pushed into D_x of them:
        // f(s) enters 8 (f(t+1) - f(t-1)) - (f(t+2) - f(t-2)) with +8 at t = s-1, -8 at
        // t = s+1, -1 at t = s-2 and +1 at t = s+2; D_z phi also goes to the plane's D_z
        // buffer (whose y-differences give D_y D_z phi two steps later), with that of the
        // frame sites in the rows above and below the tile
        Site4<T>* Z = sm.dz[s % 3];
        if (fdz) {
            const Site4<T>* F = B + fidx;
            T m2[4], m1[4], p1[4], p2[4], d[4];
            ld4(F - 2, m2);
            ld4(F - 1, m1);
            ld4(F + 1, p1);
            ld4(F + 2, p2);
#pragma unroll
            for (int A = 0; A < 4; ++A) d[A] = d1s(m2[A], m1[A], p1[A], p2[A]);
            st4(Z + fzidx, d);
        }
        {
            const Site4<T>* P = B + pidx;
            T ym2[4], ym1[4], yp1[4], yp2[4], zm2[4], zm1[4], zp1[4], zp2[4];
            ld4(P - 2 * G::PW, ym2);
            ld4(P - G::PW, ym1);
            ld4(P + G::PW, yp1);
            ld4(P + 2 * G::PW, yp2);
            ld4(P - 2, zm2);
            ld4(P - 1, zm1);
            ld4(P + 1, zp1);
            ld4(P + 2, zp2);
            T azs[4];
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                const T ay = d1s(ym2[A], ym1[A], yp1[A], yp2[A]);
                const T az = d1s(zm2[A], zm1[A], zp1[A], zp2[A]);
                azs[A] = az;
                axy[Q1][A] = fmaT(T(8), ay, axy[Q1][A]);
                axy[Q4][A] = fmaT(T(-8), ay, axy[Q4][A]);
                axy[Q2][A] -= ay;
                axy[Q3][A] += ay;
                axz[Q1][A] = fmaT(T(8), az, axz[Q1][A]);
                axz[Q4][A] = fmaT(T(-8), az, axz[Q4][A]);
                axz[Q2][A] -= az;
                axz[Q3][A] += az;
            }
            st4(Z + zidx, azs);
        }

        const int t = s - 2;
        if (t >= xa && t < xe && out) finish<Q4, Q3, Q2, Q1, Q0>(t, vcur);
#pragma unroll
        for (int A = 0; A < 4; ++A) {  // the slots of plane s-2 start plane s+3
            axy[Q2][A] = T(0);
            axz[Q2][A] = T(0);
        }
    }

    // output site (t, own column): the ring holds planes t-2 .. t+2 in slots Q4 .. Q0 and
    // the accumulators of plane t (slot Q2) are complete
    template <int Q4, int Q3, int Q2, int Q1, int Q0> __device__ __forceinline__ void finish(int t, const T (&vcur)[4])
    {
        const Site4<T>* P = sm.phi[t & 3] + pidx;
        T c[4], ax[4], ay[4], az[4], dxx[4], dyy[4], dzz[4], dyz[4], lap[4];
        {
            T ym2[4], ym1[4], yp1[4], yp2[4], zm2[4], zm1[4], zp1[4], zp2[4];
            ld4(P - 2 * G::PW, ym2);
            ld4(P - G::PW, ym1);
            ld4(P + G::PW, yp1);
            ld4(P + 2 * G::PW, yp2);
            ld4(P - 2, zm2);
            ld4(P - 1, zm1);
            ld4(P + 1, zp1);
            ld4(P + 2, zp2);
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                const T cc = ring[Q2][A];
                c[A] = cc;
                ax[A] = d1s(ring[Q4][A], ring[Q3][A], ring[Q1][A], ring[Q0][A]);
                ay[A] = d1s(ym2[A], ym1[A], yp1[A], yp2[A]);
                az[A] = d1s(zm2[A], zm1[A], zp1[A], zp2[A]);
                dxx[A] = d2s(ring[Q4][A], ring[Q3][A], cc, ring[Q1][A], ring[Q0][A]);
                dyy[A] = d2s(ym2[A], ym1[A], cc, yp1[A], yp2[A]);
                dzz[A] = d2s(zm2[A], zm1[A], cc, zp1[A], zp2[A]);
                lap[A] = (dxx[A] + dyy[A]) + dzz[A];
            }
        }
        {
            // D~_yz: the y-difference of the D_z phi plane (written two steps earlier)
            const Site4<T>* Z = sm.dz[t % 3] + zidx;
            T m2[4], m1[4], p1[4], p2[4];
            ld4(Z - 2 * G::OZ, m2);
            ld4(Z - G::OZ, m1);
            ld4(Z + G::OZ, p1);
            ld4(Z + 2 * G::OZ, p2);
#pragma unroll
            for (int A = 0; A < 4; ++A) dyz[A] = d1s(m2[A], m1[A], p1[A], p2[A]);
        }
        const T gxx = dot4(ax, ax), gyy = dot4(ay, ay), gzz = dot4(az, az);
        const T gxy = dot4(ax, ay), gxz = dot4(ax, az), gyz = dot4(ay, az);
        const T S = (gxx + gyy) + gzz;
        T cx = T(0), cy = T(0), cz = T(0), g[4];
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            const T dxy = axy[Q2][A], dxz = axz[Q2][A];
            cx += fmaT(dxx[A] - lap[A], ax[A], fmaT(dxy, ay[A], dxz * az[A]));
            cy += fmaT(dyy[A] - lap[A], ay[A], fmaT(dxy, ax[A], dyz[A] * az[A]));
            cz += fmaT(dzz[A] - lap[A], az[A], fmaT(dxz, ax[A], dyz[A] * ay[A]));
            const T gd = fmaT(gxx, dxx[A], fmaT(gyy, dyy[A], gzz * dzz[A])) +
                         T(2) * fmaT(gxy, dxy, fmaT(gxz, dxz, gyz * dyz[A]));
            g[A] = fmaT(k.K2 + S, lap[A], -gd);  // (K2 + S^) L~ - sum G^ D~, completed below
        }
#pragma unroll
        for (int A = 0; A < 4; ++A) g[A] = -fmaT(cx, ax[A], fmaT(cy, ay[A], fmaT(cz, az[A], g[A])));
        g[0] += slopeK(c[0]);

        const T e2 = k.ke2 * dot4(c, lap);
        const T e4 = k.ke4 * (gxx * gyy + gxx * gzz + gyy * gzz - gxy * gxy - gxz * gxz - gyz * gyz);
        const T e0 = potential(c[0]);
        if constexpr (MODE == MODE_STEP) {
            pe2 += (double)(e2 + e4 + e0);  // the flow needs the total energy only
        } else {
            pe2 += (double)e2;
            pe4 += (double)e4;
            pe0 += (double)e0;
            if (cm.baryon) pb_sum += (double)det4(c, ax, ay, az);
        }
        const T gp = dot4(g, c);
        T f[4];
#pragma unroll
        for (int A = 0; A < 4; ++A) f[A] = fmaT(gp, c[A], -g[A]);  // F^ = (g^.phi) phi - g^
        pf2 = fmax_nonneg(pf2, dot4(f, f));
        const unsigned base = (unsigned)t * cm.plane_b + off;
        if constexpr (MODE == MODE_STEP) {
            pp += (double)dot4(f, vcur);  // the product in the field precision, the sum in double
            if (cm.restore) {
#pragma unroll
                for (int A = 0; A < 4; ++A)
                    stb_nt(cm.vel[A], base, cm.restore == RESTORE_ZERO ? T(0) : fmaT(-k.dtK, f[A], vcur[A]));
                return;
            }
            T v[4], q[4], pn[4];
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                if constexpr (EXT) {
                    v[A] = k.grad_flow ? T(0) : fmaT(k.dtK, f[A], vcur[A]);
                    q[A] = k.grad_flow ? fmaT(k.dtK, f[A], c[A]) : fmaT(k.dt, v[A], c[A]);
                } else {
                    v[A] = fmaT(k.dtK, f[A], vcur[A]);
                    q[A] = fmaT(k.dt, v[A], c[A]);
                }
            }
            if (cm.renorm64) {
                const double s2 = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
                const double inv = 1.0 / sqrt(s2);
#pragma unroll
                for (int A = 0; A < 4; ++A) pn[A] = T((double)q[A] * inv);
            } else {
                const T inv = rnorm(dot4(q, q));
#pragma unroll
                for (int A = 0; A < 4; ++A) pn[A] = q[A] * inv;
            }
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                stb_nt(cm.pout[A], base, pn[A]);
                stb_nt(cm.vel[A], base, v[A]);
            }
        } else {
            if (cm.has_grad) {
#pragma unroll
                for (int A = 0; A < 4; ++A) stb_nt(cm.gout[A], base, (cm.projected ? -f[A] : g[A]) * k.invK);
            }
        }
    }

    // the march over one segment: steps s = xa-2 .. xe+1 finish planes xa .. xe-1, in whole
    // groups of five starting `lead` steps early (those reach no output plane)
    __device__ __forceinline__ void march()
    {
#pragma unroll
        for (int sl = 0; sl < 5; ++sl)
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                axy[sl][A] = T(0);
                axz[sl][A] = T(0);
                ring[sl][A] = T(0);
            }
        const int lead = march_lead(xa, xe);
        const int s0 = xa - 2 - lead;
        cm.load(off, s0, nxt);
        if (floader) cm.load(foff, s0, fnxt);
        if constexpr (MODE == MODE_STEP) {
            const unsigned vb = (unsigned)clampi(s0 - 2, 0, cm.n0 - 1) * cm.plane_b;
#pragma unroll
            for (int A = 0; A < 4; ++A) vnxt[A] = ldb_nt((gptr<const T>)cm.vel[A], vb + off);
        }
        const int nst = (xe - xa) + 4 + lead;
        for (int st = 0; st < nst; st += 5) {
            const int s = s0 + st;
            step<0>(s);
            step<1>(s + 1);
            step<2>(s + 2);
            step<3>(s + 3);
            step<4>(s + 4);
        }
    }
};

// One block per (slab, tile) item, block i (after the XCD remap) taking items i, i + grid, ...
template <typename T, int MODE, bool EXT>
__global__ __launch_bounds__(FpGeoOf<T>::THREADS) __attribute__((amdgpu_waves_per_eu(1, sizeof(T) == 8 ? 1 : 2)))
void formp_kernel(SweepArgs a)
{
    using G = FpGeoOf<T>;
    __shared__ FormPSmem<T, G> sm;
    const int nb = gridDim.x;
    const int b = xcd_logical_block(blockIdx.x, nb);
    SweepCommon<T, false> cm;
    int cur = 0;
    cm.redo = false;
    cm.renorm64 = false;
    cm.restore = RESTORE_NONE;
    if constexpr (MODE == MODE_STEP) {
        // the control block is the same for the whole block: its fields are read as uniform values
        const gptr<const Ctl> ctl = (gptr<const Ctl>)uniform_ptr(a.ctl);
        const auto rd = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
        cm.restore = rd(ctl->restore);
        if (rd(ctl->done) && !cm.restore) return;  // the flow has stopped
        cur = rd(ctl->cur);
        cm.redo = rd(ctl->redo) != 0;
        const int kr = rd(ctl->renorm64_every);
        const long long st = ctl->steps;
        const int st_lo = rd((int)(unsigned)(st & 0xffffffff)), st_hi = rd((int)(unsigned)(st >> 32));
        const long long steps = (long long)(((unsigned long long)(unsigned)st_hi << 32) | (unsigned)st_lo);
        cm.renorm64 = (kr > 0) && (((steps + 1) % kr) == 0);
    }
    cm.n0 = a.n0;
    cm.n1 = a.n1;
    cm.n2 = a.n2;
    cm.zlo = a.zlo;
    cm.zhi = a.zhi;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        cm.ilo[d] = a.ilo[d];
        cm.ihi[d] = a.ihi[d];
    }
    cm.olo1 = a.olo[1];
    cm.olo2 = a.olo[2];
    cm.ohi1 = a.ohi[1];
    cm.ohi2 = a.ohi[2];
    cm.plane_b = (unsigned)(a.n1 * a.n2) * (unsigned)sizeof(T);
    const long long N3 = (long long)a.n0 * a.n1 * a.n2;
    {
        const T* pin = (const T*)(MODE == MODE_STEP && cur ? (const void*)a.phi1 : a.phi0);
        T* pout = (T*)(MODE == MODE_STEP ? (cur ? (void*)a.phi0 : a.phi1) : nullptr);
        T* pvel = (T*)a.vel;
        T* pgrad = (T*)a.grad;
        pin = uniform_ptr(pin);
        pout = uniform_ptr(pout);
        pvel = uniform_ptr(pvel);
        pgrad = uniform_ptr(pgrad);
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            cm.pin[A] = (gptr<const T>)(pin + A * N3);
            cm.pout[A] = (gptr<T>)(pout ? pout + A * N3 : nullptr);
            cm.vel[A] = (gptr<T>)(pvel ? pvel + A * N3 : nullptr);
            cm.gout[A] = (gptr<T>)(pgrad ? pgrad + A * N3 : nullptr);
        }
    }
    cm.has_grad = a.grad != nullptr;
    cm.projected = a.projected != 0;
    cm.baryon = a.baryon != 0;
    FormPConst<T> k;
    k.init(a, MODE == MODE_STEP);

    const int tid = threadIdx.x;
    const int tiles = a.tiles_y * a.tiles_z;
    const int x0 = a.olo[0], nx = a.ohi[0] - a.olo[0] + 1;
    const int items = tiles * ((nx + a.xchunk - 1) / a.xchunk);
    FormP<T, MODE, EXT> fp(sm, k, cm, tid);
    for (int item = b; item < items; item += nb) {
        fp.setup(item_segment(item, tiles, a.tiles_z, x0, nx, a.xchunk), a.zstart);
        fp.march();
        __syncthreads();  // the next item's first planes reuse the buffers
    }

    // block reduction of the partial sums (fixed order), the layout of the exact sweep
    double vals[7] = {fp.pe2, fp.pe4, fp.pe0, fp.pb_sum * k.dinv12h3, (double)fp.pf2 * k.dinvK2, fp.pp * k.dinvK, 0.0};
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        double v = vals[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double w = __shfl_xor(v, o);
            v = (i == P_F2) ? fmax(v, w) : v + w;
        }
        if (lane == 0) sm.red[wave][i] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double sum[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < G::NW; ++w)
            for (int i = 0; i < 7; ++i) sum[i] = (i == P_F2) ? fmax(sum[i], sm.red[w][i]) : sum[i] + sm.red[w][i];
        double* o = a.partials + (size_t)b * NPART;
        for (int i = 0; i < 7; ++i) __hip_atomic_store(o + i, sum[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if constexpr (MODE == MODE_STEP)
        finish_step<G::THREADS, G::NW>(a.partials, nb, a.ctl, cm.restore != RESTORE_NONE, sm);
}

}  // namespace skyr

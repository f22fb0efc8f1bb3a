// sweep.hpp -- fused per-step sweep of the arrested Newton flow for gfx950.
//
// One launch evaluates, for every interior site of one field, the discrete
// energy density, the exact gradient of the discrete energy E_h (Sec. 2.1
// energy, Sec. 3 stencils), its tangent projection (Sec. 3, eq. Newton_flow)
// and either the kick-drift-renormalise update (Sec. 3) or a gradient output,
// plus FP64 per-block partial sums of E2, E4, E0, B and the largest |F|^2.
//
// The gradient is -Lap phi (with boundary terms) - sum_i D_i Q_i + V'(phi0) e0, where
// Q_i = S a_i - sum_j G_ij a_j is the flux of the quartic term at the sites of I (zero
// elsewhere).  Two stencil passes: the flux needs phi within two sites, the divergence
// needs the flux within two sites.
//
// Work decomposition (2.5D march along x):
//   * a tile is OY rows (y) x OZ columns (z) of output sites; tiles in z start on a
//     128-byte line when that costs no extra tile;
//   * the block's waves have two roles.  Interior waves hold one output site per lane
//     and do everything there: the derivatives, the Laplacian, the three fluxes, the
//     x-divergence by pushes into a register ring of five gradient accumulators, the
//     y/z-divergence from LDS and the update.  Halo waves hold the flux positions
//     around the tile (two rows above and below, two columns left and right), where
//     only one flux component is ever read (Q_y on the y-halo, Q_z on the z-halo), and
//     compute just that one;
//   * x-neighbours live in per-lane register rings of five phi planes; the march is
//     unrolled five planes deep so that every ring slot is a fixed register;
//   * y- and z-neighbours go through LDS: phi planes (with the frame of sites only the halo
//     positions read, loaded by the halo lanes) and planes of Q_y and Q_z, each
//     double-buffered by plane parity, so one block barrier per plane suffices;
//   * x is cut into slabs; a launch has one block per (slab, tile) item, so that the
//     blocks of neighbouring tiles march through the same planes together and read the
//     phi lines of their shared halo from L2 once; the velocity read and the outputs are
//     streamed past L2 (non-temporal) so that they do not displace those lines.
// Stencils are evaluated in the scaled form 8 (f[+1] - f[-1]) - (f[+2] - f[-2]) =
// 12 h D f (and 16 (...) - (...) = 12 h^2 L f); the constant factors are folded into
// the weights of the final sums.  Energy, charge and force sums are accumulated in
// double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/skyr.h"

#include <type_traits>

namespace skyr {

// partial-sum slots per thread block (doubles)
constexpr int NPART = 8;
enum : int { P_E2 = 0, P_E4 = 1, P_E0 = 2, P_B = 3, P_F2 = 4, P_POW = 5, P_E6 = 6 };
constexpr int NRED = 7;  // slots in use

// Control block of one flow, in device memory at the start of the workspace.
struct Ctl {
    int32_t cur;          // field buffer holding phi_k: 0 = phi, 1 = phi_alt
    int32_t redo;         // this sweep re-runs phi_k with v_k = 0
    int32_t done;         // 1: no further sweep does any work
    int32_t status;       // 0 running, 1 converged, 2 step target reached, 3 non-finite
    int64_t steps;        // accepted steps
    int64_t target;       // stop when steps reaches this
    int64_t arrests;
    int64_t redo_sweeps;
    int64_t sweeps;
    int32_t renorm64_every;
    int32_t nblocks;      // number of partial-sum blocks of the sweep
    int32_t flow_mode;    // skyr_flow_mode
    int32_t restore;      // after convergence: the next sweep over phi_k rewrites v_k (RESTORE_*)
    int32_t ticket;       // blocks of the running sweep that have finished (zero between sweeps)
    int32_t hold;         // timing sweeps: the sweep takes no decision (the state stays as it is)
    double E_prev;
    double E;
    double P;             // power h^3 sum F_k . v_k of the last sweep (arrest rule POWER)
    double unused_[1];
    double max_force;
    double tol;
    double h3;
    double pad[4];
};
static_assert(sizeof(Ctl) <= 256, "control block must fit its 256-byte slot");

enum : int { MODE_STEP = 0, MODE_GRAD = 1 };

// The converging sweep over phi_k has already written v_k + dt F_k over v_k.  The sweep
// after it recomputes F_k from phi_k (the same arithmetic, so the same F_k) and writes
// v_k back: v - dt F_k, or exactly zero when v_k was zero (an arrest at step k, a redo
// sweep, or the gradient flow).  No field is written by that sweep.
enum : int { RESTORE_NONE = 0, RESTORE_UNKICK = 1, RESTORE_ZERO = 2 };

struct SweepArgs {
    const void* phi0;  // field buffer 0 (phi)
    void* phi1;        // field buffer 1 (phi_alt); MODE_GRAD: unused
    void* vel;         // MODE_STEP: velocity, updated in place
    void* grad;        // MODE_GRAD: nullable gradient output
    double* partials;  // [nblocks][NPART]
    Ctl* ctl;          // MODE_STEP: control block
    int n0, n1, n2;        // extent of the stored array (the whole lattice, or a padded block)
    // elements from one component of the field to the next: n0 n1 n2 for component-major
    // arrays; the row length when the components of a row follow each other (the row of
    // n2 elements then holding all four, each in its own quarter)
    long long cstride;
    int zlo, zhi;          // the columns of a row a load may touch: z is clamped into [zlo, zhi]
    // In array coordinates: I, the sites the energy sums over and the flux lives on (the
    // lattice's interior: [2, n-3] per axis for a whole lattice), and the output region, the
    // sites this launch updates (a box within I; all of I for a whole lattice).
    int ilo[3], ihi[3];
    int olo[3], ohi[3];
    int tiles_z, tiles_y;  // output tiles of the (y, z) plane
    int zstart;            // z of the first tile's first column (at most olo[2]; below it for line-aligned tiles)
    int xchunk;            // planes per slab (the work order's outer unit)
    int projected;     // MODE_GRAD: write g - (g.phi) phi instead of g
    int baryon;        // accumulate the baryon density
    double h, dt;
    double m, m_y, m_z, m_w;  // potential masses
    double c6;                // sextic (BPS-Skyrme) coefficient
    int gradient_flow;        // MODE_STEP: phi += dt F, no velocity
};

// stencil coefficients (Sec. 3)
//   D f  = ( 2/3 (f[+1] - f[-1]) - 1/12 (f[+2] - f[-2]) ) / h
//   L f  = ( 4/3 (f[+1] + f[-1]) - 1/12 (f[+2] + f[-2]) - 5/2 f ) / h^2
//        = ( 4/3 ((f[+1] - f) + (f[-1] - f)) - 1/12 ((f[+2] - f) + (f[-2] - f)) ) / h^2
template <typename T> struct Coef {
    static constexpr T c1 = T(2.0 / 3.0);
    static constexpr T c2 = T(-1.0 / 12.0);
    static constexpr T d1 = T(4.0 / 3.0);
    static constexpr T d2 = T(-1.0 / 12.0);
    static constexpr T d0 = T(-5.0 / 2.0);
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// 1/sqrt(s) for s near 1 (a renormalisation): the hardware reciprocal square root,
// without the denormal rescaling rsqrtf wraps around it
__device__ __forceinline__ float rnorm(float s) { return __builtin_amdgcn_rsqf(s); }
__device__ __forceinline__ double rnorm(double s) { return 1.0 / sqrt(s); }

// Field access by a 32-bit byte offset from a base that is uniform over the block: the
// offset stays in one VGPR and the base in SGPRs (no 64-bit address arithmetic per
// access).  Kernel arguments are known to be global, uniform pointers; pointers read
// from a batch's job table are made so explicitly (uniform_ptr, global address space).
#define SKYR_GLOBAL __attribute__((address_space(1)))
template <typename T> using gptr = SKYR_GLOBAL T*;
template <bool GLOBAL, typename T> using fptr = std::conditional_t<GLOBAL, gptr<T>, T*>;

template <typename T> __device__ __forceinline__ T ldb(const T* base, unsigned off)
{
    return *(const T*)((const char*)base + off);
}
template <typename T> __device__ __forceinline__ void stb(T* base, unsigned off, T v)
{
    *(T*)((char*)base + off) = v;
}
template <typename T> __device__ __forceinline__ T ldb(gptr<const T> base, unsigned off)
{
    return *(gptr<const T>)((SKYR_GLOBAL const char*)base + off);
}
// Streamed accesses (the velocity read and the outputs written, used once per sweep):
// non-temporal, so that they do not displace from L2 the phi lines that neighbouring
// blocks read as their halo.
template <typename T> __device__ __forceinline__ T ldb_nt(gptr<const T> base, unsigned off)
{
    return __builtin_nontemporal_load((gptr<const T>)((SKYR_GLOBAL const char*)base + off));
}
template <typename T> __device__ __forceinline__ void stb_nt(gptr<T> base, unsigned off, T v)
{
    __builtin_nontemporal_store(v, (gptr<T>)((SKYR_GLOBAL char*)base + off));
}
template <typename T> __device__ __forceinline__ void stb(gptr<T> base, unsigned off, T v)
{
    *(gptr<T>)((SKYR_GLOBAL char*)base + off) = v;
}

// a pointer that is the same in every lane, made visibly uniform (held in SGPRs)
template <typename P> __device__ __forceinline__ P uniform_ptr(P p)
{
    const unsigned long long u = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (P)(((unsigned long long)hi << 32) | lo);
}

// max of two non-negative values (or NaN): for floats the unsigned order of the bit
// patterns is the numeric order, and a NaN pattern exceeds +inf
__device__ __forceinline__ float fmax_nonneg(float a, float b)
{
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}
__device__ __forceinline__ double fmax_nonneg(double a, double b) { return fmax(a, b); }

template <typename T> __device__ __forceinline__ T dot4(const T* a, const T* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

// det[c0 c1 c2 c3] of four column 4-vectors (expansion by 2x2 minors)
template <typename T> __device__ __forceinline__ T det4(const T* c0, const T* c1, const T* c2, const T* c3)
{
    // minors of columns (c0, c1) and (c2, c3) over row pairs
    const T m01 = c0[0] * c1[1] - c0[1] * c1[0];
    const T m02 = c0[0] * c1[2] - c0[2] * c1[0];
    const T m03 = c0[0] * c1[3] - c0[3] * c1[0];
    const T m12 = c0[1] * c1[2] - c0[2] * c1[1];
    const T m13 = c0[1] * c1[3] - c0[3] * c1[1];
    const T m23 = c0[2] * c1[3] - c0[3] * c1[2];
    const T n01 = c2[0] * c3[1] - c2[1] * c3[0];
    const T n02 = c2[0] * c3[2] - c2[2] * c3[0];
    const T n03 = c2[0] * c3[3] - c2[3] * c3[0];
    const T n12 = c2[1] * c3[2] - c2[2] * c3[1];
    const T n13 = c2[1] * c3[3] - c2[3] * c3[1];
    const T n23 = c2[2] * c3[3] - c2[3] * c3[2];
    return m01 * n23 - m02 * n13 + m03 * n12 + m12 * n03 - m13 * n02 + m23 * n01;
}

// det[c0 c1 c2 c3] and its derivatives with respect to each column (det is linear in
// every column; the derivative with respect to column k is the cofactor vector),
// from the 2x2 minors m of columns (c0, c1) and n of columns (c2, c3):
//   det = m01 n23 - m02 n13 + m03 n12 + m12 n03 - m13 n02 + m23 n01
template <typename T>
__device__ __forceinline__ T det4_cofactors(const T* c0, const T* c1, const T* c2, const T* c3, T* d0, T* d1, T* d2,
                                            T* d3)
{
    const T m01 = c0[0] * c1[1] - c0[1] * c1[0], m02 = c0[0] * c1[2] - c0[2] * c1[0];
    const T m03 = c0[0] * c1[3] - c0[3] * c1[0], m12 = c0[1] * c1[2] - c0[2] * c1[1];
    const T m13 = c0[1] * c1[3] - c0[3] * c1[1], m23 = c0[2] * c1[3] - c0[3] * c1[2];
    const T n01 = c2[0] * c3[1] - c2[1] * c3[0], n02 = c2[0] * c3[2] - c2[2] * c3[0];
    const T n03 = c2[0] * c3[3] - c2[3] * c3[0], n12 = c2[1] * c3[2] - c2[2] * c3[1];
    const T n13 = c2[1] * c3[3] - c2[3] * c3[1], n23 = c2[2] * c3[3] - c2[3] * c3[2];
    // d det / d m_ab and d det / d n_ab are the complementary minors with the signs above
    const T M01 = n23, M02 = -n13, M03 = n12, M12 = n03, M13 = -n02, M23 = n01;
    const T N23 = m01, N13 = -m02, N12 = m03, N03 = m12, N02 = -m13, N01 = m23;
    // m_ab = c0_a c1_b - c0_b c1_a:  d/dc0_a = c1_b (and -c1_a for d/dc0_b); d/dc1 likewise
    d0[0] = M01 * c1[1] + M02 * c1[2] + M03 * c1[3];
    d0[1] = -M01 * c1[0] + M12 * c1[2] + M13 * c1[3];
    d0[2] = -M02 * c1[0] - M12 * c1[1] + M23 * c1[3];
    d0[3] = -M03 * c1[0] - M13 * c1[1] - M23 * c1[2];
    d1[0] = -M01 * c0[1] - M02 * c0[2] - M03 * c0[3];
    d1[1] = M01 * c0[0] - M12 * c0[2] - M13 * c0[3];
    d1[2] = M02 * c0[0] + M12 * c0[1] - M23 * c0[3];
    d1[3] = M03 * c0[0] + M13 * c0[1] + M23 * c0[2];
    d2[0] = N01 * c3[1] + N02 * c3[2] + N03 * c3[3];
    d2[1] = -N01 * c3[0] + N12 * c3[2] + N13 * c3[3];
    d2[2] = -N02 * c3[0] - N12 * c3[1] + N23 * c3[3];
    d2[3] = -N03 * c3[0] - N13 * c3[1] - N23 * c3[2];
    d3[0] = -N01 * c2[1] - N02 * c2[2] - N03 * c2[3];
    d3[1] = N01 * c2[0] - N12 * c2[2] - N13 * c2[3];
    d3[2] = N02 * c2[0] + N12 * c2[1] - N23 * c2[3];
    d3[3] = N03 * c2[0] + N13 * c2[1] + N23 * c2[2];
    return m01 * n23 - m02 * n13 + m03 * n12 + m12 * n03 - m13 * n02 + m23 * n01;
}

// fused multiply-add in the field type
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The four components of a site, contiguous in LDS: one 16-byte (float) or two
// 16-byte (double) LDS accesses per site.
template <typename T> struct alignas(4 * sizeof(T)) Site4 {
    T v[4];
};
template <typename T> __device__ __forceinline__ void ld4(const Site4<T>* p, T (&o)[4])
{
    if constexpr (sizeof(T) == 4) {
        const float4 t = *(const float4*)p;
        o[0] = t.x, o[1] = t.y, o[2] = t.z, o[3] = t.w;
    } else {
        const double2 a = *(const double2*)p, b = *((const double2*)p + 1);
        o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
    }
}
template <typename T> __device__ __forceinline__ void st4(Site4<T>* p, const T (&i)[4])
{
    if constexpr (sizeof(T) == 4) {
        *(float4*)p = make_float4(i[0], i[1], i[2], i[3]);
    } else {
        *(double2*)p = make_double2(i[0], i[1]);
        *((double2*)p + 1) = make_double2(i[2], i[3]);
    }
}

// Tile geometry of a shape: NWI interior waves of 64 / OZ rows of OZ lanes, NWH halo
// waves whose lanes hold HPT halo positions each.
template <int NWI_, int NWH_, int HPT_, int OZ_> struct Geo {
    static constexpr int NWI = NWI_, NWH = NWH_, HPT = HPT_, OZ = OZ_;
    static constexpr int NW = NWI + NWH;
    static constexpr int THREADS = NW * 64;
    static constexpr int RPW = 64 / OZ;
    static constexpr int OY = NWI * RPW;
    // halo positions: rows -2, -1, OY, OY+1 over the OZ columns (they supply Q_y), then
    // columns -2, -1, OZ, OZ+1 of the OY rows (they supply Q_z)
    static constexpr int NHALO = 4 * OZ + 4 * OY;
    // frame: the phi sites only halo positions read (rows -4, -3, OY+2, OY+3 over the
    // columns; columns -4, -3, OZ+2, OZ+3 over the rows; the sixteen corner sites of the
    // halo rows and columns)
    static constexpr int NFRAME = 4 * OZ + 4 * OY + 16;
    static constexpr int PW = OZ + 8, PH = OY + 8;  // phi plane: rows -4 .. OY+3, columns -4 .. OZ+3
    static constexpr int QW = OZ + 4, QH = OY + 4;  // flux plane: rows -2 .. OY+1, columns -2 .. OZ+1
    static constexpr int PPLANE = PH * PW, QPLANE = QH * QW;
    static_assert(64 % OZ == 0, "an interior wave covers whole rows");
    static constexpr int FPT = (NFRAME + NWH * 64 - 1) / (NWH * 64);  // frame sites per halo lane
    static_assert(NWH * 64 * HPT >= NHALO, "every halo position has a lane");
};

template <typename T, class G> struct SweepSmem {
    Site4<T> phi[2][G::PPLANE];     // [plane parity][site]
    Site4<T> q[2][2][G::QPLANE];    // [plane parity][0: Q_y, 1: Q_z][site]
    double red[G::NW][NPART];
    int last;  // this block is the last of its field to finish the sweep
};

// EXT: 0 the plain variant (pion-mass potential, kick-drift update); 1 adds the extra
// potentials (m_y, m_z, m_w) and the gradient flow; 2 also the sextic term.  The levels
// are separate kernels so that each carries only the registers it needs.
enum : int { EXT_NONE = 0, EXT_POT = 1, EXT_SEXTIC = 2 };

// Per-launch constants.  With a^ = 12 h a (the scaled first difference), G^ = (12 h)^2 G,
// Q^ = (12 h)^3 Q and L^ = 12 h^2 Lap, the scaled gradient g^ = K g, K = (12 h)^4, is
//   g^ = lapw (L^ phi - boundary terms) - sum_i (8 (Q^_i[+1] - Q^_i[-1]) - (Q^_i[+2] - Q^_i[-2]))
//        + K V'(phi0) e0 + (sextic local term),
// and F = F^ / K with F^ = (g^.phi) phi - g^.
template <typename T> struct SweepConst {
    T lapw;                  // -K / (12 h^2) = -1728 h^2
    T ke2, ke4;              // e2 = ke2 phi.L^phi, e4 = ke4 (G^ quadratic form)
    T dt, dtK;               // dt and dt / K
    T m2, my2, mz2, mw2;     // potential energy density (unscaled)
    T m2K, my2K, mz2K, mw2K; // the same masses times K (scaled slope)
    T c6e, c6q;              // sextic: e6 = c6e det^2, flux and local weight c6q det (det of phi, a^_i)
    T invK;                  // gradient output
    double dinvK, dinvK2, dinv12h3;  // unscale the power, |F|^2 and charge-density sums
    bool more_pot, sextic, grad_flow;

    __device__ __forceinline__ void init(const SweepArgs& a, bool step_mode)
    {
        const double h = a.h, s = 12.0 * h, K = s * s * s * s;
        lapw = T(-1728.0 * h * h);
        ke2 = T(-1.0 / (24.0 * h * h));
        ke4 = T(0.5 / K);
        dt = T(a.dt);
        dtK = T(a.dt / K);
        m2 = T(a.m * a.m);
        my2 = T(a.m_y * a.m_y);
        mz2 = T(a.m_z * a.m_z);
        mw2 = T(a.m_w * a.m_w);
        m2K = T(K * a.m * a.m);
        my2K = T(K * a.m_y * a.m_y);
        mz2K = T(K * a.m_z * a.m_z);
        mw2K = T(K * a.m_w * a.m_w);
        c6e = T(0.5 * a.c6 / (K * s * s));
        c6q = T(a.c6 / (s * s));
        invK = T(1.0 / K);
        dinvK = 1.0 / K;
        dinvK2 = 1.0 / (K * K);
        dinv12h3 = 1.0 / (s * s * s);
        more_pot = a.m_y != 0.0 || a.m_z != 0.0 || a.m_w != 0.0;
        sextic = a.c6 != 0.0;
        grad_flow = step_mode && a.gradient_flow != 0;
    }
};

// One item of a field's work: output planes [xa, xe) of tile (ty, tz).
struct Segment {
    int ty, tz, xa, xe;
};

// The work of a field is cut into items, one (slab, tile) pair each (slabs of xchunk
// planes along x), numbered slab by slab and tile by tile within a slab.  Logical block
// b of nb takes items b, b + nb, ...; a launch normally has one block per item, so that
// the blocks of neighbouring tiles march through the same planes at the same time and
// the phi lines of their shared halo are read from L2 once.
__device__ __forceinline__ Segment item_segment(int item, int tiles, int tiles_z, int x0, int nx, int xchunk)
{
    const int slab = item / tiles, tile = item - slab * tiles;
    Segment s;
    s.ty = tile / tiles_z;
    s.tz = tile - s.ty * tiles_z;
    s.xa = x0 + slab * xchunk;
    s.xe = x0 + min(nx, (slab + 1) * xchunk);
    return s;
}

// A march over output planes [xa, xe) takes (xe - xa) + 4 steps (flux planes xa-2 ..
// xe+1); it runs in whole groups of five and so starts this many planes early.
__device__ __forceinline__ int march_lead(int xa, int xe) { return (5 - ((xe - xa) + 4) % 5) % 5; }

// Fields, flags and sums shared by the two roles.
template <typename T, bool FROM_TABLE> struct SweepCommon {
    // global-memory pointers, uniform over the block
    gptr<const T> pin[4];
    gptr<T> pout[4];
    gptr<T> vel[4];
    gptr<T> gout[4];
    int n0, n1, n2;
    int zlo, zhi;        // the columns of a row a load may touch
    int ilo[3], ihi[3];  // I in array coordinates
    int olo1, olo2, ohi1, ohi2;  // the output region in y and z
    unsigned plane_b;  // bytes per x-plane of one component
    bool redo, renorm64, projected, baryon, has_grad;
    int restore;       // RESTORE_*: this sweep only rewrites the velocity

    __device__ __forceinline__ void load(unsigned off, int x, T (&dst)[4]) const
    {
        const unsigned base = (unsigned)clampi(x, 0, n0 - 1) * plane_b;
#pragma unroll
        for (int A = 0; A < 4; ++A) dst[A] = ldb(pin[A], base + off);
    }
    __device__ __forceinline__ unsigned site_off(int y, int z) const
    {
        return (unsigned)(clampi(y, 0, n1 - 1) * n2 + clampi(z, zlo, zhi)) * (unsigned)sizeof(T);
    }
};

// --------------------------------------------------------------- interior role
// One output site per lane: row, col of the tile.
template <typename T, class G, int MODE, bool FROM_TABLE, int EXT> struct Interior {
    using Smem = SweepSmem<T, G>;
    Smem& sm;
    const SweepConst<T>& k;
    const SweepCommon<T, FROM_TABLE>& cm;
    int row, col;
    int pidx, qidx;    // LDS index of the own site in a phi plane and in a flux plane
    unsigned off;      // byte offset of the own site within a plane
    int xa, xe;
    bool out;          // the own site is in the output region (in y and z)
    bool in_i;         // the own site is in I (in y and z); the flux there is not zero
    bool yz_near;      // an output site within two sites of a y or z face of I
    unsigned outside;  // bit d: the y/z neighbour d (O_* below) lies outside I
    enum : unsigned { O_YP1 = 1, O_YM1 = 2, O_YP2 = 4, O_YM2 = 8, O_ZP1 = 16, O_ZM1 = 32, O_ZP2 = 64, O_ZM2 = 128 };

    T ring[5][4];  // phi of planes j-2 .. j+2 (slot = plane offset + 2 + step, mod 5)
    T acc[5][4];   // scaled gradient accumulators of planes j-2 .. j+2 (same slots)
    T nxt[4];      // prefetched phi(j+3)
    T vnxt[4];     // prefetched velocity of plane j-1

    double pe2 = 0.0, pe4 = 0.0, pe0 = 0.0, pe6 = 0.0, pb_sum = 0.0;
    double pp = 0.0;  // scaled power F^ . v of the incoming velocity
    T pf2 = T(0);     // largest scaled |F^|^2

    __device__ __forceinline__ Interior(Smem& s, const SweepConst<T>& kk, const SweepCommon<T, FROM_TABLE>& c, int tid)
        : sm(s), k(kk), cm(c)
    {
        row = tid / G::OZ;
        col = tid - row * G::OZ;
        pidx = (row + 4) * G::PW + col + 4;
        qidx = (row + 2) * G::QW + col + 2;
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
    // K dV/dphi0
    __device__ __forceinline__ T slopeK(T p0) const
    {
        const T u = T(1) - p0;
        T d = -k.m2K;
        if constexpr (EXT) {
            if (k.more_pot) d -= k.my2K * p0 + k.mz2K * u + k.mw2K * u * u * u;
        }
        return d;
    }

    __device__ __forceinline__ void setup(const Segment& s, int tiles_z_start)
    {
        const int y0 = cm.olo1 + s.ty * G::OY, z0 = tiles_z_start + s.tz * G::OZ;
        const int y = y0 + row, z = z0 + col;
        const int ly = cm.ilo[1], hy = cm.ihi[1], lz = cm.ilo[2], hz = cm.ihi[2];
        out = (y <= cm.ohi1) && (z >= cm.olo2) && (z <= cm.ohi2);
        in_i = (y >= ly) && (y <= hy) && (z >= lz) && (z <= hz);
        outside = (y + 1 > hy ? O_YP1 : 0u) | (y - 1 < ly ? O_YM1 : 0u) | (y + 2 > hy ? O_YP2 : 0u) |
                  (y - 2 < ly ? O_YM2 : 0u) | (z + 1 > hz ? O_ZP1 : 0u) | (z - 1 < lz ? O_ZM1 : 0u) |
                  (z + 2 > hz ? O_ZP2 : 0u) | (z - 2 < lz ? O_ZM2 : 0u);
        yz_near = out && outside != 0u;
        off = cm.site_off(y, z);
        xa = s.xa;
        xe = s.xe;
    }

    template <int SM2, int SM1, int S0, int SP1, int SP2>
    __device__ __forceinline__ void boundary_terms(int j, const Site4<T>* P)
    {
        if (!out) return;
        const int lx = cm.ilo[0], hx = cm.ihi[0];
        const T* pa0 = P[pidx].v;
        constexpr int W = 4 * G::PW;  // one row of sites, in elements
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            const T* pa = pa0 + A;
            T o1 = T(0), o2 = T(0);  // outside first / second neighbours
            if (j + 1 > hx) o1 += ring[SP1][A];
            if (j - 1 < lx) o1 += ring[SM1][A];
            if (j + 2 > hx) o2 += ring[SP2][A];
            if (j - 2 < lx) o2 += ring[SM2][A];
            if (outside & O_YP1) o1 += pa[W];
            if (outside & O_YM1) o1 += pa[-W];
            if (outside & O_ZP1) o1 += pa[4];
            if (outside & O_ZM1) o1 += pa[-4];
            if (outside & O_YP2) o2 += pa[2 * W];
            if (outside & O_YM2) o2 += pa[-2 * W];
            if (outside & O_ZP2) o2 += pa[8];
            if (outside & O_ZM2) o2 += pa[-8];
            // + 1/2 the outside terms of Lap phi: 12 h^2 x that is 8 o1 - o2 / 2, and L^ enters
            // the scaled gradient with weight lapw < 0 and the opposite sign
            acc[S0][A] = fmaT(k.lapw, fmaT(T(0.5), o2, T(-8) * o1), acc[S0][A]);
        }
    }

    template <int U> __device__ __forceinline__ void step(int j, int pb)
    {
        constexpr int SM2 = U % 5, SM1 = (U + 1) % 5, S0 = (U + 2) % 5, SP1 = (U + 3) % 5, SP2 = (U + 4) % 5;
        const int qb = pb ^ 1;
        // Opaque to the optimiser from here on: the LDS and global addresses and the x-stencil
        // arithmetic of this plane are then formed within it, not carried over from an
        // earlier plane in registers across the barriers.
        asm volatile("" : "+v"(pidx), "+v"(qidx), "+v"(off));
#pragma unroll
        for (int sl = 0; sl < 5; ++sl)
            asm volatile("" : "+v"(ring[sl][0]), "+v"(ring[sl][1]), "+v"(ring[sl][2]), "+v"(ring[sl][3]));
        // stage phi(j+1) into the other phi buffer (its last reads, of phi(j-1), came before
        // the last barrier), then prefetch
        st4(&sm.phi[qb][pidx], ring[SP1]);
        // the velocity of output plane j-2 was prefetched one plane earlier; the velocity of
        // plane j-1 is loaded now, before the prefetch of phi(j+3) (loads complete in order)
        T vcur[4];
        if constexpr (MODE == MODE_STEP) {
            const unsigned vb = (unsigned)clampi(j - 1, 0, cm.n0 - 1) * cm.plane_b;
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                vcur[A] = vnxt[A];
                vnxt[A] = ldb_nt((gptr<const T>)cm.vel[A], vb + off);
            }
        }
#pragma unroll
        for (int A = 0; A < 4; ++A) ring[SP2][A] = nxt[A];
        cm.load(off, j + 3, nxt);
        if constexpr (MODE == MODE_STEP) {
            if (cm.redo) {  // a redo sweep starts from zero velocity
#pragma unroll
                for (int A = 0; A < 4; ++A) vcur[A] = T(0);
            }
        }
        const bool j_in = (j >= cm.ilo[0]) && (j <= cm.ihi[0]);
        const bool j_out = (j >= xa) && (j < xe);

        const Site4<T>* P = sm.phi[pb];
        T c[4], ax[4], ay[4], az[4];
        T Ym2[4], Ym1[4], Yp1[4], Yp2[4], Zm2[4], Zm1[4], Zp1[4], Zp2[4];
        ld4(P + pidx - 2 * G::PW, Ym2);
        ld4(P + pidx - G::PW, Ym1);
        ld4(P + pidx + G::PW, Yp1);
        ld4(P + pidx + 2 * G::PW, Yp2);
        ld4(P + pidx - 2, Zm2);
        ld4(P + pidx - 1, Zm1);
        ld4(P + pidx + 1, Zp1);
        ld4(P + pidx + 2, Zp2);
        T cl = T(0);
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            const T cc = ring[S0][A];
            const T xm2 = ring[SM2][A], xm1 = ring[SM1][A], xp1 = ring[SP1][A], xp2 = ring[SP2][A];
            const T ym2 = Ym2[A], ym1 = Ym1[A], yp1 = Yp1[A], yp2 = Yp2[A];
            const T zm2 = Zm2[A], zm1 = Zm1[A], zp1 = Zp1[A], zp2 = Zp2[A];
            c[A] = cc;
            ax[A] = fmaT(T(8), xp1 - xm1, xm2 - xp2);
            ay[A] = fmaT(T(8), yp1 - ym1, ym2 - yp2);
            az[A] = fmaT(T(8), zp1 - zm1, zm2 - zp2);
            if (j_out) {
                T lap;  // 12 h^2 Lap phi
                if constexpr (sizeof(T) == 4) {
                    // differences from the centre: no cancellation of O(1) terms in single precision
                    const T s1 = ((xp1 - cc) + (xm1 - cc)) + ((yp1 - cc) + (ym1 - cc)) + ((zp1 - cc) + (zm1 - cc));
                    const T s2 = ((xp2 - cc) + (xm2 - cc)) + ((yp2 - cc) + (ym2 - cc)) + ((zp2 - cc) + (zm2 - cc));
                    lap = fmaT(T(16), s1, -s2);
                } else {
                    const T s1 = ((xp1 + xm1) + (yp1 + ym1)) + (zp1 + zm1);
                    const T s2 = ((xp2 + xm2) + (yp2 + ym2)) + (zp2 + zm2);
                    lap = fmaT(T(-90), cc, fmaT(T(16), s1, -s2));
                }
                cl = fmaT(cc, lap, cl);
                acc[S0][A] = fmaT(k.lapw, lap, acc[S0][A]);
            }
        }
        // The E2 part of the gradient is -1/2 (Lap phi + Lap(1_I phi)): the terms of Lap phi
        // whose neighbour lies outside I count half.  Only sites within two of a face of I
        // have such terms; a wave none of whose sites has one skips this.
        const bool x_near = (j <= cm.ilo[0] + 1) || (j >= cm.ihi[0] - 1);
        if (j_out && (x_near || __builtin_amdgcn_ballot_w64(yz_near) != 0)) boundary_terms<SM2, SM1, S0, SP1, SP2>(j, P);

        const T gxx = dot4(ax, ax), gyy = dot4(ay, ay), gzz = dot4(az, az);
        const T gxy = dot4(ax, ay), gxz = dot4(ax, az), gyz = dot4(ay, az);
        const bool valid = in_i && j_in;
        // the flux vanishes outside I: zero the Gram entries it is built from
        const T fxx = valid ? gxx : T(0), fyy = valid ? gyy : T(0), fzz = valid ? gzz : T(0);
        const T fxy = valid ? gxy : T(0), fxz = valid ? gxz : T(0), fyz = valid ? gyz : T(0);
        const T sx = fyy + fzz, sy = fxx + fzz, sz = fxx + fyy;
        T qx[4], qy[4], qz[4];
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            qx[A] = fmaT(sx, ax[A], -fmaT(fxy, ay[A], fxz * az[A]));
            qy[A] = fmaT(sy, ay[A], -fmaT(fxy, ax[A], fyz * az[A]));
            qz[A] = fmaT(sz, az[A], -fmaT(fxz, ax[A], fyz * ay[A]));
        }
        T e6 = T(0);
        if constexpr (EXT == EXT_SEXTIC) {
            if (k.sextic) {
                // e6 = c6 det^2 / 2, det = det[phi, a_x, a_y, a_z]: flux c6 det ddet/da_i (zero
                // outside I) and the local term c6 det ddet/dphi
                T C0[4], C1[4], C2[4], C3[4];
                const T det = det4_cofactors(c, ax, ay, az, C0, C1, C2, C3);
                const T dv = valid ? k.c6q * det : T(0);
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    qx[A] = fmaT(dv, C1[A], qx[A]);
                    qy[A] = fmaT(dv, C2[A], qy[A]);
                    qz[A] = fmaT(dv, C3[A], qz[A]);
                    acc[S0][A] = fmaT(dv, C0[A], acc[S0][A]);
                }
                e6 = k.c6e * det * det;
            }
        }
        st4(&sm.q[pb][0][qidx], qy);
        st4(&sm.q[pb][1][qidx], qz);
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            // x-divergence pushed to the accumulators of planes j-2 .. j+2
            acc[SM1][A] = fmaT(T(-8), qx[A], acc[SM1][A]);
            acc[SP1][A] = fmaT(T(8), qx[A], acc[SP1][A]);
            acc[SM2][A] += qx[A];
            acc[SP2][A] -= qx[A];
        }
        if (out && j_out) {
            const T e2 = k.ke2 * cl;
            const T e4 = k.ke4 * (gxx * gyy + gxx * gzz + gyy * gzz - gxy * gxy - gxz * gxz - gyz * gyz);
            const T e0 = potential(c[0]);
            if constexpr (MODE == MODE_STEP) {
                pe2 += (double)(e2 + e4 + e0 + e6);  // the flow needs the total energy only
            } else {
                pe2 += (double)e2;
                pe4 += (double)e4;
                pe0 += (double)e0;
                pe6 += (double)e6;
                if (cm.baryon) pb_sum += (double)det4(c, ax, ay, az);
            }
        }

        // y- and z-divergence of the flux of plane j-1 (written before the last barrier)
        if (j - 1 >= xa && j - 1 < xe) {
            const Site4<T>* fy = sm.q[qb][0] + qidx;
            const Site4<T>* fz = sm.q[qb][1] + qidx;
            T ym2[4], ym1[4], yp1[4], yp2[4], zm2[4], zm1[4], zp1[4], zp2[4];
            ld4(fy - 2 * G::QW, ym2);
            ld4(fy - G::QW, ym1);
            ld4(fy + G::QW, yp1);
            ld4(fy + 2 * G::QW, yp2);
            ld4(fz - 2, zm2);
            ld4(fz - 1, zm1);
            ld4(fz + 1, zp1);
            ld4(fz + 2, zp2);
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                const T t = (ym1[A] - yp1[A]) + (zm1[A] - zp1[A]);
                const T u = (yp2[A] - ym2[A]) + (zp2[A] - zm2[A]);
                acc[SM1][A] = fmaT(T(8), t, acc[SM1][A]) + u;
            }
        }

        // output plane j-2 is complete
        if (j - 2 >= xa && j - 2 < xe && out) {
            const unsigned base = (unsigned)(j - 2) * cm.plane_b + off;
            T g[4], p[4], f[4];
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                g[A] = acc[SM2][A];
                p[A] = ring[SM2][A];
            }
            g[0] += slopeK(p[0]);
            const T gp = dot4(g, p);
#pragma unroll
            for (int A = 0; A < 4; ++A) f[A] = fmaT(gp, p[A], -g[A]);  // F^ = (g^.phi) phi - g^
            pf2 = fmax_nonneg(pf2, dot4(f, f));
            if constexpr (MODE == MODE_STEP) {
                pp += (double)dot4(f, vcur);  // the product in the field precision, the sum in double
                if (cm.restore) {
#pragma unroll
                    for (int A = 0; A < 4; ++A)
                        stb_nt(cm.vel[A], base, cm.restore == RESTORE_ZERO ? T(0) : fmaT(-k.dtK, f[A], vcur[A]));
                } else {
                    T v[4], q[4], pn[4];
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        if constexpr (EXT) {
                            v[A] = k.grad_flow ? T(0) : fmaT(k.dtK, f[A], vcur[A]);
                            q[A] = k.grad_flow ? fmaT(k.dtK, f[A], p[A]) : fmaT(k.dt, v[A], p[A]);
                        } else {
                            v[A] = fmaT(k.dtK, f[A], vcur[A]);
                            q[A] = fmaT(k.dt, v[A], p[A]);
                        }
                    }
                    if (cm.renorm64) {
                        const double s2 = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] +
                                          (double)q[3] * q[3];
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
                }
            } else {
                if (cm.has_grad) {
#pragma unroll
                    for (int A = 0; A < 4; ++A) stb_nt(cm.gout[A], base, (cm.projected ? -f[A] : g[A]) * k.invK);
                }
            }
        }
#pragma unroll
        for (int A = 0; A < 4; ++A) acc[SM2][A] = T(0);  // the slot starts plane j+3
        __syncthreads();
    }

    // the march over one segment
    __device__ __forceinline__ void march()
    {
#pragma unroll
        for (int s = 0; s < 5; ++s)
#pragma unroll
            for (int A = 0; A < 4; ++A) acc[s][A] = T(0);
        // the march runs in groups of five planes; it starts `lead` planes early so that the
        // last group ends with output plane xe-1 (the early planes reach no output plane)
        const int lead = march_lead(xa, xe);
        const int js = xa - 2 - lead;  // first flux plane; ring slots 0 .. 3 hold planes js-2 .. js+1
        cm.load(off, js - 2, ring[0]);
        cm.load(off, js - 1, ring[1]);
        cm.load(off, js, ring[2]);
        cm.load(off, js + 1, ring[3]);
        cm.load(off, js + 2, nxt);
        if constexpr (MODE == MODE_STEP) {
            const unsigned vb = (unsigned)clampi(js - 2, 0, cm.n0 - 1) * cm.plane_b;
#pragma unroll
            for (int A = 0; A < 4; ++A) vnxt[A] = ldb_nt((gptr<const T>)cm.vel[A], vb + off);
        }
        st4(&sm.phi[0][pidx], ring[2]);
        __syncthreads();
        const int nst = (xe - xa) + 4 + lead;
        for (int st = 0; st < nst; st += 5) {
            const int j = js + st, pb = st & 1;
            step<0>(j, pb);
            step<1>(j + 1, pb ^ 1);
            step<2>(j + 2, pb);
            step<3>(j + 3, pb ^ 1);
            step<4>(j + 4, pb);
        }
    }
};

// ------------------------------------------------------------------ halo role
// HPT halo positions per lane; each supplies one flux component: Q_y on the y-halo
// rows, Q_z on the z-halo columns.
template <typename T, class G, bool FROM_TABLE, int EXT> struct Halo {
    using Smem = SweepSmem<T, G>;
    static constexpr int HPT = G::HPT;
    Smem& sm;
    const SweepConst<T>& k;
    const SweepCommon<T, FROM_TABLE>& cm;
    int pos[HPT];        // halo position index (>= NHALO: none)
    int pidx[HPT];       // LDS index in a phi plane
    int qidx[HPT];       // LDS index of the supplied flux (Q_y or Q_z plane, component 0)
    unsigned off[HPT];
    bool active[HPT], is_y[HPT], vyz[HPT];
    int hr[HPT], hc[HPT];  // tile-relative row and column
    static constexpr int FPT = G::FPT;
    bool floader[FPT];     // frame sites of this lane
    int fr[FPT], fc[FPT];  // their tile-relative rows and columns
    int fidx[FPT];         // LDS index in a phi plane
    unsigned foff[FPT];    // byte offset in the current segment
    int xa, xe;
    T ring[HPT][5][4];
    T nxt[HPT][4];
    T fnxt[FPT][4];        // prefetched frame sites of phi(j+2)

    __device__ __forceinline__ Halo(Smem& s, const SweepConst<T>& kk, const SweepCommon<T, FROM_TABLE>& c, int u)
        : sm(s), k(kk), cm(c)
    {
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int p = u + i * G::NWH * 64;
            active[i] = p < G::NHALO;
            const int pp = active[i] ? p : 0;
            int r, cc;
            bool yh;
            if (pp < 4 * G::OZ) {
                const int q = pp / G::OZ;
                r = q < 2 ? q - 2 : G::OY + q - 2;
                cc = pp - q * G::OZ;
                yh = true;
            } else {
                const int g = pp - 4 * G::OZ, q = g & 3;
                r = g >> 2;
                cc = q < 2 ? q - 2 : G::OZ + q - 2;
                yh = false;
            }
            hr[i] = r;
            hc[i] = cc;
            is_y[i] = yh;
            pidx[i] = (r + 4) * G::PW + cc + 4;
            qidx[i] = (yh ? 0 : G::QPLANE) + (r + 2) * G::QW + cc + 2;
        }
#pragma unroll
        for (int i = 0; i < FPT; ++i) {
            const int f0 = u + i * G::NWH * 64;
            floader[i] = f0 < G::NFRAME;
            const int f = floader[i] ? f0 : 0;
            int r, cc;
            if (f < 4 * G::OZ) {
                const int q = f / G::OZ;
                r = q < 2 ? q - 4 : G::OY + q;
                cc = f - q * G::OZ;
            } else if (f < 4 * G::OZ + 4 * G::OY) {
                const int g = f - 4 * G::OZ, q = g & 3;
                r = g >> 2;
                cc = q < 2 ? q - 4 : G::OZ + q;
            } else {
                const int g = f - 4 * G::OZ - 4 * G::OY, qr = g >> 2, qc = g & 3;
                r = qr < 2 ? qr - 2 : G::OY + qr - 2;
                cc = qc < 2 ? qc - 2 : G::OZ + qc - 2;
            }
            fr[i] = r;
            fc[i] = cc;
            fidx[i] = (r + 4) * G::PW + cc + 4;
        }
    }

    __device__ __forceinline__ void setup(const Segment& s, int tiles_z_start)
    {
        const int y0 = cm.olo1 + s.ty * G::OY, z0 = tiles_z_start + s.tz * G::OZ;
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            const int y = y0 + hr[i], z = z0 + hc[i];
            vyz[i] = (y >= cm.ilo[1]) && (y <= cm.ihi[1]) && (z >= cm.ilo[2]) && (z <= cm.ihi[2]);
            off[i] = cm.site_off(y, z);
        }
#pragma unroll
        for (int i = 0; i < FPT; ++i) foff[i] = cm.site_off(y0 + fr[i], z0 + fc[i]);
        xa = s.xa;
        xe = s.xe;
    }

    template <int U> __device__ __forceinline__ void step(int j, int pb)
    {
        constexpr int SM2 = U % 5, SM1 = (U + 1) % 5, S0 = (U + 2) % 5, SP1 = (U + 3) % 5, SP2 = (U + 4) % 5;
        const int qb = pb ^ 1;
        Site4<T>* Pn = sm.phi[qb];
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            asm volatile("" : "+v"(pidx[i]), "+v"(qidx[i]), "+v"(off[i]));
#pragma unroll
            for (int sl = 0; sl < 5; ++sl)
                asm volatile("" : "+v"(ring[i][sl][0]), "+v"(ring[i][sl][1]), "+v"(ring[i][sl][2]), "+v"(ring[i][sl][3]));
            // stage phi(j+1) into the other phi buffer, then prefetch
            if (active[i]) st4(Pn + pidx[i], ring[i][SP1]);
#pragma unroll
            for (int A = 0; A < 4; ++A) ring[i][SP2][A] = nxt[i][A];
            if (active[i]) cm.load(off[i], j + 3, nxt[i]);
        }
        // the frame sites of phi(j+1) likewise
#pragma unroll
        for (int i = 0; i < FPT; ++i) {
            asm volatile("" : "+v"(fidx[i]), "+v"(foff[i]));
            if (floader[i]) {
                st4(Pn + fidx[i], fnxt[i]);
                cm.load(foff[i], j + 2, fnxt[i]);
            }
        }
        const bool j_in = (j >= cm.ilo[0]) && (j <= cm.ihi[0]);
        const Site4<T>* P = sm.phi[pb];
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            if (!active[i]) continue;
            T c[4], ax[4], ap[4], aq[4];
            const bool yh = is_y[i];
            T Ym2[4], Ym1[4], Yp1[4], Yp2[4], Zm2[4], Zm1[4], Zp1[4], Zp2[4];
            const Site4<T>* pa = P + pidx[i];
            ld4(pa - 2 * G::PW, Ym2);
            ld4(pa - G::PW, Ym1);
            ld4(pa + G::PW, Yp1);
            ld4(pa + 2 * G::PW, Yp2);
            ld4(pa - 2, Zm2);
            ld4(pa - 1, Zm1);
            ld4(pa + 1, Zp1);
            ld4(pa + 2, Zp2);
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                c[A] = ring[i][S0][A];
                ax[A] = fmaT(T(8), ring[i][SP1][A] - ring[i][SM1][A], ring[i][SM2][A] - ring[i][SP2][A]);
                const T ay = fmaT(T(8), Yp1[A] - Ym1[A], Ym2[A] - Yp2[A]);
                const T az = fmaT(T(8), Zp1[A] - Zm1[A], Zm2[A] - Zp2[A]);
                ap[A] = yh ? ay : az;
                aq[A] = yh ? az : ay;
            }
            const bool valid = vyz[i] && j_in;
            const T gxx = valid ? dot4(ax, ax) : T(0), gqq = valid ? dot4(aq, aq) : T(0);
            const T gpx = valid ? dot4(ap, ax) : T(0), gpq = valid ? dot4(ap, aq) : T(0);
            const T sp = gxx + gqq;
            T qp[4];
#pragma unroll
            for (int A = 0; A < 4; ++A) qp[A] = fmaT(sp, ap[A], -fmaT(gpx, ax[A], gpq * aq[A]));
            if constexpr (EXT == EXT_SEXTIC) {
                if (k.sextic) {
                    // the sextic flux of the supplied direction, c6 det ddet/da_p
                    T ay[4], az[4], C0[4], C1[4], C2[4], C3[4];
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        ay[A] = yh ? ap[A] : aq[A];
                        az[A] = yh ? aq[A] : ap[A];
                    }
                    const T det = det4_cofactors(c, ax, ay, az, C0, C1, C2, C3);
                    const T dv = valid ? k.c6q * det : T(0);
#pragma unroll
                    for (int A = 0; A < 4; ++A) qp[A] = fmaT(dv, yh ? C2[A] : C3[A], qp[A]);
                }
            }
            st4(sm.q[pb][0] + qidx[i], qp);
        }
        __syncthreads();
    }

    __device__ __forceinline__ void march()
    {
        const int lead = march_lead(xa, xe);
        const int js = xa - 2 - lead;
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            if (!active[i]) continue;
            cm.load(off[i], js - 2, ring[i][0]);
            cm.load(off[i], js - 1, ring[i][1]);
            cm.load(off[i], js, ring[i][2]);
            cm.load(off[i], js + 1, ring[i][3]);
            cm.load(off[i], js + 2, nxt[i]);
        }
        Site4<T>* Q = sm.phi[0];
#pragma unroll
        for (int i = 0; i < HPT; ++i) {
            if (!active[i]) continue;
            st4(Q + pidx[i], ring[i][2]);
        }
#pragma unroll
        for (int i = 0; i < FPT; ++i) {
            if (!floader[i]) continue;
            T f0[4];
            cm.load(foff[i], js, f0);
            cm.load(foff[i], js + 1, fnxt[i]);
            st4(Q + fidx[i], f0);
        }
        __syncthreads();
        const int nst = (xe - xa) + 4 + lead;
        for (int st = 0; st < nst; st += 5) {
            const int j = js + st, pb = st & 1;
            step<0>(j, pb);
            step<1>(j + 1, pb ^ 1);
            step<2>(j + 2, pb);
            step<3>(j + 3, pb ^ 1);
            step<4>(j + 4, pb);
        }
    }
};

// The flow's decision after the sweep over phi_k (Sec. 3), from the sums of that sweep
// (s: the reduced partial-sum slots): arrest when E_k > E_{k-1} (energy rule) or when the
// power h^3 sum F_k . v_k < 0 (power rule), re-running the sweep with v_k = 0; stop when
// max|F_k| < tol; otherwise accept the update (swap the field buffers).  One thread.
__device__ inline void flow_decide(const double* s, Ctl* ctl)
{
    // the flow sweep sums the whole energy density in slot P_E2 (slots P_E4, P_E0, P_E6 are zero)
    const double E = ctl->h3 * s[P_E2];
    const double r = sqrt(s[P_F2]);
    ctl->sweeps += 1;
    ctl->E = E;
    ctl->P = ctl->h3 * s[P_POW];
    ctl->max_force = r;
    if (!isfinite(E) || !isfinite(r)) {
        ctl->done = 1;
        ctl->status = 3;
        return;
    }
    bool arrest = false;
    if (!ctl->redo && ((ctl->flow_mode == SKYR_ARREST_POWER && ctl->P < 0.0) ||
                       (ctl->flow_mode == SKYR_ARREST_ENERGY && E > ctl->E_prev))) {
        arrest = true;
        ctl->arrests += 1;
    }
    if (r < ctl->tol) {
        ctl->done = 1;
        ctl->status = 1;
        // the sweep wrote v_k + dt F_k over v_k; the next one puts v_k back (zero if v_k was
        // reset by an arrest at this step or was zero on this redo sweep)
        const bool v_zero = ctl->redo || arrest || ctl->flow_mode == SKYR_GRADIENT_FLOW;
        ctl->restore = v_zero ? RESTORE_ZERO : RESTORE_UNKICK;
        ctl->redo = 0;
        return;
    }
    if (arrest) {
        ctl->redo = 1;
        ctl->redo_sweeps += 1;
        return;
    }
    ctl->cur ^= 1;
    ctl->redo = 0;
    ctl->E_prev = E;
    ctl->steps += 1;
    if (ctl->steps >= ctl->target) {
        ctl->done = 1;
        ctl->status = 2;
    }
}

// End of a step sweep: every block has published its partial sums; the block that
// finishes last (a ticket counter in the control block, no waiting) sums them all in a
// fixed order (thread t takes blocks t, t + THREADS, ..., then a fixed butterfly per wave
// and the waves in order) and takes the flow's decision.  A restore sweep only clears the
// restore flag; a sweep on a held control block only resets the ticket.
// The partial sums are agent-scope atomic stores, complete (s_waitcnt) before the block's
// ticket, and the last block reads them with agent-scope atomic loads: they are coherent
// across the XCDs' L2 caches without a device-wide fence, which would write back and
// invalidate the whole L2 of the block's XCD while its neighbours still read halo lines.
// The fields of the control block other than the ticket change only between launches.
// Smem: shared memory with `int last` and `double red[NW][NPART]`; THREADS threads in NW waves.
template <int THREADS, int NW, class Smem>
__device__ __forceinline__ void finish_step(const double* part, int nb, Ctl* ctl, bool restore, Smem& sm)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        __builtin_amdgcn_s_waitcnt(0);  // this block's partial sums before its ticket
        sm.last = __hip_atomic_fetch_add(&ctl->ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nb - 1;
    }
    __syncthreads();
    if (!sm.last) return;
    if (restore || ctl->hold) {
        if (tid == 0) {
            if (restore) ctl->restore = RESTORE_NONE;
            __hip_atomic_store(&ctl->ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    double v[NRED];
#pragma unroll
    for (int i = 0; i < NRED; ++i) v[i] = 0.0;
    for (int b = tid; b < nb; b += THREADS) {
        const double* p = part + (size_t)b * NPART;
#pragma unroll
        for (int i = 0; i < NRED; ++i) {
            const double x = __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            v[i] = (i == P_F2) ? fmax(v[i], x) : v[i] + x;
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < NRED; ++i) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double w = __shfl_xor(v[i], o);
            v[i] = (i == P_F2) ? fmax(v[i], w) : v[i] + w;
        }
        if (lane == 0) sm.red[wave][i] = v[i];
    }
    __syncthreads();
    if (tid == 0) {
        double sum[NRED];
#pragma unroll
        for (int i = 0; i < NRED; ++i) sum[i] = 0.0;
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int i = 0; i < NRED; ++i) sum[i] = (i == P_F2) ? fmax(sum[i], sm.red[w][i]) : sum[i] + sm.red[w][i];
        flow_decide(sum, ctl);
        __hip_atomic_store(&ctl->ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One block's share of one field: logical block b of nb blocks, which takes the items b,
// b + nb, ... of the field's work.  Used by the single-field and the batched kernels
// (FROM_TABLE: the arguments were read from the batch's job table).
template <typename T, class G, int MODE, bool FROM_TABLE = false, int EXT = EXT_NONE>
__device__ __forceinline__ void sweep_block(const SweepArgs& a, int b, int nb, SweepSmem<T, G>& sm)
{
    SweepCommon<T, FROM_TABLE> cm;
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
    const long long N3 = a.cstride;
    {
        const T* pin = (const T*)(MODE == MODE_STEP && cur ? (const void*)a.phi1 : a.phi0);
        T* pout = (T*)(MODE == MODE_STEP ? (cur ? (void*)a.phi0 : a.phi1) : nullptr);
        T* pvel = (T*)a.vel;
        T* pgrad = (T*)a.grad;
        // the same for the whole block (kernel arguments or the job table): kept in SGPRs
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
    SweepConst<T> k;
    k.init(a, MODE == MODE_STEP);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tiles = a.tiles_y * a.tiles_z;
    const int x0 = a.olo[0], nx = a.ohi[0] - a.olo[0] + 1;
    const int items = tiles * ((nx + a.xchunk - 1) / a.xchunk);

    double vals[7] = {0, 0, 0, 0, 0, 0, 0};
    if (wave < G::NWI) {
        Interior<T, G, MODE, FROM_TABLE, EXT> it(sm, k, cm, tid);
        for (int item = b; item < items; item += nb) {
            it.setup(item_segment(item, tiles, a.tiles_z, x0, nx, a.xchunk), a.zstart);
            it.march();
        }
        vals[0] = it.pe2;
        vals[1] = it.pe4;
        vals[2] = it.pe0;
        vals[3] = it.pb_sum * k.dinv12h3;
        vals[4] = (double)it.pf2 * k.dinvK2;
        vals[5] = it.pp * k.dinvK;
        vals[6] = it.pe6;
    } else {
        Halo<T, G, FROM_TABLE, EXT> hl(sm, k, cm, tid - G::NWI * 64);
        for (int item = b; item < items; item += nb) {
            hl.setup(item_segment(item, tiles, a.tiles_z, x0, nx, a.xchunk), a.zstart);
            hl.march();
        }
    }

    // block reduction of the partial sums (fixed order)
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        double v = vals[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double w = __shfl_xor(v, o);
            v = (i == P_F2) ? fmax(v, w) : v + w;
        }
        vals[i] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 7; ++i) sm.red[wave][i] = vals[i];
    }
    __syncthreads();
    if (tid == 0) {
        double sum[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int wv = 0; wv < G::NWI; ++wv)
            for (int i = 0; i < 7; ++i) sum[i] = (i == P_F2) ? fmax(sum[i], sm.red[wv][i]) : sum[i] + sm.red[wv][i];
        double* o = a.partials + (size_t)b * NPART;
        for (int i = 0; i < 7; ++i) __hip_atomic_store(o + i, sum[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if constexpr (MODE == MODE_STEP) finish_step<G::THREADS, G::NW>(a.partials, nb, a.ctl, cm.restore != RESTORE_NONE, sm);
}

// Blocks are dispatched round-robin over the eight XCDs (block i to XCD i % 8).
// The logical index gives each XCD a contiguous run of the work: neighbouring
// tiles of one slab, which march through the same planes and share halo rows
// in one L2.
__device__ __forceinline__ int xcd_logical_block(int i, int n)
{
    const int xcd = i % 8, q8 = n / 8, r8 = n % 8;
    return xcd * q8 + min(xcd, r8) + i / 8;
}

template <typename T, class G, int MODE, int EXT>
__global__ __launch_bounds__(G::THREADS) void sweep_kernel(SweepArgs a)
{
    __shared__ SweepSmem<T, G> smem;
    const int nb = gridDim.x;
    sweep_block<T, G, MODE, false, EXT>(a, xcd_logical_block(blockIdx.x, nb), nb, smem);
}

// Many fields in one launch: launch block p sweeps block slot[p].y of field slot[p].x
// (no field when slot[p].x < 0: a padding block that ends at once).  The host lays the
// slots out for the round-robin dispatch of blocks over the XCDs (block p runs on XCD
// p mod 8); every field's blocks and partial sums are exactly those of a launch of that
// field alone.
template <typename T, class G, int EXT>
__global__ __launch_bounds__(G::THREADS) void batch_sweep_kernel(const SweepArgs* __restrict__ jobs,
                                                                 const int2* __restrict__ slot,
                                                                 const int* __restrict__ blocks_of_job)
{
    __shared__ SweepSmem<T, G> smem;
    const int2 e = slot[blockIdx.x];
    if (e.x < 0) return;
    const SweepArgs a = jobs[e.x];
    sweep_block<T, G, MODE_STEP, true, EXT>(a, e.y, blocks_of_job[e.x], smem);
}

}  // namespace skyr

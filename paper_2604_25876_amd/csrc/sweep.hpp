// sweep.hpp -- fused per-step sweep of the arrested Newton flow for gfx950.
//
// One launch evaluates, for every interior site of one field, the discrete
// energy density, the exact gradient of the discrete energy E_h (Sec. 2.1
// energy, Sec. 3 stencils), its tangent projection (Sec. 3, eq. Newton_flow)
// and either the kick-drift-renormalise update (Sec. 3) or a gradient output,
// plus FP64 per-block partial sums of E2, E4, E0, B and the largest |F|^2.
//
// Work decomposition (2.5D march):
//   * a thread block owns an output tile of (PY-4) rows (y) x (LW-4) columns (z)
//     and a chunk of planes [xb, xe) along x, and marches through x;
//   * every thread owns RY "flux positions" (rows r_k, column zl); the flux
//     region is PY x LW and overlaps neighbouring tiles by two rows/columns;
//   * x-neighbours live in registers: a ring of five phi planes per position
//     and a ring of five gradient accumulators (planes j-2..j+2);
//   * y- and z-neighbours go through LDS: one phi plane with a two-site halo on
//     all four sides, and one plane each of the y- and z-flux;
//   * the x-flux of plane j is pushed into the accumulators of planes j+-1, j+-2;
//     output plane j-2 is complete after plane j and is written at once.
// Energy, charge and force sums are accumulated in double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace skyr {

// partial-sum slots per thread block (doubles)
constexpr int NPART = 8;
enum : int { P_E2 = 0, P_E4 = 1, P_E0 = 2, P_B = 3, P_F2 = 4, P_POW = 5, P_E6 = 6 };

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
    int n0, n1, n2;
    int tiles_z, tiles_y;  // output tiles of the (y, z) plane
    int xchunk;            // planes per slab
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

template <typename T, int NW, int LW, int RY> struct Tile {
    static constexpr int RPW = 64 / LW;     // rows per wave
    static constexpr int R0 = NW * RPW;     // rows per row group
    static constexpr int PY = R0 * RY;      // flux rows per tile
    static constexpr int OY = PY - 4;       // output rows per tile
    static constexpr int OZ = LW - 4;       // output columns per tile
    static constexpr int THREADS = NW * 64;
    // phi halo of a plane: rows 0, 1, PY+2, PY+3 over all LW+4 columns, then
    // columns 0, 1, LW+2, LW+3 of rows 2 .. PY+1; one site per loading thread
    static constexpr int NH_ROWS = 4 * (LW + 4);
    static constexpr int NH = NH_ROWS + 4 * PY;
    static_assert(THREADS >= NH, "every halo site of a plane has its own loading thread");
};

// EXT: 0 the plain variant (pion-mass potential, kick-drift update); 1 adds the extra
// potentials (m_y, m_z, m_w) and the gradient flow; 2 also the sextic term.  The levels
// are separate kernels so that each carries only the registers it needs.
enum : int { EXT_NONE = 0, EXT_POT = 1, EXT_SEXTIC = 2 };
template <typename T, int NW, int LW, int RY, int MODE, bool FROM_TABLE = false, int EXT = EXT_NONE> struct Sweeper {
    using TL = Tile<T, NW, LW, RY>;
    static constexpr int PY = TL::PY;
    static constexpr int R0 = TL::R0;
    using C = Coef<T>;
    // Waves made only of y-halo flux rows take a short path (y-flux only).  Enabled in
    // double precision; in single precision the extra code path costs the register that
    // keeps the 1024-thread shape at four waves per SIMD.
    static constexpr bool kHaloFast = sizeof(T) == 8;
    // Double precision runs two waves per SIMD: a wave that reaches one of the plane's LDS
    // read phases (the phi stencil after the barrier, the flux divergence) is raised above
    // waves that are computing, so that its reads are issued early (4.6% at 256^3; in single
    // precision, with four waves per SIMD, the same hint costs 4%).
    static constexpr bool kPrio = sizeof(T) == 8;

    struct Smem {
        T phi[2][4][PY + 4][LW + 4];  // phi of two planes, rows y0-4 .. y0+PY-1, columns z0-4 .. z0+LW-1
        // y- and z-flux of two planes, flux row r at [r + 2]: two unwritten rows above and below
        // let the divergence read rows r-2 .. r+2 and (row-major, flat) columns c-2 .. c+2
        // without clamping; the values read there only reach positions whose result is
        // discarded.  The row stride stays LW, so the two rows of a wave fall on distinct banks.
        T qy[2][4][PY + 4][LW];
        T qz[2][4][PY + 4][LW];
        double red[NW][NPART];
    };

    Smem& sm;
    // per-component base pointers (uniform); element offsets within a component fit 32 bits
    fptr<FROM_TABLE, const T> pin[4];
    fptr<FROM_TABLE, T> pout[4];
    fptr<FROM_TABLE, T> vel[4];
    fptr<FROM_TABLE, T> gout[4];
    int n0, n1, n2;
    unsigned plane_b;  // bytes per x-plane of one component
    int xb, xe;
    int zl, rg, z, hrow, hcol;
    unsigned hoff;  // byte offset of this thread's halo site within a plane
    bool halo_loader, redo, renorm64, projected, baryon, has_grad;
    int restore;     // RESTORE_*: this sweep only rewrites the velocity
    bool halo_wave;  // every flux row of this wave is a y-halo row (only its y-flux is used)
    int yk[RY];
    unsigned offk[RY];  // byte offsets of the flux positions within a plane
    bool row_out[RY], yz_in[RY], y_near[RY], z_near;
    T c1h, c2h, d1h, d2h, hd1h, hd2h, dt;  // stencil weights with 1/h, 1/h^2 (and 1/2) folded in
    T m2, my2, mz2, mw2;                   // squared potential masses
    T c6;                                  // sextic coefficient
    bool more_pot;                         // any of m_y, m_z, m_w nonzero
    bool sextic;                           // c6 nonzero
    bool grad_flow;                        // gradient flow: phi += dt F, no velocity

    // registers carried along the march
    T ring[5][4][RY];  // phi at planes j-2 .. j+2 (slot = plane mod 5 relative to the start)
    T acc[5][4][RY];   // gradient accumulators of planes j-2 .. j+2
    T nxt[4][RY];      // prefetched phi(j+3)
    T hnxt[4];         // prefetched halo rows of phi(j+1)

    // FP64 partial sums of this thread: E2, E4, E0 and B densities (gradient mode); the
    // flow step keeps the total energy density in pe2 and leaves the others at zero
    double pe2 = 0.0, pe4 = 0.0, pe0 = 0.0, pb_sum = 0.0, pe6 = 0.0;
    double pp = 0.0;  // power F . v of the incoming velocity (flow step; used by the power arrest rule)
    T pf2 = T(0);

    __device__ __forceinline__ Sweeper(Smem& s) : sm(s) {}

    // potential density V(phi0) and dV/dphi0: m^2 (1 - phi0) + m_y^2 (1 - phi0^2)/2
    // + m_z^2 (1 - phi0)^2/2 + m_w^2 (1 - phi0)^4/4 (the program's four potentials,
    // Sec. 7.7, halved to this energy's normalisation)
    __device__ __forceinline__ T potential(T p0) const
    {
        const T u = T(1) - p0;
        T v = m2 * u;
        if constexpr (EXT) {
            if (more_pot) v += T(0.5) * my2 * (T(1) - p0 * p0) + T(0.5) * mz2 * u * u + T(0.25) * mw2 * (u * u) * (u * u);
        }
        return v;
    }
    __device__ __forceinline__ T potential_slope(T p0) const
    {
        const T u = T(1) - p0;
        T d = -m2;
        if constexpr (EXT) {
            if (more_pot) d -= my2 * p0 + mz2 * u + mw2 * u * u * u;
        }
        return d;
    }

    __device__ __forceinline__ void load_plane(int x, T (&dst)[4][RY]) const
    {
        const unsigned base = (unsigned)clampi(x, 0, n0 - 1) * plane_b;
#pragma unroll
        for (int A = 0; A < 4; ++A)
#pragma unroll
            for (int k = 0; k < RY; ++k) dst[A][k] = ldb(pin[A], base + offk[k]);
    }

    __device__ __forceinline__ void load_halo(int x, T (&dst)[4]) const
    {
        if (halo_loader) {
            const unsigned base = (unsigned)clampi(x, 0, n0 - 1) * plane_b;
#pragma unroll
            for (int A = 0; A < 4; ++A) dst[A] = ldb(pin[A], base + hoff);
        }
    }

    // one plane of the march, between two block barriers: flux at plane j, y/z-divergence
    // of plane j-1, output of plane j-2, and staging of phi(j+1).  LDS buffers alternate
    // by plane parity: phi(j) and the flux of plane j live in buffer pb, phi(j+1) and the
    // flux of plane j-1 in buffer pb ^ 1, so one barrier per plane suffices.  Ring and
    // accumulator slots 0..4 hold planes j-2 .. j+2 and are shifted at the end of the step.
    __device__ __forceinline__ void step(int j, int pb)
    {
        constexpr int S_M2 = 0, S_M1 = 1, S_0 = 2, S_P1 = 3, S_P2 = 4;
        const int qb = pb ^ 1;

        if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
        // commit the prefetched plane j+2 and the halo of plane j+1; prefetch j+3 and the halo of j+2
        T hcur[4];
#pragma unroll
        for (int A = 0; A < 4; ++A) {
#pragma unroll
            for (int k = 0; k < RY; ++k) ring[S_P2][A][k] = nxt[A][k];
            hcur[A] = hnxt[A];
        }
        load_plane(j + 3, nxt);
        load_halo(j + 2, hnxt);
        // velocity of the output plane j-2, used at the end of this step
        T vcur[4][RY];
        if constexpr (MODE == MODE_STEP) {
            const unsigned vb = (unsigned)clampi(j - 2, 0, n0 - 1) * plane_b;
#pragma unroll
            for (int A = 0; A < 4; ++A)
#pragma unroll
                for (int k = 0; k < RY; ++k) vcur[A][k] = redo ? T(0) : ldb((fptr<FROM_TABLE, const T>)vel[A], vb + offk[k]);
        }

        const bool j_in = (j >= 2) && (j <= n0 - 3);
        const bool j_out = (j >= xb) && (j < xe);
        const bool j_near = (j <= 3) || (j >= n0 - 4);
        const bool full = !(kHaloFast && halo_wave);  // uniform over the wave

#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int r = rg + k * R0 + 2;  // LDS row and column of this position in sm.phi
            const int cz = zl + 2;
            T c[4], ax[4], ay[4], az[4];
            T cl = T(0);  // phi . Lap phi
#pragma unroll
            for (int A = 0; A < 4; ++A) {
                c[A] = ring[S_0][A][k];
                const T xm2 = ring[S_M2][A][k], xm1 = ring[S_M1][A][k];
                const T xp1 = ring[S_P1][A][k], xp2 = ring[S_P2][A][k];
                const T ym2 = sm.phi[pb][A][r - 2][cz], ym1 = sm.phi[pb][A][r - 1][cz];
                const T yp1 = sm.phi[pb][A][r + 1][cz], yp2 = sm.phi[pb][A][r + 2][cz];
                const T zm2 = sm.phi[pb][A][r][cz - 2], zm1 = sm.phi[pb][A][r][cz - 1];
                const T zp1 = sm.phi[pb][A][r][cz + 1], zp2 = sm.phi[pb][A][r][cz + 2];
                ax[A] = c1h * (xp1 - xm1) + c2h * (xp2 - xm2);
                ay[A] = c1h * (yp1 - ym1) + c2h * (yp2 - ym2);
                az[A] = c1h * (zp1 - zm1) + c2h * (zp2 - zm2);
                if (full && j_out) {
                    // the five-point weights sum to zero, so the Laplacian is a weighted sum of
                    // differences from the centre: no cancellation of O(1) terms in single precision
                    const T lap = d1h * (((xp1 - c[A]) + (xm1 - c[A])) + ((yp1 - c[A]) + (ym1 - c[A])) +
                                         ((zp1 - c[A]) + (zm1 - c[A]))) +
                                  d2h * (((xp2 - c[A]) + (xm2 - c[A])) + ((yp2 - c[A]) + (ym2 - c[A])) +
                                         ((zp2 - c[A]) + (zm2 - c[A])));
                    cl += c[A] * lap;
                    // E2 part of the gradient: -1/2 (Lap phi + Lap(1_I phi)) = -Lap phi + 1/2 (the
                    // terms of Lap phi whose neighbour lies outside I); only sites within two of a
                    // face of I have such terms, one direction at a time
                    T o1 = T(0), o2 = T(0);  // sums of the outside first / second neighbours
                    if (j_near) {            // uniform over the block
                        if (j + 1 > n0 - 3) o1 += xp1;
                        if (j - 1 < 2) o1 += xm1;
                        if (j + 2 > n0 - 3) o2 += xp2;
                        if (j - 2 < 2) o2 += xm2;
                    }
                    if (y_near[k]) {
                        const int y = yk[k];
                        o1 += ((y + 1 > n1 - 3) ? yp1 : T(0)) + ((y - 1 < 2) ? ym1 : T(0));
                        o2 += ((y + 2 > n1 - 3) ? yp2 : T(0)) + ((y - 2 < 2) ? ym2 : T(0));
                    }
                    if (z_near) {
                        o1 += ((z + 1 > n2 - 3) ? zp1 : T(0)) + ((z - 1 < 2) ? zm1 : T(0));
                        o2 += ((z + 2 > n2 - 3) ? zp2 : T(0)) + ((z - 2 < 2) ? zm2 : T(0));
                    }
                    acc[S_0][A][k] += (hd1h * o1 + hd2h * o2) - lap;
                }
            }

            if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
            const T gxx = dot4(ax, ax), gyy = dot4(ay, ay), gzz = dot4(az, az);
            const T gxy = dot4(ax, ay), gxz = dot4(ax, az), gyz = dot4(ay, az);
            const bool valid = yz_in[k] && j_in;
            // the flux vanishes outside I: zero the Gram entries it is built from
            const T fxx = valid ? gxx : T(0), fyy = valid ? gyy : T(0), fzz = valid ? gzz : T(0);
            const T fxy = valid ? gxy : T(0), fxz = valid ? gxz : T(0), fyz = valid ? gyz : T(0);
            T e6 = T(0);
            if constexpr (EXT < EXT_SEXTIC) {
#pragma unroll
                for (int A = 0; A < 4; ++A) sm.qy[pb][A][r][zl] = (fxx + fzz) * ay[A] - fxy * ax[A] - fyz * az[A];
                if (full) {
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        const T qx = (fyy + fzz) * ax[A] - fxy * ay[A] - fxz * az[A];
                        sm.qz[pb][A][r][zl] = (fxx + fyy) * az[A] - fxz * ax[A] - fyz * ay[A];
                        // push the x-flux: g(j-1) -= D q, g(j+1) += D q (weights c1/h), g(j-2), g(j+2) (c2/h)
                        acc[S_M1][A][k] -= c1h * qx;
                        acc[S_P1][A][k] += c1h * qx;
                        acc[S_M2][A][k] -= c2h * qx;
                        acc[S_P2][A][k] += c2h * qx;
                    }
                }
            } else {
                T qx[4], qy[4], qz[4];
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    qx[A] = (fyy + fzz) * ax[A] - fxy * ay[A] - fxz * az[A];
                    qy[A] = (fxx + fzz) * ay[A] - fxy * ax[A] - fyz * az[A];
                    qz[A] = (fxx + fyy) * az[A] - fxz * ax[A] - fyz * ay[A];
                }
                if (sextic) {
                    // e6 = c6 det^2 / 2, det = det[phi, a_x, a_y, a_z]: flux c6 det dDet/da_i
                    // (zero outside I) and the local term c6 det dDet/dphi
                    T C0[4], C1[4], C2[4], C3[4];
                    const T det = det4_cofactors(c, ax, ay, az, C0, C1, C2, C3);
                    const T dv = valid ? c6 * det : T(0);
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        qx[A] += dv * C1[A];
                        qy[A] += dv * C2[A];
                        qz[A] += dv * C3[A];
                        acc[S_0][A][k] += dv * C0[A];
                    }
                    e6 = T(0.5) * c6 * det * det;
                }
#pragma unroll
                for (int A = 0; A < 4; ++A) sm.qy[pb][A][r][zl] = qy[A];
                if (full) {
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        sm.qz[pb][A][r][zl] = qz[A];
                        acc[S_M1][A][k] -= c1h * qx[A];
                        acc[S_P1][A][k] += c1h * qx[A];
                        acc[S_M2][A][k] -= c2h * qx[A];
                        acc[S_P2][A][k] += c2h * qx[A];
                    }
                }
            }
            if (full) {
                if (row_out[k] && j_out) {
                    const T e2 = T(-0.5) * cl;
                    const T e4 = T(0.5) * (gxx * gyy + gxx * gzz + gyy * gzz - gxy * gxy - gxz * gxz - gyz * gyz);
                    const T e0 = potential(c[0]);
                    if constexpr (MODE == MODE_STEP) {
                        if constexpr (EXT == EXT_SEXTIC)
                            pe2 += (double)(e2 + e4 + e0 + e6);  // the flow needs the total energy only
                        else
                            pe2 += (double)(e2 + e4 + e0);
                    } else {
                        pe2 += (double)e2;
                        pe4 += (double)e4;
                        pe0 += (double)e0;
                        if constexpr (EXT == EXT_SEXTIC) pe6 += (double)e6;
                        if (baryon) pb_sum += (double)det4(c, ax, ay, az);
                    }
                }
            }
        }

        // y- and z-divergence of the flux of plane j-1 (written before the last barrier)
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
        if (full && j - 1 >= xb && j - 1 < xe) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                const int o = (rg + k * R0 + 2) * LW + zl;
#pragma unroll
                for (int A = 0; A < 4; ++A) {
                    const T* qy = &sm.qy[qb][A][0][0] + o;
                    const T* qz = &sm.qz[qb][A][0][0] + o;
                    const T dy = c1h * (qy[LW] - qy[-LW]) + c2h * (qy[2 * LW] - qy[-2 * LW]);
                    const T dz = c1h * (qz[1] - qz[-1]) + c2h * (qz[2] - qz[-2]);
                    acc[S_M1][A][k] -= dy + dz;
                }
            }
        }

        if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
        // output plane j-2 is complete
        if (full && j - 2 >= xb && j - 2 < xe) {
            const unsigned base = (unsigned)(j - 2) * plane_b;
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                if (row_out[k]) {
                    T g[4], p[4], f[4];
#pragma unroll
                    for (int A = 0; A < 4; ++A) {
                        g[A] = acc[S_M2][A][k];
                        p[A] = ring[S_M2][A][k];
                    }
                    g[0] += potential_slope(p[0]);
                    const T gp = dot4(g, p);
#pragma unroll
                    for (int A = 0; A < 4; ++A) f[A] = gp * p[A] - g[A];  // F = -(g - (g.phi) phi)
                    pf2 = fmax_nonneg(pf2, dot4(f, f));
                    if constexpr (MODE == MODE_STEP) {
                        // power of the incoming velocity (zero on a redo sweep, where v = 0)
                        pp += (double)f[0] * vcur[0][k] + (double)f[1] * vcur[1][k] + (double)f[2] * vcur[2][k] +
                              (double)f[3] * vcur[3][k];
                        if (restore) {
#pragma unroll
                            for (int A = 0; A < 4; ++A)
                                stb(vel[A], base + offk[k], restore == RESTORE_ZERO ? T(0) : vcur[A][k] - dt * f[A]);
                            continue;
                        }
                        T v[4], q[4], pn[4];
#pragma unroll
                        for (int A = 0; A < 4; ++A) {
                            if constexpr (EXT) {
                                v[A] = grad_flow ? T(0) : vcur[A][k] + dt * f[A];
                                q[A] = p[A] + dt * (grad_flow ? f[A] : v[A]);
                            } else {
                                v[A] = vcur[A][k] + dt * f[A];
                                q[A] = p[A] + dt * v[A];
                            }
                        }
                        if (renorm64) {
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
                            stb(pout[A], base + offk[k], pn[A]);
                            stb(vel[A], base + offk[k], v[A]);
                        }
                    } else {
                        if (has_grad) {
#pragma unroll
                            for (int A = 0; A < 4; ++A) stb(gout[A], base + offk[k], projected ? -f[A] : g[A]);
                        }
                    }
                }
            }
        }

        // stage phi(j+1) and its halo for the next plane
#pragma unroll
        for (int A = 0; A < 4; ++A) {
#pragma unroll
            for (int k = 0; k < RY; ++k) sm.phi[qb][A][rg + k * R0 + 2][zl + 2] = ring[S_P1][A][k];
            if (halo_loader) sm.phi[qb][A][hrow][hcol] = hcur[A];
        }
        __syncthreads();

        // advance the rings by one plane; the freed accumulator starts plane j+3
#pragma unroll
        for (int A = 0; A < 4; ++A)
#pragma unroll
            for (int k = 0; k < RY; ++k) {
#pragma unroll
                for (int sl = 0; sl < 4; ++sl) {
                    ring[sl][A][k] = ring[sl + 1][A][k];
                    acc[sl][A][k] = acc[sl + 1][A][k];
                }
                acc[4][A][k] = T(0);
            }
    }
};

// One block's share of one field: logical block b of nb blocks covering the
// field's work items.  Used by the single-field and the batched kernels
// (FROM_TABLE: the arguments were read from the batch's job table).
template <typename T, int NW, int LW, int RY, int MODE, bool FROM_TABLE = false, int EXT = EXT_NONE>
__device__ __forceinline__ void sweep_block(const SweepArgs& a, int b, int nb,
                                            typename Sweeper<T, NW, LW, RY, MODE, FROM_TABLE, EXT>::Smem& smem)
{
    using SW = Sweeper<T, NW, LW, RY, MODE, FROM_TABLE, EXT>;
    using TL = typename SW::TL;
    constexpr int PY = TL::PY;
    constexpr int R0 = TL::R0;

    const Ctl* ctl = a.ctl;
    int cur = 0;
    SW sw(smem);
    sw.redo = false;
    sw.renorm64 = false;
    sw.restore = RESTORE_NONE;
    if constexpr (MODE == MODE_STEP) {
        sw.restore = ctl->restore;
        if (ctl->done && !sw.restore) return;  // uniform: the flow has stopped
        cur = ctl->cur;
        sw.redo = ctl->redo != 0;
        const int kr = ctl->renorm64_every;
        sw.renorm64 = (kr > 0) && (((ctl->steps + 1) % kr) == 0);
    }
    sw.n0 = a.n0;
    sw.n1 = a.n1;
    sw.n2 = a.n2;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    sw.plane_b = (unsigned)(n1 * n2) * (unsigned)sizeof(T);
    const long long N3 = (long long)n0 * n1 * n2;
    {
        const T* pin = (const T*)(MODE == MODE_STEP && cur ? (const void*)a.phi1 : a.phi0);
        T* pout = (T*)(MODE == MODE_STEP ? (cur ? (void*)a.phi0 : a.phi1) : nullptr);
        T* pvel = (T*)a.vel;
        T* pgrad = (T*)a.grad;
        if constexpr (FROM_TABLE) {
            // read from the job table: the same for the whole block, kept in SGPRs
            pin = uniform_ptr(pin);
            pout = uniform_ptr(pout);
            pvel = uniform_ptr(pvel);
        }
#pragma unroll
        for (int A = 0; A < 4; ++A) {
            sw.pin[A] = (fptr<FROM_TABLE, const T>)(pin + A * N3);
            sw.pout[A] = (fptr<FROM_TABLE, T>)(pout ? pout + A * N3 : nullptr);
            sw.vel[A] = (fptr<FROM_TABLE, T>)(pvel ? pvel + A * N3 : nullptr);
            sw.gout[A] = (fptr<FROM_TABLE, T>)(pgrad ? pgrad + A * N3 : nullptr);
        }
    }
    sw.has_grad = a.grad != nullptr;
    sw.projected = a.projected != 0;
    sw.baryon = a.baryon != 0;

    sw.c1h = T(Coef<double>::c1 / a.h);
    sw.c2h = T(Coef<double>::c2 / a.h);
    sw.d1h = T(Coef<double>::d1 / (a.h * a.h));
    sw.d2h = T(Coef<double>::d2 / (a.h * a.h));
    sw.hd1h = T(0.5 * Coef<double>::d1 / (a.h * a.h));
    sw.hd2h = T(0.5 * Coef<double>::d2 / (a.h * a.h));
    sw.dt = T(a.dt);
    sw.m2 = T(a.m * a.m);
    sw.my2 = T(a.m_y * a.m_y);
    sw.mz2 = T(a.m_z * a.m_z);
    sw.mw2 = T(a.m_w * a.m_w);
    sw.more_pot = a.m_y != 0.0 || a.m_z != 0.0 || a.m_w != 0.0;
    sw.c6 = T(a.c6);
    sw.sextic = a.c6 != 0.0;
    sw.grad_flow = MODE == MODE_STEP && a.gradient_flow != 0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    sw.zl = lane % LW;
    sw.rg = wave * TL::RPW + lane / LW;
    sw.halo_loader = tid < TL::NH;
    if (tid < TL::NH_ROWS) {
        const int q = tid / (LW + 4);
        sw.hrow = q < 2 ? q : PY + q;
        sw.hcol = tid % (LW + 4);
    } else {
        const int u = min(tid, TL::NH - 1) - TL::NH_ROWS;  // 0 .. 4 PY - 1
        const int q = u & 3;
        sw.hrow = 2 + (u >> 2);
        sw.hcol = q < 2 ? q : LW + q;
    }
    {
        // rows of this wave: w*RPW + (0..RPW-1) + k*R0; all of them in {0, 1, PY-2, PY-1}?
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        bool all_halo = true;
        for (int k = 0; k < RY; ++k)
            for (int q = 0; q < TL::RPW; ++q) {
                const int r = wv * TL::RPW + q + k * R0;
                all_halo = all_halo && (r < 2 || r >= PY - 2);
            }
        sw.halo_wave = all_halo;
    }

    // Work items: x is cut into slabs of `xchunk` planes; an item is one (y, z) tile of
    // one slab, items ordered slab-major with the tiles of a slab consecutive.  Items are
    // divided evenly over the nb logical blocks of this field.
    const int nx = n0 - 4;
    const int ncols = a.tiles_z * a.tiles_y;
    const int nslabs = (nx + a.xchunk - 1) / a.xchunk;
    const long long W = (long long)ncols * nslabs;
    const long long w1 = W * (b + 1) / nb;
    for (long long w = W * b / nb; w < w1; ++w) {
        const int slab = (int)(w / ncols);
        const int tile = (int)(w % ncols);
        const int x0 = slab * a.xchunk;
        const int x1 = min(nx, x0 + a.xchunk);
        const int tz = tile % a.tiles_z;
        const int ty = tile / a.tiles_z;
        const int z0 = 2 + tz * TL::OZ;
        const int y0 = 2 + ty * TL::OY;
        sw.xb = 2 + x0;
        sw.xe = 2 + x1;
        sw.z = z0 - 2 + sw.zl;
        const int zc = clampi(sw.z, 0, n2 - 1);
        const bool lane_out = (sw.zl >= 2) && (sw.zl < LW - 2) && (sw.z <= n2 - 3);
        const bool z_in = (sw.z >= 2) && (sw.z <= n2 - 3);
        sw.z_near = (sw.z <= 3) || (sw.z >= n2 - 4);
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int r = sw.rg + k * R0;
            const int y = y0 - 2 + r;
            sw.yk[k] = y;
            sw.offk[k] = (unsigned)(clampi(y, 0, n1 - 1) * n2 + zc) * (unsigned)sizeof(T);
            sw.row_out[k] = (r >= 2) && (r < PY - 2) && (y <= n1 - 3) && lane_out;
            sw.yz_in[k] = z_in && (y >= 2) && (y <= n1 - 3);
            sw.y_near[k] = (y <= 3) || (y >= n1 - 4);
        }
        // halo site of the phi plane loaded by this thread
        sw.hoff = (unsigned)(clampi(y0 - 4 + sw.hrow, 0, n1 - 1) * n2 + clampi(z0 - 4 + sw.hcol, 0, n2 - 1)) *
                  (unsigned)sizeof(T);

#pragma unroll
        for (int s = 0; s < 5; ++s)
#pragma unroll
            for (int A = 0; A < 4; ++A)
#pragma unroll
                for (int k = 0; k < RY; ++k) sw.acc[s][A][k] = T(0);

        // prologue: ring slots 0..3 hold planes jstart-2 .. jstart+1; nxt holds jstart+2
        const int jstart = sw.xb - 2;
        const int nst = (sw.xe - sw.xb) + 4;
        sw.load_plane(jstart - 2, sw.ring[0]);
        sw.load_plane(jstart - 1, sw.ring[1]);
        sw.load_plane(jstart, sw.ring[2]);
        sw.load_plane(jstart + 1, sw.ring[3]);
        sw.load_plane(jstart + 2, sw.nxt);
        // phi(jstart) and its halo go to LDS buffer 0 before the first plane; the halo of
        // jstart+1 is prefetched
        {
            T h0[4];
            sw.load_halo(jstart, h0);
            sw.load_halo(jstart + 1, sw.hnxt);
#pragma unroll
            for (int A = 0; A < 4; ++A) {
#pragma unroll
                for (int k = 0; k < RY; ++k) smem.phi[0][A][sw.rg + k * R0 + 2][sw.zl + 2] = sw.ring[2][A][k];
                if (sw.halo_loader) smem.phi[0][A][sw.hrow][sw.hcol] = h0[A];
            }
        }
        __syncthreads();
        for (int st = 0; st < nst; ++st) sw.step(jstart + st, st & 1);
    }

    // block reduction of the partial sums (fixed order)
    double vals[7] = {sw.pe2, sw.pe4, sw.pe0, sw.pb_sum, (double)sw.pf2, sw.pp, sw.pe6};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        double v = vals[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = (i == 4) ? fmax(v, o) : v + o;
        }
        vals[i] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 7; ++i) smem.red[wave][i] = vals[i];
    }
    __syncthreads();
    if (tid == 0) {
        double sum[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int wv = 0; wv < NW; ++wv) {
            for (int i = 0; i < 7; ++i) sum[i] = (i == 4) ? fmax(sum[i], smem.red[wv][i]) : sum[i] + smem.red[wv][i];
        }
        double* out = a.partials + (size_t)b * NPART;
        for (int i = 0; i < 7; ++i) out[i] = sum[i];
    }
}

// Blocks are dispatched round-robin over the eight XCDs (block i to XCD i % 8).
// The logical index gives each XCD a contiguous run: neighbouring tiles of one
// slab, which march through the same planes and share halo rows in one L2.
__device__ __forceinline__ int xcd_logical_block(int i, int n)
{
    const int xcd = i % 8, q8 = n / 8, r8 = n % 8;
    return xcd * q8 + min(xcd, r8) + i / 8;
}

template <typename T, int NW, int LW, int RY, int MODE, int EXT>
__global__ __launch_bounds__(NW * 64) void sweep_kernel(SweepArgs a)
{
    __shared__ typename Sweeper<T, NW, LW, RY, MODE, false, EXT>::Smem smem;
    const int nb = gridDim.x;
    sweep_block<T, NW, LW, RY, MODE, false, EXT>(a, xcd_logical_block(blockIdx.x, nb), nb, smem);
}

// Many fields in one launch: block i (after the XCD remap) belongs to field
// job_of_block[i] and is its block (i - first_block[job]); every field's blocks
// and partial sums are exactly those of a launch of that field alone.
template <typename T, int NW, int LW, int RY, int EXT>
__global__ __launch_bounds__(NW * 64) void batch_sweep_kernel(const SweepArgs* __restrict__ jobs,
                                                              const int* __restrict__ job_of_block,
                                                              const int* __restrict__ first_block,
                                                              const int* __restrict__ blocks_of_job)
{
    __shared__ typename Sweeper<T, NW, LW, RY, MODE_STEP, true, EXT>::Smem smem;
    const int i = xcd_logical_block(blockIdx.x, gridDim.x);
    const int j = job_of_block[i];
    const SweepArgs a = jobs[j];
    sweep_block<T, NW, LW, RY, MODE_STEP, true, EXT>(a, i - first_block[j], blocks_of_job[j], smem);
}

}  // namespace skyr

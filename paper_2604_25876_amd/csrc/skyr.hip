// skyr.hip -- host side of the C ABI (include/skyr.h) and the small kernels
// around the fused sweep: initial data, frozen-layer copy, gradient zeroing,
// fixed-order reduction of the per-block partial sums and the flow's device
// state machine (arrest / redo / convergence, Sec. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/skyr.h"
#include "sweep.hpp"
#include "moments.hpp"
#include "formp.hpp"

namespace skyr {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

static skyr_status fail(skyr_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

#define SKYR_HIP(call)                                                                                       \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return fail(SKYR_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));                   \
    } while (0)

// the same, handing the failure to `on_fail` (a cleanup that returns the status it is given)
#define SKYR_HIP_OR(call, on_fail)                                                                           \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return on_fail(fail(SKYR_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)));          \
    } while (0)

// ------------------------------------------------------------ tile choice
// A tile shape is (interior waves, halo waves, halo positions per halo lane,
// output columns); a tile has interior waves x 64 / columns rows.  A few shapes
// are compiled per precision.  x is cut into slabs of `xchunk` planes; a launch
// has one block per (slab, tile) item, so that the blocks of neighbouring tiles
// march through the same planes together and share their halo lines in L2.  The
// choice for a (lattice, precision) pair is a process-wide setting
// (skyr_set_tile / skyr_autotune).  The last entry of a shape is the relative time of one
// output site and plane of an item in a full round of the chip (measured at 256^3; a shape
// that puts two blocks on a CU takes about twice as long per item), for the default choice.
struct Shape {
    int nwi, nwh, hpt, cols;
    int per_cu;   // blocks resident on one CU (LDS and registers)
    double cost;  // relative time per output site and plane
    int threads() const { return (nwi + nwh) * 64; }
    int oy() const { return nwi * 64 / cols; }
    int oz() const { return cols; }
};

#include "shapes.hpp"
#define SKYR_SHAPE_ENTRY(a, b, c, d, e, f) Shape{a, b, c, d, e, f},
static const Shape kShapesF64[] = {SKYR_SHAPES_F64(SKYR_SHAPE_ENTRY)};
static const Shape kShapesF32[] = {SKYR_SHAPES_F32(SKYR_SHAPE_ENTRY)};
constexpr int kMinChunk = 16;  // shortest slab (planes)
constexpr int kMaxSlabs = 8;   // the default and the autotuner use 1 .. kMaxSlabs slabs
constexpr int kCUs = 256;      // compute units of the device the launches are sized for

static int shape_count(skyr_precision prec)
{
    return prec == SKYR_F64 ? (int)(sizeof kShapesF64 / sizeof kShapesF64[0])
                            : (int)(sizeof kShapesF32 / sizeof kShapesF32[0]);
}
static const Shape& shape_of(skyr_precision prec, int v) { return prec == SKYR_F64 ? kShapesF64[v] : kShapesF32[v]; }

struct Launch {
    int variant;
    Shape shape;
    int xchunk;  // planes per slab
    int tiles_z, tiles_y, zstart, slabs;
    int blocks() const { return tiles_z * tiles_y * slabs; }
    int threads() const { return shape.threads(); }
};

struct TileKey {
    int n0, n1, n2, prec;
    bool operator<(const TileKey& o) const
    {
        return std::tie(n0, n1, n2, prec) < std::tie(o.n0, o.n1, o.n2, o.prec);
    }
};
static std::mutex g_tile_mu;
static std::map<TileKey, std::pair<int, int>> g_tiles;        // (variant, planes per slab)
static std::map<TileKey, std::pair<int, int>> g_batch_tiles;  // the same, for fields in batches

// Tiles of the (y, z) plane: rows from y = 2; columns from z = 0 (so that tile rows
// start on 128-byte lines when the row length allows) unless starting at z = 2 saves a
// tile.
static void tile_grid(const skyr_lattice* lat, const Shape& sh, int& tiles_y, int& tiles_z, int& zstart)
{
    const int iy = lat->n[1] - 4, n2 = lat->n[2];
    tiles_y = (iy + sh.oy() - 1) / sh.oy();
    const int aligned = (n2 - 3) / sh.oz() + 1;
    const int inner = (n2 - 4 + sh.oz() - 1) / sh.oz();
    zstart = aligned <= inner ? 0 : 2;
    tiles_z = aligned <= inner ? aligned : inner;
}

static Launch plan_with(const skyr_lattice* lat, skyr_precision prec, int variant, int xchunk)
{
    Launch L{};
    L.variant = variant;
    L.shape = shape_of(prec, variant);
    L.xchunk = xchunk;
    tile_grid(lat, L.shape, L.tiles_y, L.tiles_z, L.zstart);
    const int nx = lat->n[0] - 4;
    L.slabs = (nx + xchunk - 1) / xchunk;
    return L;
}

// a launch of more than one round loses some of the lockstep between neighbouring tiles
// and ends with a partly idle round
constexpr double kMultiRoundCost = 1.15;
// the autotuner replaces the default tile only by one at least this much faster
constexpr double kAutotuneMargin = 0.97;

// Estimated sweep cost of shape v with the even split of x into `slabs` slabs: rounds of
// the chip times the (padded) work of one item, the march's four extra planes included.
static double plan_cost(const skyr_lattice* lat, skyr_precision prec, int v, int slabs)
{
    const Shape& sh = shape_of(prec, v);
    int ty = 0, tz = 0, zs = 0;
    tile_grid(lat, sh, ty, tz, zs);
    const int nx = lat->n[0] - 4;
    const int xc = (nx + slabs - 1) / slabs;
    const long long items = (long long)ty * tz * ((nx + xc - 1) / xc);
    const long long per_round = (long long)kCUs * sh.per_cu;
    const long long rounds = (items + per_round - 1) / per_round;
    return (double)rounds * (rounds > 1 ? kMultiRoundCost : 1.0) * sh.oy() * sh.oz() * (xc + 4) *
           sh.cost;
}

// Tile shape and slab length of a lattice the autotuner has not seen: the pair of least
// estimated cost over the compiled shapes and 1 .. kMaxSlabs slabs (of at least kMinChunk
// planes), the fewer items on ties.
static void default_tile(const skyr_lattice* lat, skyr_precision prec, int& v_out, int& xc_out)
{
    const int nx = lat->n[0] - 4;
    const int most = std::max(1, std::min(kMaxSlabs, nx / kMinChunk));
    double best = INFINITY;
    v_out = 0;
    xc_out = nx;
    for (int v = 0; v < shape_count(prec); ++v)
        for (int sl = 1; sl <= most; ++sl) {
            const double c = plan_cost(lat, prec, v, sl);
            if (c < best * (1.0 - 1e-9)) {
                best = c;
                v_out = v;
                xc_out = std::max(1, (nx + sl - 1) / sl);
            }
        }
}

static Launch plan(const skyr_lattice* lat, skyr_precision prec)
{
    int v = 0, xc = 0;
    {
        std::lock_guard<std::mutex> g(g_tile_mu);
        auto it = g_tiles.find(TileKey{lat->n[0], lat->n[1], lat->n[2], (int)prec});
        if (it != g_tiles.end()) {
            v = it->second.first;
            xc = it->second.second;
        }
    }
    if (xc == 0) default_tile(lat, prec, v, xc);
    return plan_with(lat, prec, v, xc);
}

// Tile shape and slab length of a field in a batch on a lattice that no one has set or
// tuned for batches.  The shape is the precision's first: fields of one precision then
// share one launch per sweep slot (fields of other shapes run as concurrent launches,
// which mix their blocks on the CUs so that a field's neighbouring tiles no longer march
// together; each extra launch cost the 64-field mix a few percent).  The batch's other
// fields fill the device, so the field need not: x is split evenly into the fewest slabs
// of at most kBatchSlab planes, so that the last blocks of a launch end early.
constexpr int kBatchShape = 0;
constexpr int kBatchSlab = 64;
static void batch_default_tile(const skyr_lattice* lat, skyr_precision prec, int& v_out, int& xc_out)
{
    const int nx = lat->n[0] - 4;
    const int slabs = std::max(1, (nx + kBatchSlab - 1) / kBatchSlab);
    (void)prec;
    v_out = kBatchShape;
    xc_out = std::max(std::min(kMinChunk, nx), (nx + slabs - 1) / slabs);
}

static Launch plan_batch(const skyr_lattice* lat, skyr_precision prec)
{
    int v = 0, xc = 0;
    {
        std::lock_guard<std::mutex> g(g_tile_mu);
        auto it = g_batch_tiles.find(TileKey{lat->n[0], lat->n[1], lat->n[2], (int)prec});
        if (it != g_batch_tiles.end()) {
            v = it->second.first;
            xc = it->second.second;
        }
    }
    if (xc == 0) batch_default_tile(lat, prec, v, xc);
    return plan_with(lat, prec, v, xc);
}

// The printed-form sweep: its fixed tile shape, one block per (slab, tile) item, and the
// slab length whose items cost least in rounds of the chip (as for the exact sweep).
static Launch plan_printed(const skyr_lattice* lat, skyr_precision prec)
{
    const int oy = prec == SKYR_F64 ? FpGeoF64::OY : FpGeoF32::OY;
    const int oz = prec == SKYR_F64 ? FpGeoF64::OZ : FpGeoF32::OZ;
    Launch L{};
    L.variant = 0;
    L.shape = Shape{oy * oz / 64, 0, 0, oz, 1, 1.0};
    tile_grid(lat, L.shape, L.tiles_y, L.tiles_z, L.zstart);
    const int nx = lat->n[0] - 4, tiles = L.tiles_y * L.tiles_z;
    const int most = std::max(1, std::min(kMaxSlabs, nx / kMinChunk));
    double best = INFINITY;
    for (int sl = 1; sl <= most; ++sl) {
        const int xc = std::max(1, (nx + sl - 1) / sl);
        const long long items = (long long)tiles * ((nx + xc - 1) / xc);
        const long long rounds = (items + kCUs - 1) / kCUs;
        const double c = (double)rounds * (rounds > 1 ? kMultiRoundCost : 1.0) * (xc + 4);
        if (c < best * (1.0 - 1e-9)) {
            best = c;
            L.xchunk = xc;
        }
    }
    L.slabs = (nx + L.xchunk - 1) / L.xchunk;
    return L;
}

constexpr size_t CTL_BYTES = 256;
// observables (8 doubles), then the moments' centre (4 doubles at +64) and result (at +128)
constexpr size_t OBS_BYTES = 512;
constexpr size_t MOM_CENTRE_OFFSET = 64;
constexpr size_t MOM_OUT_OFFSET = 128;
static_assert(MOM_OUT_OFFSET + MOM_OUT_DOUBLES * sizeof(double) <= OBS_BYTES, "moment result must fit");
static_assert(sizeof(skyr_moment_obs) == MOM_OUT_DOUBLES * sizeof(double), "moment record layout");

// enough partial-sum slots for every shape and slab length >= the shortest
// supported, and for the moment passes
static size_t workspace_bytes(const skyr_lattice* lat, skyr_precision prec)
{
    int most = 0;
    for (int v = 0; v < shape_count(prec); ++v) most = std::max(most, plan_with(lat, prec, v, kMinChunk).blocks());
    most = std::max(most, plan_printed(lat, prec).blocks());
    const size_t sweep_part = (size_t)most * NPART * sizeof(double);
    const size_t mom_part = (size_t)MOM_MAX_BLOCKS * MOM_NACC * sizeof(double);
    return CTL_BYTES + OBS_BYTES + std::max(sweep_part, mom_part);
}

static skyr_status check_lattice(const skyr_lattice* lat, skyr_precision prec)
{
    if (!lat) return fail(SKYR_E_INVAL, "lattice is null");
    if (prec != SKYR_F64 && prec != SKYR_F32_BULK) return fail(SKYR_E_INVAL, "unknown precision");
    for (int i = 0; i < 3; ++i)
        if (lat->n[i] < 5) return fail(SKYR_E_INVAL, "every lattice dimension must be at least 5");
    if (!(lat->h > 0.0) || !std::isfinite(lat->h)) return fail(SKYR_E_INVAL, "lattice spacing must be positive");
    const long long n3 = (long long)lat->n[0] * lat->n[1] * lat->n[2];
    if (n3 >= (1LL << 31) / 4) return fail(SKYR_E_INVAL, "lattice too large for 32-bit component offsets");
    return SKYR_OK;
}

static size_t elem_bytes(skyr_precision prec) { return prec == SKYR_F64 ? sizeof(double) : sizeof(float); }

static long long sites(const skyr_lattice* lat) { return (long long)lat->n[0] * lat->n[1] * lat->n[2]; }

// ------------------------------------------------------------ initial data
struct DevConstituent {
    int degree;
    double p[9][2], q[9][2];
    double X[3], quat[4];
    double prof_a, prof_lambda;
    double orient[4];  // spatial orientation B (identity when rotated == 0)
    int rotated;
};

// n_R of R = p/q at direction d (Sec. 4.1) in homogeneous form, z = u / w:
// u = x1 + i x2, w = r + x3 on the upper half (x3 >= 0); u = r - x3,
// w = x1 - i x2 on the lower half, which reaches the south pole z = infinity
// (w = 0) where the first pair is 0/0.  With P(u, w) = sum_k p_k u^k w^(B-k),
// n_R = (2 Re(P conj Q), 2 Im(P conj Q), |Q|^2 - |P|^2) / (|P|^2 + |Q|^2).
// At d = 0 the direction is undefined and the north pole's is used.
__device__ static void rm_direction(const DevConstituent& c, const double d_in[3], double nh[3])
{
    double d0 = d_in[0], d1 = d_in[1], d2 = d_in[2];
    double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (r == 0.0) {
        d2 = 1.0;
        r = 1.0;
    }
    const bool upper = d2 >= 0.0;
    const double ur = upper ? d0 : r - d2, ui = upper ? d1 : 0.0;
    const double wr = upper ? r + d2 : d0, wi = upper ? 0.0 : -d1;
    double Pr = 0, Pi = 0, Qr = 0, Qi = 0;
    double wkr = 1.0, wki = 0.0;  // w^(B-k)
    // homogeneous Horner scheme: P <- P u + p_k w^(B-k), k = B .. 0
    for (int k = c.degree; k >= 0; --k) {
        const double nPr = Pr * ur - Pi * ui, nPi = Pr * ui + Pi * ur;
        const double nQr = Qr * ur - Qi * ui, nQi = Qr * ui + Qi * ur;
        Pr = nPr + (c.p[k][0] * wkr - c.p[k][1] * wki);
        Pi = nPi + (c.p[k][0] * wki + c.p[k][1] * wkr);
        Qr = nQr + (c.q[k][0] * wkr - c.q[k][1] * wki);
        Qi = nQi + (c.q[k][0] * wki + c.q[k][1] * wkr);
        const double tr = wkr * wr - wki * wi, ti = wkr * wi + wki * wr;
        wkr = tr;
        wki = ti;
    }
    const double cr = Pr * Qr + Pi * Qi, ci = Pi * Qr - Pr * Qi;
    const double p2 = Pr * Pr + Pi * Pi, q2 = Qr * Qr + Qi * Qi;
    const double den = p2 + q2;
    nh[0] = 2.0 * cr / den;
    nh[1] = 2.0 * ci / den;
    nh[2] = (q2 - p2) / den;
}

template <typename T>
__global__ void init_kernel(T* __restrict__ phi, int n0, int n1, int n2, double h, const DevConstituent* __restrict__ cs,
                            int nc)
{
    const long long N3 = (long long)n0 * n1 * n2;
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N3) return;
    const int iz = (int)(s % n2);
    const int iy = (int)((s / n2) % n1);
    const int ix = (int)(s / ((long long)n1 * n2));
    double U[4] = {1.0, 0.0, 0.0, 0.0};
    const bool in = ix >= 2 && ix <= n0 - 3 && iy >= 2 && iy <= n1 - 3 && iz >= 2 && iz <= n2 - 3;
    if (in) {
        const double x[3] = {(ix - 0.5 * (n0 - 1)) * h, (iy - 0.5 * (n1 - 1)) * h, (iz - 0.5 * (n2 - 1)) * h};
        for (int k = 0; k < nc; ++k) {
            const DevConstituent& c = cs[k];
            double d[3] = {x[0] - c.X[0], x[1] - c.X[1], x[2] - c.X[2]};
            if (c.rotated) {
                // d <- D(B)^T d = D(B^dagger) d: with b -> -b in
                // D(B) v = (b0^2 - |b|^2) v + 2 (b.v) b - 2 b0 (b x v)
                const double b0 = c.orient[0], b1 = c.orient[1], b2 = c.orient[2], b3 = c.orient[3];
                const double kb = b0 * b0 - (b1 * b1 + b2 * b2 + b3 * b3);
                const double bd = b1 * d[0] + b2 * d[1] + b3 * d[2];
                const double e0 = kb * d[0] + 2.0 * bd * b1 + 2.0 * b0 * (b2 * d[2] - b3 * d[1]);
                const double e1 = kb * d[1] + 2.0 * bd * b2 + 2.0 * b0 * (b3 * d[0] - b1 * d[2]);
                const double e2 = kb * d[2] + 2.0 * bd * b3 + 2.0 * b0 * (b1 * d[1] - b2 * d[0]);
                d[0] = e0;
                d[1] = e1;
                d[2] = e2;
            }
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double f = c.prof_a * exp(-r / c.prof_lambda);
            double nh[3];
            rm_direction(c, d, nh);
            // isorotation A (n.tau) A^dagger = (D(A) n).tau, D(A) n = (a0^2 - |a|^2) n + 2 (a.n) a - 2 a0 a x n
            const double a0 = c.quat[0], a1 = c.quat[1], a2 = c.quat[2], a3 = c.quat[3];
            const double aa = a1 * a1 + a2 * a2 + a3 * a3;
            const double an = a1 * nh[0] + a2 * nh[1] + a3 * nh[2];
            const double cx = a2 * nh[2] - a3 * nh[1], cy = a3 * nh[0] - a1 * nh[2], cz = a1 * nh[1] - a2 * nh[0];
            const double k0 = a0 * a0 - aa;
            const double rx = k0 * nh[0] + 2.0 * an * a1 - 2.0 * a0 * cx;
            const double ry = k0 * nh[1] + 2.0 * an * a2 - 2.0 * a0 * cy;
            const double rz = k0 * nh[2] + 2.0 * an * a3 - 2.0 * a0 * cz;
            const double sf = sin(f), cf = cos(f);
            const double V[4] = {cf, sf * rx, sf * ry, sf * rz};
            // U <- U V with (u0 + i u.tau)(v0 + i v.tau) = (u0 v0 - u.v) + i (u0 v + v0 u - u x v).tau
            const double w0 = U[0] * V[0] - (U[1] * V[1] + U[2] * V[2] + U[3] * V[3]);
            const double w1 = U[0] * V[1] + V[0] * U[1] - (U[2] * V[3] - U[3] * V[2]);
            const double w2 = U[0] * V[2] + V[0] * U[2] - (U[3] * V[1] - U[1] * V[3]);
            const double w3 = U[0] * V[3] + V[0] * U[3] - (U[1] * V[2] - U[2] * V[1]);
            U[0] = w0;
            U[1] = w1;
            U[2] = w2;
            U[3] = w3;
        }
    }
    for (int A = 0; A < 4; ++A) phi[A * N3 + s] = T(U[A]);
}

// ---------------------------------------------------------- small kernels
template <typename T> __global__ void fill_kernel(T* __restrict__ p, long long n, T v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// copy the frozen layers (everything outside the interior) of src to dst
template <typename T>
__global__ void copy_frozen_kernel(const T* __restrict__ src, T* __restrict__ dst, int n0, int n1, int n2)
{
    const long long N3 = (long long)n0 * n1 * n2;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < N3; s += (long long)gridDim.x * blockDim.x) {
        const int iz = (int)(s % n2);
        const int iy = (int)((s / n2) % n1);
        const int ix = (int)(s / ((long long)n1 * n2));
        const bool in = ix >= 2 && ix <= n0 - 3 && iy >= 2 && iy <= n1 - 3 && iz >= 2 && iz <= n2 - 3;
        if (!in)
            for (int A = 0; A < 4; ++A) dst[A * N3 + s] = src[A * N3 + s];
    }
}

// Fixed-order reduction of the per-block partials: thread t sums blocks
// t, t + 256, ... in order, then a fixed tree.
// out = {E2, E4, E0, Bsum, maxF2, power, E6}.
__device__ static void reduce_partials(const double* __restrict__ part, int nblocks, double out[NRED])
{
    __shared__ double red[256][NRED];
    const int t = threadIdx.x;
    double s[NRED] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = t; b < nblocks; b += 256) {
        const double* p = part + (size_t)b * NPART;
        for (int i = 0; i < NRED; ++i) s[i] = (i == P_F2) ? fmax(s[i], p[i]) : s[i] + p[i];
    }
    for (int i = 0; i < NRED; ++i) red[t][i] = s[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            for (int i = 0; i < NRED; ++i)
                red[t][i] = (i == P_F2) ? fmax(red[t][i], red[t + w][i]) : red[t][i] + red[t + w][i];
        }
        __syncthreads();
    }
    for (int i = 0; i < NRED; ++i) out[i] = red[0][i];
}

// obs = {E, E2, E4, E0, B, virial, max_force, E6}; the virial is the
// derivative of E under x -> lambda x at lambda = 1, E2 - E4 + 3 E0 - 3 E6.
__global__ void observe_kernel(const double* __restrict__ part, int nblocks, double h, double* __restrict__ obs)
{
    double s[NRED];
    reduce_partials(part, nblocks, s);
    if (threadIdx.x == 0) {
        const double h3 = h * h * h;
        const double E2 = h3 * s[P_E2], E4 = h3 * s[P_E4], E0 = h3 * s[P_E0], E6 = h3 * s[P_E6];
        obs[0] = E2 + E4 + E0 + E6;
        obs[1] = E2;
        obs[2] = E4;
        obs[3] = E0;
        obs[4] = -h3 * s[P_B] / (2.0 * M_PI * M_PI);
        obs[5] = E2 - E4 + 3.0 * E0 - 3.0 * E6;
        obs[6] = sqrt(s[P_F2]);
        obs[7] = E6;
    }
}


// ------------------------------------------------------------- launches
// the kernel variant with the extra potentials and the gradient flow is used only
// by models and flows that need it
// kernel variant a field needs: the sextic term, else the extra potentials or the
// gradient flow, else the plain sweep
static int ext_level(const SweepArgs& a)
{
    if (a.c6 != 0.0) return EXT_SEXTIC;
    return (a.m_y != 0.0 || a.m_z != 0.0 || a.m_w != 0.0 || a.gradient_flow != 0) ? EXT_POT : EXT_NONE;
}

template <typename T, class G, int MODE>
static void launch_level(int ext, dim3 grid, dim3 block, const SweepArgs& args, hipStream_t s)
{
    if (ext == EXT_SEXTIC)
        hipLaunchKernelGGL((sweep_kernel<T, G, MODE, EXT_SEXTIC>), grid, block, 0, s, args);
    else if (ext == EXT_POT)
        hipLaunchKernelGGL((sweep_kernel<T, G, MODE, EXT_POT>), grid, block, 0, s, args);
    else
        hipLaunchKernelGGL((sweep_kernel<T, G, MODE, EXT_NONE>), grid, block, 0, s, args);
}

template <typename T, class G>
static hipError_t launch_shape(int mode, const Launch& L, const SweepArgs& args, hipStream_t s)
{
    const dim3 grid(L.blocks()), block(G::THREADS);
    if (mode == MODE_STEP)
        launch_level<T, G, MODE_STEP>(ext_level(args), grid, block, args, s);
    else
        launch_level<T, G, MODE_GRAD>(ext_level(args), grid, block, args, s);
    return hipGetLastError();
}

static hipError_t sweep(skyr_precision prec, int mode, const Launch& L, const SweepArgs& args, hipStream_t s)
{
    int v = 0;
    if (prec == SKYR_F64) {
#define SKYR_CASE64(a, b, c, d, e, f)                                                                          \
    if (L.variant == v) return launch_shape<double, Geo<a, b, c, d>>(mode, L, args, s);                      \
    ++v;
        SKYR_SHAPES_F64(SKYR_CASE64)
#undef SKYR_CASE64
    } else {
#define SKYR_CASE32(a, b, c, d, e, f)                                                                          \
    if (L.variant == v) return launch_shape<float, Geo<a, b, c, d>>(mode, L, args, s);                       \
    ++v;
        SKYR_SHAPES_F32(SKYR_CASE32)
#undef SKYR_CASE32
    }
    return hipErrorInvalidValue;
}

// The step-sweep kernel of a tile shape at a kernel variant, and its block size (for
// the nodes of a graph).
template <typename T, class G> static const void* step_fn(int ext, int& threads)
{
    threads = G::THREADS;
    if (ext == EXT_SEXTIC) return (const void*)sweep_kernel<T, G, MODE_STEP, EXT_SEXTIC>;
    if (ext == EXT_POT) return (const void*)sweep_kernel<T, G, MODE_STEP, EXT_POT>;
    return (const void*)sweep_kernel<T, G, MODE_STEP, EXT_NONE>;
}

static const void* step_kernel(skyr_precision prec, int variant, int ext, int& threads)
{
    int v = 0;
    if (prec == SKYR_F64) {
#define SKYR_S64(a, b, c, d, e, f)                                              \
    if (variant == v) return step_fn<double, Geo<a, b, c, d>>(ext, threads); \
    ++v;
        SKYR_SHAPES_F64(SKYR_S64)
#undef SKYR_S64
    } else {
#define SKYR_S32(a, b, c, d, e, f)                                             \
    if (variant == v) return step_fn<float, Geo<a, b, c, d>>(ext, threads); \
    ++v;
        SKYR_SHAPES_F32(SKYR_S32)
#undef SKYR_S32
    }
    threads = 0;
    return nullptr;
}

template <typename T> static const void* printed_fn(int mode, bool ext)
{
    if (mode == MODE_STEP)
        return ext ? (const void*)formp_kernel<T, MODE_STEP, true> : (const void*)formp_kernel<T, MODE_STEP, false>;
    return ext ? (const void*)formp_kernel<T, MODE_GRAD, true> : (const void*)formp_kernel<T, MODE_GRAD, false>;
}

// the printed-form kernel of a precision and mode for arguments a, and its block size
static const void* printed_kernel(skyr_precision prec, int mode, const SweepArgs& a, int& threads)
{
    const bool ext = ext_level(a) != EXT_NONE;
    threads = prec == SKYR_F64 ? FpGeoF64::THREADS : FpGeoF32::THREADS;
    return prec == SKYR_F64 ? printed_fn<double>(mode, ext) : printed_fn<float>(mode, ext);
}

// The printed-form sweep: one launch, arguments made by make_args with plan_printed's launch.
static hipError_t sweep_printed(skyr_precision prec, int mode, const Launch& L, const SweepArgs& args, hipStream_t s)
{
    int threads = 0;
    const void* fn = printed_kernel(prec, mode, args, threads);
    void* argv[1] = {const_cast<SweepArgs*>(&args)};
    return hipLaunchKernel(fn, dim3(L.blocks()), dim3(threads), argv, 0, s);
}

// The batched-sweep kernel of one (precision, tile shape) group at a kernel variant, and
// its block size.
template <typename T, class G> static const void* batch_fn(int ext, int& threads)
{
    threads = G::THREADS;
    if (ext == EXT_SEXTIC) return (const void*)batch_sweep_kernel<T, G, EXT_SEXTIC>;
    if (ext == EXT_POT) return (const void*)batch_sweep_kernel<T, G, EXT_POT>;
    return (const void*)batch_sweep_kernel<T, G, EXT_NONE>;
}

static const void* batch_kernel(skyr_precision prec, int variant, int ext, int& threads)
{
    int v = 0;
    if (prec == SKYR_F64) {
#define SKYR_B64(a, b, c, d, e, f)                                               \
    if (variant == v) return batch_fn<double, Geo<a, b, c, d>>(ext, threads); \
    ++v;
        SKYR_SHAPES_F64(SKYR_B64)
#undef SKYR_B64
    } else {
#define SKYR_B32(a, b, c, d, e, f)                                              \
    if (variant == v) return batch_fn<float, Geo<a, b, c, d>>(ext, threads); \
    ++v;
        SKYR_SHAPES_F32(SKYR_B32)
#undef SKYR_B32
    }
    threads = 0;
    return nullptr;
}

static SweepArgs make_args(const skyr_lattice* lat, const Launch& L, const skyr_model* model, double dt)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof a);  // padding too: flow graphs are looked up by these bytes
    a.n0 = lat->n[0];
    a.n1 = lat->n[1];
    a.n2 = lat->n[2];
    a.cstride = sites(lat);
    a.zlo = 0;
    a.zhi = lat->n[2] - 1;
    for (int d = 0; d < 3; ++d) {  // a whole lattice: I and the output region are its interior
        a.ilo[d] = a.olo[d] = 2;
        a.ihi[d] = a.ohi[d] = lat->n[d] - 3;
    }
    a.tiles_z = L.tiles_z;
    a.tiles_y = L.tiles_y;
    a.zstart = L.zstart;
    a.xchunk = L.xchunk;
    a.h = lat->h;
    a.m = model->m;
    a.m_y = model->m_y;
    a.m_z = model->m_z;
    a.m_w = model->m_w;
    a.c6 = model->c6;
    a.dt = dt;
    return a;
}

// Sweep arguments for fields in padded rows of `pitch` elements with the four components of
// a row one after the other and the lattice's z = 0 at element `lead`: the same tiles over
// the same lattice sites, each component addressed within its quarter of a row four
// pitches long; lanes beyond the lattice read its frozen end columns, as in a dense row.
static void use_padded_rows(SweepArgs& a, const skyr_lattice* lat, int lead, int pitch)
{
    a.n2 = 4 * pitch;
    a.cstride = pitch;
    a.zlo = lead;
    a.zhi = lead + lat->n[2] - 1;
    a.ilo[2] += lead;
    a.ihi[2] += lead;
    a.olo[2] += lead;
    a.ohi[2] += lead;
    a.zstart += lead;
}

// the layout checks of a padded field: lead >= 0, pitch >= lead + n2, offsets within 32 bits
static skyr_status check_padded_rows(const skyr_lattice* lat, skyr_precision prec, int lead, int pitch)
{
    if (lead < 0 || pitch < (long long)lead + lat->n[2]) return fail(SKYR_E_INVAL, "need lead >= 0 and pitch >= lead + n2");
    if (4LL * lat->n[0] * lat->n[1] * pitch * (long long)elem_bytes(prec) >= (1LL << 32))
        return fail(SKYR_E_INVAL, "padded arrays too large for 32-bit offsets");
    return SKYR_OK;
}

static hipError_t fill(void* p, long long n, skyr_precision prec, double v, hipStream_t s)
{
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    if (prec == SKYR_F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(blocks), dim3(256), 0, s, (double*)p, n, v);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(blocks), dim3(256), 0, s, (float*)p, n, (float)v);
    return hipGetLastError();
}

static bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// ------------------------------------------------------------- timing
// Per-thread event pool around sweep launches (measurement only).
struct Timing {
    bool on = false;
    double ms = 0.0;
    int64_t launches = 0;
    std::vector<hipEvent_t> ev;  // 2 per launch of the current group
    int used = 0;
    ~Timing()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
static thread_local Timing g_timing;

static hipError_t timing_mark(hipStream_t s)
{
    Timing& t = g_timing;
    if (!t.on) return hipSuccess;
    if (t.used == (int)t.ev.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        t.ev.push_back(e);
    }
    return hipEventRecord(t.ev[t.used++], s);
}

// after the stream has been synchronised: add up the recorded pairs
static hipError_t timing_collect()
{
    Timing& t = g_timing;
    for (int i = 0; i + 1 < t.used; i += 2) {
        float ms = 0.0f;
        hipError_t r = hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]);
        if (r != hipSuccess) return r;
        t.ms += ms;
        t.launches += 1;
    }
    t.used = 0;
    return hipSuccess;
}

}  // namespace skyr

using namespace skyr;

// ================================================================== C ABI
extern "C" {

const char* skyr_version(void) { return "skyr 0.1 (gfx950)"; }

const char* skyr_last_error(void) { return g_last_error.c_str(); }

size_t skyr_workspace_bytes(const skyr_lattice* lat, skyr_precision prec)
{
    if (check_lattice(lat, prec) != SKYR_OK) return 0;
    return workspace_bytes(lat, prec);
}

void skyr_anf_state_init(skyr_anf_state* st)
{
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    st->E_prev = INFINITY;
    st->E = NAN;
    st->max_force = NAN;
}

skyr_status skyr_random_constituents(uint64_t seed, int32_t B, double radius, double prof_a, double prof_lambda,
                                     skyr_constituent* out)
{
    if (!out) return fail(SKYR_E_INVAL, "output array is null");
    if (B < 1 || B > 64) return fail(SKYR_E_INVAL, "B must be in 1..64");
    if (!(radius >= 0.0) || !(prof_lambda > 0.0)) return fail(SKYR_E_INVAL, "radius must be >= 0, prof_lambda > 0");
    // SplitMix64: state advances by the golden-ratio increment, output is the finaliser of the state
    uint64_t state = seed;
    auto next = [&]() {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    auto uniform = [&]() { return (double)(next() >> 11) * 0x1.0p-53; };
    for (int k = 0; k < B; ++k) {
        skyr_constituent& c = out[k];
        std::memset(&c, 0, sizeof c);
        c.degree = 1;
        c.p[1][0] = 1.0;  // p = z
        c.q[0][0] = 1.0;  // q = 1
        for (;;) {
            const double x = radius * (2.0 * uniform() - 1.0);
            const double y = radius * (2.0 * uniform() - 1.0);
            const double z = radius * (2.0 * uniform() - 1.0);
            if (x * x + y * y + z * z <= radius * radius) {
                c.X[0] = x;
                c.X[1] = y;
                c.X[2] = z;
                break;
            }
        }
        const double u1 = uniform(), u2 = uniform(), u3 = uniform();
        const double s1 = std::sqrt(1.0 - u1), s2 = std::sqrt(u1);
        c.quat[0] = s1 * std::sin(2.0 * M_PI * u2);
        c.quat[1] = s1 * std::cos(2.0 * M_PI * u2);
        c.quat[2] = s2 * std::sin(2.0 * M_PI * u3);
        c.quat[3] = s2 * std::cos(2.0 * M_PI * u3);
        c.prof_a = prof_a;
        c.prof_lambda = prof_lambda;
    }
    return SKYR_OK;
}

// B(n, t) = cos(t/2) - i sin(t/2) n.tau has D(B) = the right-handed rotation by
// t about n (D(B) v = (b0^2 - |b|^2) v + 2 (b.v) b - 2 b0 (b x v) with
// b = -sin(t/2) n is Rodrigues' formula), and D(B1 B2) = D(B1) D(B2).
void skyr_orientation_zyz(const double angles[3], double out[4])
{
    const double cz1 = std::cos(0.5 * angles[0]), sz1 = std::sin(0.5 * angles[0]);
    const double cy = std::cos(0.5 * angles[1]), sy = std::sin(0.5 * angles[1]);
    const double cz2 = std::cos(0.5 * angles[2]), sz2 = std::sin(0.5 * angles[2]);
    // quaternion product (a0 + i a.tau)(c0 + i c.tau) = (a0 c0 - a.c) + i (a0 c + c0 a - a x c).tau
    auto mul = [](const double a[4], const double c[4], double o[4]) {
        o[0] = a[0] * c[0] - (a[1] * c[1] + a[2] * c[2] + a[3] * c[3]);
        o[1] = a[0] * c[1] + c[0] * a[1] - (a[2] * c[3] - a[3] * c[2]);
        o[2] = a[0] * c[2] + c[0] * a[2] - (a[3] * c[1] - a[1] * c[3]);
        o[3] = a[0] * c[3] + c[0] * a[3] - (a[1] * c[2] - a[2] * c[1]);
    };
    const double Bz1[4] = {cz1, 0.0, 0.0, -sz1}, By[4] = {cy, 0.0, -sy, 0.0}, Bz2[4] = {cz2, 0.0, 0.0, -sz2};
    double t[4];
    mul(Bz1, By, t);
    mul(t, Bz2, out);
    if (out[0] < 0.0)
        for (int k = 0; k < 4; ++k) out[k] = -out[k];
}

skyr_status skyr_init_field(const skyr_lattice* lat, skyr_precision prec, const skyr_init_spec* spec, void* phi,
                            void* stream)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (!spec || !phi) return fail(SKYR_E_INVAL, "spec and phi must be non-null");
    hipStream_t s = (hipStream_t)stream;
    DevConstituent host[64];
    int nc = 0;
    auto convert = [&](const skyr_constituent& c) -> bool {
        if (c.degree < 1 || c.degree > 8 || !(c.prof_lambda > 0.0)) return false;
        DevConstituent& d = host[nc++];
        std::memset(&d, 0, sizeof d);
        d.degree = c.degree;
        std::memcpy(d.p, c.p, sizeof d.p);
        std::memcpy(d.q, c.q, sizeof d.q);
        std::memcpy(d.X, c.X, sizeof d.X);
        std::memcpy(d.quat, c.quat, sizeof d.quat);
        d.prof_a = c.prof_a;
        d.prof_lambda = c.prof_lambda;
        std::memcpy(d.orient, c.orient, sizeof d.orient);
        d.rotated = c.orient[0] != 0.0 || c.orient[1] != 0.0 || c.orient[2] != 0.0 || c.orient[3] != 0.0;
        return true;
    };
    switch (spec->kind) {
    case SKYR_INIT_HEDGEHOG: {
        if (!(spec->prof_lambda > 0.0)) return fail(SKYR_E_INVAL, "prof_lambda must be positive");
        skyr_constituent c;
        std::memset(&c, 0, sizeof c);
        c.degree = 1;
        c.p[1][0] = 1.0;
        c.q[0][0] = 1.0;
        c.quat[0] = 1.0;
        c.prof_a = spec->prof_a;
        c.prof_lambda = spec->prof_lambda;
        convert(c);
        break;
    }
    case SKYR_INIT_RATIONAL_MAP:
        if (!spec->c) return fail(SKYR_E_INVAL, "rational map needs c[0]");
        if (!convert(spec->c[0])) return fail(SKYR_E_INVAL, "constituent degree must be 1..8, prof_lambda > 0");
        break;
    case SKYR_INIT_PRODUCT:
        if (!spec->c || spec->count < 1 || spec->count > 64) return fail(SKYR_E_INVAL, "product needs 1..64 constituents");
        for (int k = 0; k < spec->count; ++k)
            if (!convert(spec->c[k])) return fail(SKYR_E_INVAL, "constituent degree must be 1..8, prof_lambda > 0");
        break;
    case SKYR_INIT_RANDOM_PRODUCT: {
        skyr_constituent cs[64];
        st = skyr_random_constituents(spec->seed, spec->B, spec->ball_radius, spec->prof_a, spec->prof_lambda, cs);
        if (st != SKYR_OK) return st;
        for (int k = 0; k < spec->B; ++k) convert(cs[k]);
        break;
    }
    default:
        return fail(SKYR_E_INVAL, "unknown initial-data kind");
    }
    DevConstituent* dev = nullptr;
    SKYR_HIP(hipMalloc((void**)&dev, sizeof(DevConstituent) * nc));
    hipError_t e = hipMemcpyAsync(dev, host, sizeof(DevConstituent) * nc, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return fail(SKYR_E_DEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    }
    const long long N3 = sites(lat);
    const int blocks = (int)((N3 + 255) / 256);
    if (prec == SKYR_F64)
        hipLaunchKernelGGL(init_kernel<double>, dim3(blocks), dim3(256), 0, s, (double*)phi, lat->n[0], lat->n[1],
                           lat->n[2], lat->h, dev, nc);
    else
        hipLaunchKernelGGL(init_kernel<float>, dim3(blocks), dim3(256), 0, s, (float*)phi, lat->n[0], lat->n[1],
                           lat->n[2], lat->h, dev, nc);
    e = hipGetLastError();
    // the copy from the host stack array and the kernel must finish before the table is freed
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(SKYR_E_DEVICE, std::string("init_kernel: ") + hipGetErrorString(e));
    return SKYR_OK;
}

static skyr_status run_gradient(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model, const void* phi,
                                void* grad, int projected, int baryon, double obs_out[7], void* work, hipStream_t s)
{
    const bool printed = model->form == SKYR_FORM_PRINTED;
    const Launch L = printed ? plan_printed(lat, prec) : plan(lat, prec);
    SweepArgs a = make_args(lat, L, model, 0.0);
    a.phi0 = phi;
    a.grad = grad;
    a.projected = projected;
    a.baryon = baryon;
    char* w = (char*)work;
    a.partials = (double*)(w + CTL_BYTES + OBS_BYTES);
    double* obs = (double*)(w + CTL_BYTES);
    if (grad) SKYR_HIP(fill(grad, 4 * sites(lat), prec, 0.0, s));
    if (printed)
        SKYR_HIP(sweep_printed(prec, MODE_GRAD, L, a, s));
    else
        SKYR_HIP(sweep(prec, MODE_GRAD, L, a, s));
    if (obs_out) {
        hipLaunchKernelGGL(observe_kernel, dim3(1), dim3(256), 0, s, a.partials, L.blocks(), lat->h, obs);
        SKYR_HIP(hipGetLastError());
        SKYR_HIP(hipMemcpyAsync(obs_out, obs, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        SKYR_HIP(hipStreamSynchronize(s));
    }
    return SKYR_OK;
}

static skyr_status check_common(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model, const void* phi,
                                void* work)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (!model || !phi || !work) return fail(SKYR_E_INVAL, "model, phi and work must be non-null");
    if (!std::isfinite(model->m) || !std::isfinite(model->m_y) || !std::isfinite(model->m_z) ||
        !std::isfinite(model->m_w) || !std::isfinite(model->c6))
        return fail(SKYR_E_INVAL, "masses and c6 must be finite");
    if (model->form != SKYR_FORM_EXACT && model->form != SKYR_FORM_PRINTED)
        return fail(SKYR_E_INVAL, "unknown gradient form");
    if (model->form == SKYR_FORM_PRINTED && model->c6 != 0.0)
        return fail(SKYR_E_INVAL, "the printed form has no sextic term");
    if (!aligned256(work)) return fail(SKYR_E_INVAL, "workspace must be 256-byte aligned");
    return SKYR_OK;
}

skyr_status skyr_energy_gradient(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                 const void* phi, void* grad, int32_t projected, skyr_obs* parts, void* work,
                                 void* stream)
{
    skyr_status st = check_common(lat, prec, model, phi, work);
    if (st != SKYR_OK) return st;
    double o[8];
    st = run_gradient(lat, prec, model, phi, grad, projected ? 1 : 0, 0, parts ? o : nullptr, work, (hipStream_t)stream);
    if (st != SKYR_OK) return st;
    if (parts) {
        parts->E = o[0];
        parts->E2 = o[1];
        parts->E4 = o[2];
        parts->E0 = o[3];
        parts->B = 0.0;
        parts->virial = o[5];
        parts->max_force = o[6];
        parts->E6 = o[7];
    }
    return SKYR_OK;
}

skyr_status skyr_observables(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model, const void* phi,
                             skyr_obs* out, void* work, void* stream)
{
    skyr_status st = check_common(lat, prec, model, phi, work);
    if (st != SKYR_OK) return st;
    if (!out) return fail(SKYR_E_INVAL, "out must be non-null");
    double o[8];
    st = run_gradient(lat, prec, model, phi, nullptr, 0, 1, o, work, (hipStream_t)stream);
    if (st != SKYR_OK) return st;
    out->E = o[0];
    out->E2 = o[1];
    out->E4 = o[2];
    out->E0 = o[3];
    out->B = o[4];
    out->virial = o[5];
    out->max_force = o[6];
    out->E6 = o[7];
    return SKYR_OK;
}

skyr_status skyr_kinetic_energy(const skyr_lattice* lat, skyr_precision prec, const void* vel, double* out,
                                void* work, void* stream)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (!vel || !out || !work) return fail(SKYR_E_INVAL, "vel, out and work must be non-null");
    if (!aligned256(work)) return fail(SKYR_E_INVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)work;
    double* partials = (double*)(w + CTL_BYTES + OBS_BYTES);
    double* res = (double*)(w + CTL_BYTES + MOM_OUT_OFFSET);
    const long long nI = (long long)(lat->n[0] - 4) * (lat->n[1] - 4) * (lat->n[2] - 4);
    const int nb = (int)std::min<long long>(MOM_MAX_BLOCKS, (nI + MOM_THREADS - 1) / MOM_THREADS);
    if (prec == SKYR_F64)
        hipLaunchKernelGGL(kinetic_kernel<double>, dim3(nb), dim3(MOM_THREADS), 0, s, (const double*)vel, lat->n[0],
                           lat->n[1], lat->n[2], partials);
    else
        hipLaunchKernelGGL(kinetic_kernel<float>, dim3(nb), dim3(MOM_THREADS), 0, s, (const float*)vel, lat->n[0],
                           lat->n[1], lat->n[2], partials);
    SKYR_HIP(hipGetLastError());
    hipLaunchKernelGGL(kinetic_finish_kernel, dim3(1), dim3(MOM_THREADS), 0, s, partials, nb, lat->h, res);
    SKYR_HIP(hipGetLastError());
    SKYR_HIP(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s));
    SKYR_HIP(hipStreamSynchronize(s));
    return SKYR_OK;
}

skyr_status skyr_moments(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model, const void* phi,
                         skyr_moment_obs* out, void* work, void* stream)
{
    skyr_status st = check_common(lat, prec, model, phi, work);
    if (st != SKYR_OK) return st;
    if (!out) return fail(SKYR_E_INVAL, "out must be non-null");
    hipStream_t s = (hipStream_t)stream;
    double o[8];
    st = run_gradient(lat, prec, model, phi, nullptr, 0, 1, o, work, s);  // E on the device at obs[0]
    if (st != SKYR_OK) return st;
    char* w = (char*)work;
    MomArgs m;
    m.phi = phi;
    m.n0 = lat->n[0];
    m.n1 = lat->n[1];
    m.n2 = lat->n[2];
    m.h = lat->h;
    m.partials = (double*)(w + CTL_BYTES + OBS_BYTES);
    m.obs = (const double*)(w + CTL_BYTES);
    m.centre = (double*)(w + CTL_BYTES + MOM_CENTRE_OFFSET);
    m.out = (double*)(w + CTL_BYTES + MOM_OUT_OFFSET);
    const long long nI = (long long)(lat->n[0] - 4) * (lat->n[1] - 4) * (lat->n[2] - 4);
    const int nb = (int)std::min<long long>(MOM_MAX_BLOCKS, (nI + MOM_THREADS - 1) / MOM_THREADS);
    if (prec == SKYR_F64)
        hipLaunchKernelGGL((moments_kernel<double, MOM_PASS_CENTRE>), dim3(nb), dim3(MOM_THREADS), 0, s, m);
    else
        hipLaunchKernelGGL((moments_kernel<float, MOM_PASS_CENTRE>), dim3(nb), dim3(MOM_THREADS), 0, s, m);
    SKYR_HIP(hipGetLastError());
    hipLaunchKernelGGL(moments_centre_kernel, dim3(1), dim3(MOM_THREADS), 0, s, m, nb);
    SKYR_HIP(hipGetLastError());
    if (prec == SKYR_F64)
        hipLaunchKernelGGL((moments_kernel<double, MOM_PASS_TENSORS>), dim3(nb), dim3(MOM_THREADS), 0, s, m);
    else
        hipLaunchKernelGGL((moments_kernel<float, MOM_PASS_TENSORS>), dim3(nb), dim3(MOM_THREADS), 0, s, m);
    SKYR_HIP(hipGetLastError());
    hipLaunchKernelGGL(moments_finish_kernel, dim3(1), dim3(MOM_THREADS), 0, s, m, nb);
    SKYR_HIP(hipGetLastError());
    SKYR_HIP(hipMemcpyAsync(out, m.out, sizeof(skyr_moment_obs), hipMemcpyDeviceToHost, s));
    SKYR_HIP(hipStreamSynchronize(s));
    if (!(std::fabs(out->B) >= 1e-6)) return fail(SKYR_E_NONFINITE, "|B| < 1e-6: the centre of mass is undefined");
    const double* v = &out->B;
    for (int k = 0; k < MOM_OUT_DOUBLES; ++k)
        if (!std::isfinite(v[k])) return fail(SKYR_E_NONFINITE, "a moment observable is not finite");
    return SKYR_OK;
}

}  // extern "C"

namespace skyr {

// argument checks of a flow call (before any device work)
static skyr_status check_flow(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                              const skyr_flow* flow, void* phi, void* phi_alt, void* vel, skyr_anf_state* st,
                              int64_t nsteps, void* work)
{
    skyr_status rc = check_common(lat, prec, model, phi, work);
    if (rc != SKYR_OK) return rc;
    if (!flow || !phi_alt || !vel || !st) return fail(SKYR_E_INVAL, "flow, phi_alt, vel and st must be non-null");
    if (!(flow->dt > 0.0) || !std::isfinite(flow->dt)) return fail(SKYR_E_INVAL, "dt must be positive");
    if (!(flow->tol >= 0.0)) return fail(SKYR_E_INVAL, "tol must be >= 0");
    if (nsteps < 0 || flow->max_steps < 0 || flow->renorm64_every < 0) return fail(SKYR_E_INVAL, "negative step count");
    if (flow->mode < SKYR_ARREST_ENERGY || flow->mode > SKYR_GRADIENT_FLOW) return fail(SKYR_E_INVAL, "unknown flow mode");
    if (phi == phi_alt || phi == vel || phi_alt == vel) return fail(SKYR_E_INVAL, "phi, phi_alt and vel must differ");
    return SKYR_OK;
}

// bytes of workspace one flow call uses: control block, observables and the partial
// sums of the sweep it launches
static size_t flow_work_bytes(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model)
{
    const int nb = model->form == SKYR_FORM_PRINTED ? plan_printed(lat, prec).blocks() : plan(lat, prec).blocks();
    return CTL_BYTES + OBS_BYTES + (size_t)nb * NPART * sizeof(double);
}

// ------------------------------------------------------------ flow graphs
// The single-field flow replays its step sweeps in groups of kFlowGraphSweeps from a graph
// instantiated once per launch (kernel, grid, block size, the sweep's arguments, device); a
// small cache keeps the most recently used.  Launches happen under the cache lock, so that
// no graph is destroyed while another thread enqueues it.
constexpr int kFlowGraphSweeps = 32;
constexpr size_t kFlowGraphCache = 8;
struct FlowGraph {
    int device;
    const void* fn;
    int grid, threads;
    SweepArgs args;
    hipGraph_t graph;
    hipGraphExec_t exec;
};
static std::mutex g_flow_graph_mu;
static std::vector<FlowGraph> g_flow_graphs;  // least recently used first

// enqueue reps x kFlowGraphSweeps launches of step kernel fn (grid x threads) with
// arguments a on stream s
static skyr_status flow_graph_launch(const void* fn, int grid, int threads, const SweepArgs& a, int reps,
                                     hipStream_t s)
{
    if (!fn) return fail(SKYR_E_INVAL, "no step kernel for this tile shape");
    int dev = 0;
    SKYR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_flow_graph_mu);
    size_t i = 0;
    for (; i < g_flow_graphs.size(); ++i) {
        const FlowGraph& f = g_flow_graphs[i];
        if (f.device == dev && f.fn == fn && f.grid == grid && f.threads == threads &&
            std::memcmp(&f.args, &a, sizeof a) == 0)
            break;
    }
    if (i == g_flow_graphs.size()) {
        FlowGraph f{dev, fn, grid, threads, a, nullptr, nullptr};
        void* argv[1] = {&f.args};
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(fn);
        p.gridDim = dim3(grid);
        p.blockDim = dim3(threads);
        p.sharedMemBytes = 0;
        p.kernelParams = argv;
        p.extra = nullptr;
        hipError_t e = hipGraphCreate(&f.graph, 0);
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < kFlowGraphSweeps && e == hipSuccess; ++k) {
            hipGraphNode_t node = nullptr;
            e = hipGraphAddKernelNode(&node, f.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
            prev = node;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&f.exec, f.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (f.graph) (void)hipGraphDestroy(f.graph);
            return fail(SKYR_E_DEVICE, std::string("flow graph: ") + hipGetErrorString(e));
        }
        if (g_flow_graphs.size() == kFlowGraphCache) {
            // the evicted graph may still run on some stream of this process
            SKYR_HIP(hipDeviceSynchronize());
            (void)hipGraphExecDestroy(g_flow_graphs.front().exec);
            (void)hipGraphDestroy(g_flow_graphs.front().graph);
            g_flow_graphs.erase(g_flow_graphs.begin());
        }
        g_flow_graphs.push_back(f);
        i = g_flow_graphs.size() - 1;
    } else if (i + 1 != g_flow_graphs.size()) {
        std::rotate(g_flow_graphs.begin() + i, g_flow_graphs.begin() + i + 1, g_flow_graphs.end());
        i = g_flow_graphs.size() - 1;
    }
    for (int r = 0; r < reps; ++r) SKYR_HIP(hipGraphLaunch(g_flow_graphs[i].exec, s));
    return SKYR_OK;
}

// the flow itself, after the argument checks.  timed: record sweep events while timing is
// enabled (skyr_timing_enable; every sweep is then launched directly); graphs: replay whole
// groups of sweeps from a cached graph (exact form, timing off)
static skyr_status anf_run(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                           const skyr_flow* flow, void* phi, void* phi_alt, void* vel, skyr_anf_state* st,
                           int64_t nsteps, void* work, hipStream_t s, bool timed, bool graphs, int lead = 0,
                           int pitch = 0)
{
    const int64_t target = std::min<int64_t>(st->steps + nsteps, flow->max_steps);
    if (st->converged || target <= st->steps) return SKYR_OK;

    const bool printed = model->form == SKYR_FORM_PRINTED;
    const Launch L = printed ? plan_printed(lat, prec) : plan(lat, prec);
    char* w = (char*)work;
    Ctl* ctl = (Ctl*)w;
    SweepArgs a = make_args(lat, L, model, flow->dt);
    if (pitch > 0) use_padded_rows(a, lat, lead, pitch);
    const long long array_sites = pitch > 0 ? (long long)lat->n[0] * lat->n[1] * pitch : sites(lat);
    a.gradient_flow = flow->mode == SKYR_GRADIENT_FLOW;
    a.phi0 = phi;
    a.phi1 = phi_alt;
    a.vel = vel;
    a.partials = (double*)(w + CTL_BYTES + OBS_BYTES);
    a.ctl = ctl;

    Ctl h{};
    h.cur = 0;
    h.redo = st->redo_pending;
    h.steps = st->steps;
    h.target = target;
    h.arrests = st->arrests;
    h.redo_sweeps = st->redo_sweeps;
    h.sweeps = st->sweeps;
    h.renorm64_every = prec == SKYR_F32_BULK ? flow->renorm64_every : 0;
    h.flow_mode = flow->mode;
    h.nblocks = L.blocks();
    h.E_prev = st->E_prev;
    h.E = st->E;
    h.max_force = st->max_force;
    h.tol = flow->tol;
    h.h3 = lat->h * lat->h * lat->h;
    SKYR_HIP(hipMemcpyAsync(ctl, &h, sizeof h, hipMemcpyHostToDevice, s));
    // the frozen layers of phi_alt must match those of phi (padded rows: the whole arrays)
    if (pitch > 0) {
        SKYR_HIP(hipMemcpyAsync(phi_alt, phi, 4 * array_sites * elem_bytes(prec), hipMemcpyDeviceToDevice, s));
    } else {
        const long long N3 = sites(lat);
        const int blocks = (int)std::min<long long>((N3 + 255) / 256, 8192);
        if (prec == SKYR_F64)
            hipLaunchKernelGGL(copy_frozen_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)phi,
                               (double*)phi_alt, lat->n[0], lat->n[1], lat->n[2]);
        else
            hipLaunchKernelGGL(copy_frozen_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)phi,
                               (float*)phi_alt, lat->n[0], lat->n[1], lat->n[2]);
        SKYR_HIP(hipGetLastError());
    }
    // sweeps are enqueued in groups; the host looks at the control block between groups
    // (sweeps after the flow has stopped return at once)
    graphs = graphs && !(timed && g_timing.on);
    const int64_t max_group = graphs ? 4 * kFlowGraphSweeps : 32;
    const int64_t remaining = target - st->steps;
    int64_t group = std::min<int64_t>(std::max<int64_t>(remaining, 1), max_group);
    int64_t budget = 2 * remaining + 2;  // every step takes at most one redo sweep
    // (each sweep takes the flow's decision in its last block)
    auto enqueue_sweep = [&](bool timed) -> hipError_t {
        hipError_t e = timed ? timing_mark(s) : hipSuccess;
        if (e == hipSuccess) e = printed ? sweep_printed(prec, MODE_STEP, L, a, s) : sweep(prec, MODE_STEP, L, a, s);
        if (e == hipSuccess && timed) e = timing_mark(s);
        return e;
    };
    for (;;) {
        if (graphs && group >= kFlowGraphSweeps) {
            const int reps = (int)(group / kFlowGraphSweeps);
            int threads = 0;
            const void* fn = printed ? printed_kernel(prec, MODE_STEP, a, threads)
                                     : step_kernel(prec, L.variant, ext_level(a), threads);
            const skyr_status rc = flow_graph_launch(fn, L.blocks(), threads, a, reps, s);
            if (rc != SKYR_OK) return rc;
            group = (int64_t)reps * kFlowGraphSweeps;
        } else {
            for (int64_t i = 0; i < group; ++i) SKYR_HIP(enqueue_sweep(timed));
        }
        budget -= group;
        SKYR_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
        SKYR_HIP(hipStreamSynchronize(s));
        if (timed) SKYR_HIP(timing_collect());
        if (h.done || budget <= 0) break;
        group = std::min<int64_t>(std::max<int64_t>(h.target - h.steps, 1), max_group);
    }
    if (h.restore) {
        // converged in the last sweep of a group: one more sweep puts v_k back
        SKYR_HIP(enqueue_sweep(false));
        SKYR_HIP(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
        SKYR_HIP(hipStreamSynchronize(s));
    }
    if (h.cur == 1) {
        SKYR_HIP(hipMemcpyAsync(phi, phi_alt, 4 * array_sites * elem_bytes(prec), hipMemcpyDeviceToDevice, s));
        SKYR_HIP(hipStreamSynchronize(s));
    }
    st->steps = h.steps;
    st->arrests = h.arrests;
    st->redo_sweeps = h.redo_sweeps;
    st->sweeps = h.sweeps;
    st->E_prev = h.E_prev;
    st->E = h.E;
    st->max_force = h.max_force;
    st->converged = h.status == 1;
    st->redo_pending = h.redo;
    st->nonfinite = h.status == 3;
    if (st->nonfinite) return fail(SKYR_E_NONFINITE, "energy or force is not finite");
    if (!h.done) return fail(SKYR_E_DEVICE, "flow did not reach its target within the sweep budget");
    return SKYR_OK;
}

// ------------------------------------------------------ allocation-free flow
// The workspace of skyr_anf_step_noalloc: a fixed device array.  Every device holds
// its own copy at its own address (taken once per device with hipGetSymbolAddress and
// kept for the life of the process); host code uses only that address, never the
// array's name, which on the host is a stand-in and not a device pointer.
static __device__ __align__(256) unsigned char scratch[SKYR_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// the scratch address on the current device
static skyr_status scratch_on_current_device(void** out)
{
    int dev = -1;
    SKYR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SKYR_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(SKYR_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SKYR_OK;
}

}  // namespace skyr

extern "C" {

skyr_status skyr_anf_step(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                          const skyr_flow* flow, void* phi, void* phi_alt, void* vel, skyr_anf_state* st,
                          int64_t nsteps, void* work, void* stream)
{
    const skyr_status rc = check_flow(lat, prec, model, flow, phi, phi_alt, vel, st, nsteps, work);
    if (rc != SKYR_OK) return rc;
    return anf_run(lat, prec, model, flow, phi, phi_alt, vel, st, nsteps, work, (hipStream_t)stream, true, true);
}

skyr_status skyr_anf_step_padded(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                 const skyr_flow* flow, void* phi, void* phi_alt, void* vel, skyr_anf_state* st,
                                 int64_t nsteps, void* work, int32_t lead, int32_t pitch, void* stream)
{
    skyr_status rc = check_flow(lat, prec, model, flow, phi, phi_alt, vel, st, nsteps, work);
    if (rc != SKYR_OK) return rc;
    if (model->form != SKYR_FORM_EXACT) return fail(SKYR_E_INVAL, "padded fields run the exact-gradient sweep only");
    rc = check_padded_rows(lat, prec, lead, pitch);
    if (rc != SKYR_OK) return rc;
    return anf_run(lat, prec, model, flow, phi, phi_alt, vel, st, nsteps, work, (hipStream_t)stream, true, true, lead,
                   pitch);
}

skyr_status skyr_anf_step_noalloc(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                  const skyr_flow* flow, void* phi, void* phi_alt, void* vel, skyr_anf_state* st,
                                  int64_t nsteps, void* stream)
{
    // the checks need a non-null, aligned workspace; the scratch address is known only
    // after the lattice has been checked, so a stand-in value is checked first
    void* const stand_in = (void*)(uintptr_t)256;
    skyr_status rc = check_flow(lat, prec, model, flow, phi, phi_alt, vel, st, nsteps, stand_in);
    if (rc != SKYR_OK) return rc;
    const size_t need = flow_work_bytes(lat, prec, model);
    if (need > SKYR_NOALLOC_SCRATCH_BYTES)
        return fail(SKYR_E_INVAL, "this lattice needs " + std::to_string(need) + " bytes of workspace; the fixed scratch holds " +
                                      std::to_string((size_t)SKYR_NOALLOC_SCRATCH_BYTES));
    void* work = nullptr;
    rc = scratch_on_current_device(&work);
    if (rc != SKYR_OK) return rc;
    // direct launches only: instantiating a graph may allocate
    return anf_run(lat, prec, model, flow, phi, phi_alt, vel, st, nsteps, work, (hipStream_t)stream, false, false);
}

}  // extern "C"

// ============================================================ block sweeps
namespace skyr {

// Geometry of a block: padded extents and the ranges, in padded coordinates, of the own
// box, of I (the lattice's interior) and of the output region (own sites in I).
struct BlockGeo {
    int P[3];         // padded extent per axis
    int e[3];         // own extent
    int org[3];       // origin
    int n[3];         // lattice
    int ilo[3], ihi[3];
    int olo[3], ohi[3];
    bool empty;       // no own site in I
    __host__ __device__ long long sites() const { return (long long)P[0] * P[1] * P[2]; }
    __host__ __device__ long long shell() const { return sites() - (long long)e[0] * e[1] * e[2]; }
};

static skyr_status block_geo(const skyr_block* blk, BlockGeo& g)
{
    if (!blk) return fail(SKYR_E_INVAL, "block is null");
    const skyr_lattice& L = blk->lattice;
    for (int d = 0; d < 3; ++d)
        if (L.n[d] < 5) return fail(SKYR_E_INVAL, "every lattice dimension must be at least 5");
    if (!(L.h > 0.0) || !std::isfinite(L.h)) return fail(SKYR_E_INVAL, "lattice spacing must be positive");
    g.empty = false;
    for (int d = 0; d < 3; ++d) {
        const int o = blk->origin[d], e = blk->extent[d];
        if (e < 1 || o < 0 || (long long)o + e > L.n[d]) return fail(SKYR_E_INVAL, "block outside its lattice");
        g.e[d] = e;
        g.org[d] = o;
        g.n[d] = L.n[d];
        g.P[d] = e + 8;
        // padded index p holds lattice site p + o - 4
        g.ilo[d] = 2 - (o - 4);
        g.ihi[d] = L.n[d] - 3 - (o - 4);
        g.olo[d] = std::max(4, g.ilo[d]);
        g.ohi[d] = std::min(e + 3, g.ihi[d]);
        if (g.olo[d] > g.ohi[d]) g.empty = true;
    }
    if (g.sites() >= (1LL << 31) / 4) return fail(SKYR_E_INVAL, "padded block too large for 32-bit component offsets");
    return SKYR_OK;
}

// tile shape, slab length and tile grid of a block's output region
static Launch plan_block(const BlockGeo& g, skyr_precision prec)
{
    int oe[3];
    for (int d = 0; d < 3; ++d) oe[d] = std::max(1, g.ohi[d] - g.olo[d] + 1);
    // the shape and slabs of a lattice whose interior has the region's extents
    skyr_lattice pseudo{};
    for (int d = 0; d < 3; ++d) pseudo.n[d] = oe[d] + 4;
    pseudo.h = 1.0;
    Launch L = plan(&pseudo, prec);
    L.tiles_y = (oe[1] + L.shape.oy() - 1) / L.shape.oy();
    L.tiles_z = (oe[2] + L.shape.oz() - 1) / L.shape.oz();
    L.zstart = g.olo[2];
    L.slabs = (oe[0] + L.xchunk - 1) / L.xchunk;
    return L;
}

static size_t block_work_bytes(const BlockGeo& g, skyr_precision prec)
{
    return CTL_BYTES + OBS_BYTES + (size_t)plan_block(g, prec).blocks() * NPART * sizeof(double);
}

// rank of padded site (x, y, z) among the shell sites (row-major order, own box left out)
__device__ __forceinline__ long long shell_rank(int x, int y, int z, int P1, int P2, int e0, int e1, int e2)
{
    const long long plane = (long long)P1 * P2, ring = plane - (long long)e1 * e2;
    if (x < 4) return x * plane + (long long)y * P2 + z;
    if (x >= 4 + e0) return 4 * plane + e0 * ring + (long long)(x - 4 - e0) * plane + (long long)y * P2 + z;
    long long r = 4 * plane + (long long)(x - 4) * ring;
    if (y < 4) return r + (long long)y * P2 + z;
    if (y >= 4 + e1) return r + 4LL * P2 + (long long)e1 * (P2 - e2) + (long long)(y - 4 - e1) * P2 + z;
    return r + 4LL * P2 + (long long)(y - 4) * (P2 - e2) + (z < 4 ? z : z - e2);
}

// The shell of a padded block field.  Pass 0: shell sites inside the lattice from the
// shell buffer.  Pass 1 (after pass 0): shell sites outside the lattice from the nearest
// lattice site, which pass 0 or the own box has filled.
template <typename T>
__global__ void block_shell_kernel(T* __restrict__ phi, const T* __restrict__ shell, BlockGeo g, int pass, int lead,
                                   int pitch)
{
    const long long N = g.sites(), S = g.shell();
    const int P1 = g.P[1], P2 = g.P[2];
    // the stored element of component A at padded site (x, y, z): component-major arrays, or
    // (pitch > 0) rows of `pitch` elements holding the four components one after the other
    const auto at = [&](int A, int x, int y, int z) -> long long {
        return pitch > 0 ? ((long long)((long long)x * P1 + y) * 4 + A) * pitch + lead + z
                         : (long long)A * N + ((long long)x * P1 + y) * P2 + z;
    };
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < N; s += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(s % P2), y = (int)((s / P2) % P1), x = (int)(s / ((long long)P1 * P2));
        const int p[3] = {x, y, z};
        bool own = true, inside = true;
        int q[3];
        for (int d = 0; d < 3; ++d) {
            own = own && p[d] >= 4 && p[d] < 4 + g.e[d];
            const int gl = p[d] + g.org[d] - 4;  // lattice site
            inside = inside && gl >= 0 && gl < g.n[d];
            q[d] = min(max(gl, 0), g.n[d] - 1) - g.org[d] + 4;  // padded index of the nearest lattice site
        }
        if (own) continue;
        if (pass == 0 && inside) {
            const long long r = shell_rank(x, y, z, P1, P2, g.e[0], g.e[1], g.e[2]);
            for (int A = 0; A < 4; ++A) phi[at(A, x, y, z)] = shell[A * S + r];
        } else if (pass == 1 && !inside) {
            for (int A = 0; A < 4; ++A) phi[at(A, x, y, z)] = phi[at(A, q[0], q[1], q[2])];
        }
    }
}

// the control block of one block step: no decision taken (the caller's), state as given
__global__ void block_ctl_kernel(Ctl* __restrict__ ctl, int redo, int renorm64, int nblocks)
{
    if (threadIdx.x != 0) return;
    Ctl c{};
    c.redo = redo;
    c.renorm64_every = renorm64 ? 1 : 0;
    c.nblocks = nblocks;
    c.hold = 1;
    c.target = INT64_MAX;
    c.E_prev = INFINITY;
    *ctl = c;
}

// out = {E, E2, E4, E0, E6, power, max_force}
__global__ void block_sums_kernel(const double* __restrict__ part, int nblocks, double h, int step,
                                  double* __restrict__ out)
{
    double s[NRED];
    reduce_partials(part, nblocks, s);
    if (threadIdx.x == 0) {
        const double h3 = h * h * h;
        const double E2 = h3 * s[P_E2], E4 = h3 * s[P_E4], E0 = h3 * s[P_E0], E6 = h3 * s[P_E6];
        out[0] = E2 + E4 + E0 + E6;  // in step mode the whole density is summed in the first slot
        out[1] = step ? 0.0 : E2;
        out[2] = E4;
        out[3] = E0;
        out[4] = E6;
        out[5] = h3 * s[P_POW];
        out[6] = sqrt(s[P_F2]);
    }
}

}  // namespace skyr

extern "C" {

int64_t skyr_block_sites(const skyr_block* blk)
{
    BlockGeo g;
    return block_geo(blk, g) == SKYR_OK ? g.sites() : 0;
}

int64_t skyr_block_shell_sites(const skyr_block* blk)
{
    BlockGeo g;
    return block_geo(blk, g) == SKYR_OK ? g.shell() : 0;
}

size_t skyr_block_workspace_bytes(const skyr_block* blk, skyr_precision prec)
{
    BlockGeo g;
    if (block_geo(blk, g) != SKYR_OK) return 0;
    if (prec != SKYR_F64 && prec != SKYR_F32_BULK) return 0;
    return block_work_bytes(g, prec);
}

}  // extern "C"

namespace skyr {

// skyr_block_sweep and skyr_block_sweep_padded (pitch > 0: the stored arrays hold rows of
// `pitch` elements with the four components of a row one after the other, the padded
// index z of a row at element lead + z)
static skyr_status block_sweep_impl(const skyr_block* blk, skyr_precision prec, const skyr_model* model, int32_t mode,
                                    int32_t projected, double dt, int32_t redo, int32_t renorm64, void* phi,
                                    const void* shell, void* out, void* vel, skyr_block_sums* sums, void* work,
                                    void* stream, int lead, int pitch)
{
    BlockGeo g;
    skyr_status rc = block_geo(blk, g);
    if (rc != SKYR_OK) return rc;
    if (pitch > 0) {
        if (lead < 0 || pitch < (long long)lead + g.P[2]) return fail(SKYR_E_INVAL, "need lead >= 0 and pitch >= lead + P2");
        if (4LL * g.P[0] * g.P[1] * pitch * (long long)elem_bytes(prec) >= (1LL << 32))
            return fail(SKYR_E_INVAL, "padded block arrays too large for 32-bit offsets");
    }
    rc = check_common(&blk->lattice, prec, model, phi, work);
    if (rc != SKYR_OK) return rc;
    if (model->form != SKYR_FORM_EXACT) return fail(SKYR_E_INVAL, "block sweeps use the exact-gradient form");
    if (mode != SKYR_BLOCK_GRADIENT && mode != SKYR_BLOCK_STEP) return fail(SKYR_E_INVAL, "unknown block mode");
    if (!shell || !out) return fail(SKYR_E_INVAL, "shell and out must be non-null");
    const bool step = mode == SKYR_BLOCK_STEP;
    if (step && !vel) return fail(SKYR_E_INVAL, "a step needs vel");
    if (step && (!(dt > 0.0) || !std::isfinite(dt))) return fail(SKYR_E_INVAL, "dt must be positive");
    if (out == phi || (step && (vel == phi || vel == out))) return fail(SKYR_E_INVAL, "phi, out and vel must differ");
    hipStream_t s = (hipStream_t)stream;
    if (g.empty) {
        if (sums) *sums = skyr_block_sums{};
        return SKYR_OK;
    }
    // the shell
    {
        const int blocks = (int)std::min<long long>((g.sites() + 255) / 256, 8192);
        for (int pass = 0; pass < 2; ++pass) {
            if (prec == SKYR_F64)
                hipLaunchKernelGGL(block_shell_kernel<double>, dim3(blocks), dim3(256), 0, s, (double*)phi,
                                   (const double*)shell, g, pass, lead, pitch);
            else
                hipLaunchKernelGGL(block_shell_kernel<float>, dim3(blocks), dim3(256), 0, s, (float*)phi,
                                   (const float*)shell, g, pass, lead, pitch);
            SKYR_HIP(hipGetLastError());
        }
    }
    const Launch L = plan_block(g, prec);
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.n0 = g.P[0];
    a.n1 = g.P[1];
    a.n2 = g.P[2];
    a.cstride = g.sites();
    a.zlo = 0;
    a.zhi = g.P[2] - 1;
    for (int d = 0; d < 3; ++d) {
        a.ilo[d] = g.ilo[d];
        a.ihi[d] = g.ihi[d];
        a.olo[d] = g.olo[d];
        a.ohi[d] = g.ohi[d];
    }
    a.tiles_z = L.tiles_z;
    a.tiles_y = L.tiles_y;
    a.zstart = L.zstart;
    a.xchunk = L.xchunk;
    if (pitch > 0) {
        // the same tiles over the same padded sites, each component within its quarter of a row
        a.n2 = 4 * pitch;
        a.cstride = pitch;
        a.zlo = lead;
        a.zhi = lead + g.P[2] - 1;
        a.ilo[2] += lead;
        a.ihi[2] += lead;
        a.olo[2] += lead;
        a.ohi[2] += lead;
        a.zstart += lead;
    }
    a.h = blk->lattice.h;
    a.m = model->m;
    a.m_y = model->m_y;
    a.m_z = model->m_z;
    a.m_w = model->m_w;
    a.c6 = model->c6;
    a.dt = step ? dt : 0.0;
    char* w = (char*)work;
    Ctl* ctl = (Ctl*)w;
    double* res = (double*)(w + CTL_BYTES);
    a.partials = (double*)(w + CTL_BYTES + OBS_BYTES);
    a.phi0 = phi;
    if (step) {
        a.phi1 = out;
        a.vel = vel;
        a.ctl = ctl;
        hipLaunchKernelGGL(block_ctl_kernel, dim3(1), dim3(64), 0, s, ctl, redo ? 1 : 0,
                           (prec == SKYR_F32_BULK && renorm64) ? 1 : 0, L.blocks());
        SKYR_HIP(hipGetLastError());
    } else {
        a.grad = out;
        a.projected = projected ? 1 : 0;
    }
    SKYR_HIP(timing_mark(s));
    SKYR_HIP(sweep(prec, step ? MODE_STEP : MODE_GRAD, L, a, s));
    SKYR_HIP(timing_mark(s));
    if (sums) {
        hipLaunchKernelGGL(block_sums_kernel, dim3(1), dim3(256), 0, s, a.partials, L.blocks(), blk->lattice.h,
                           step ? 1 : 0, res);
        SKYR_HIP(hipGetLastError());
        double o[7];
        SKYR_HIP(hipMemcpyAsync(o, res, sizeof o, hipMemcpyDeviceToHost, s));
        SKYR_HIP(hipStreamSynchronize(s));
        SKYR_HIP(timing_collect());
        sums->E = o[0];
        sums->E2 = o[1];
        sums->E4 = o[2];
        sums->E0 = o[3];
        sums->E6 = o[4];
        sums->power = o[5];
        sums->max_force = o[6];
    }
    return SKYR_OK;
}

}  // namespace skyr

extern "C" {

skyr_status skyr_block_sweep(const skyr_block* blk, skyr_precision prec, const skyr_model* model, int32_t mode,
                             int32_t projected, double dt, int32_t redo, int32_t renorm64, void* phi,
                             const void* shell, void* out, void* vel, skyr_block_sums* sums, void* work, void* stream)
{
    return skyr::block_sweep_impl(blk, prec, model, mode, projected, dt, redo, renorm64, phi, shell, out, vel, sums,
                                  work, stream, 0, 0);
}

skyr_status skyr_block_sweep_padded(const skyr_block* blk, skyr_precision prec, const skyr_model* model, int32_t mode,
                                    int32_t projected, double dt, int32_t redo, int32_t renorm64, void* phi,
                                    const void* shell, void* out, void* vel, skyr_block_sums* sums, void* work,
                                    int32_t lead, int32_t pitch, void* stream)
{
    if (pitch <= 0) return fail(SKYR_E_INVAL, "pitch must be positive");
    return skyr::block_sweep_impl(blk, prec, model, mode, projected, dt, redo, renorm64, phi, shell, out, vel, sums,
                                  work, stream, lead, pitch);
}

skyr_status skyr_block_layout(const skyr_block* blk, skyr_precision prec, int32_t* lead, int32_t* pitch)
{
    BlockGeo g;
    skyr_status rc = block_geo(blk, g);
    if (rc != SKYR_OK) return rc;
    if (prec != SKYR_F64 && prec != SKYR_F32_BULK) return fail(SKYR_E_INVAL, "unknown precision");
    if (!lead || !pitch) return fail(SKYR_E_INVAL, "lead and pitch must be non-null");
    // the first tile column of the block's sweep on a 128-byte line
    const int line = 128 / (int)elem_bytes(prec);
    const int zstart = g.empty ? 0 : plan_block(g, prec).zstart;
    *lead = (line - zstart % line) % line;
    *pitch = (*lead + g.P[2] + line - 1) / line * line;
    return SKYR_OK;
}

int32_t skyr_tile_variants(skyr_precision prec)
{
    if (prec != SKYR_F64 && prec != SKYR_F32_BULK) return 0;
    return shape_count(prec);
}

skyr_status skyr_tile_variant_info(skyr_precision prec, int32_t variant, int32_t info[3])
{
    if (prec != SKYR_F64 && prec != SKYR_F32_BULK) return fail(SKYR_E_INVAL, "unknown precision");
    if (!info || variant < 0 || variant >= shape_count(prec)) return fail(SKYR_E_INVAL, "no such tile variant");
    const Shape& sh = shape_of(prec, variant);
    info[0] = sh.threads();
    info[1] = sh.oy();
    info[2] = sh.oz();
    return SKYR_OK;
}

skyr_status skyr_set_tile(const skyr_lattice* lat, skyr_precision prec, int32_t variant, int32_t xchunk)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (variant < 0 || variant >= shape_count(prec)) return fail(SKYR_E_INVAL, "no such tile variant");
    if (xchunk < kMinChunk) return fail(SKYR_E_INVAL, "slabs must have at least 16 planes");
    std::lock_guard<std::mutex> g(g_tile_mu);
    g_tiles[TileKey{lat->n[0], lat->n[1], lat->n[2], (int)prec}] = {variant, xchunk};
    return SKYR_OK;
}

skyr_status skyr_get_tile(const skyr_lattice* lat, skyr_precision prec, int32_t* variant, int32_t* xchunk)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    const Launch L = plan(lat, prec);
    if (variant) *variant = L.variant;
    if (xchunk) *xchunk = L.xchunk;
    return SKYR_OK;
}

skyr_status skyr_set_batch_tile(const skyr_lattice* lat, skyr_precision prec, int32_t variant, int32_t xchunk)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (variant < 0 || variant >= shape_count(prec)) return fail(SKYR_E_INVAL, "no such tile variant");
    if (xchunk < kMinChunk) return fail(SKYR_E_INVAL, "slabs must have at least 16 planes");
    std::lock_guard<std::mutex> g(g_tile_mu);
    g_batch_tiles[TileKey{lat->n[0], lat->n[1], lat->n[2], (int)prec}] = {variant, xchunk};
    return SKYR_OK;
}

skyr_status skyr_get_batch_tile(const skyr_lattice* lat, skyr_precision prec, int32_t* variant, int32_t* xchunk)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    const Launch L = plan_batch(lat, prec);
    if (variant) *variant = L.variant;
    if (xchunk) *xchunk = L.xchunk;
    return SKYR_OK;
}

skyr_status skyr_autotune(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model, const skyr_flow* flow,
                          const void* phi, void* phi_alt, void* vel, void* work, void* stream, int32_t* variant_out,
                          int32_t* xchunk_out, double* best_us_out)
{
    skyr_status rc = check_common(lat, prec, model, phi, work);
    if (rc != SKYR_OK) return rc;
    if (model->form != SKYR_FORM_EXACT) return fail(SKYR_E_INVAL, "the autotuner times the exact-gradient sweep");
    if (!flow || !phi_alt || !vel) return fail(SKYR_E_INVAL, "flow, phi_alt and vel must be non-null");
    if (!(flow->dt > 0.0) || !std::isfinite(flow->dt)) return fail(SKYR_E_INVAL, "dt must be positive");
    if (phi == phi_alt || phi == vel || phi_alt == vel) return fail(SKYR_E_INVAL, "phi, phi_alt and vel must differ");
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)work;
    Ctl* ctl = (Ctl*)w;
    // every candidate runs the same sweep: phi -> phi_alt with zero incoming velocity, on a
    // held control block (the sweeps take no decision)
    Ctl h{};
    h.hold = 1;
    h.redo = 1;
    h.target = INT64_MAX;
    h.E_prev = INFINITY;
    SKYR_HIP(hipMemcpyAsync(ctl, &h, sizeof h, hipMemcpyHostToDevice, s));
    // one event pair per timed sweep; the median of a candidate's sweeps is its time
    constexpr int kReps = 5;
    hipEvent_t ev[kReps + 1];
    int made = 0;
    auto cleanup = [&]() {
        for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    };
    for (; made <= kReps; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) {
            cleanup();
            return fail(SKYR_E_DEVICE, "autotune: event creation failed");
        }
    struct Cand {
        int v, xc;
        double us;
        std::vector<double> rounds;  // the medians of the interleaved rounds
    };
    std::vector<Cand> cands;
    // slab lengths: the even splits of the interior x-extent into s = 1, 2, ... slabs
    // (ceil(nx / s) planes, at least kMinChunk), so that the block count is a multiple
    // of the tile count that can be matched to the number of compute units
    const int nx = lat->n[0] - 4;
    for (int v = 0; v < shape_count(prec); ++v) {
        int prev = -1;
        for (int sl = 1; sl <= kMaxSlabs; ++sl) {
            const int xc = std::max(std::min(kMinChunk, nx), (nx + sl - 1) / sl);
            if (xc == prev) continue;
            prev = xc;
            cands.push_back({v, xc, INFINITY, {}});
        }
    }
    auto time_one = [&](Cand& cd, int warm, bool round) -> hipError_t {
        const Launch L = plan_with(lat, prec, cd.v, cd.xc);
        SweepArgs a = make_args(lat, L, model, flow->dt);
        a.gradient_flow = flow->mode == SKYR_GRADIENT_FLOW;
        a.phi0 = phi;
        a.phi1 = phi_alt;
        a.vel = vel;
        a.partials = (double*)(w + CTL_BYTES + OBS_BYTES);
        a.ctl = ctl;
        hipError_t e = hipSuccess;
        for (int r = 0; r < warm && e == hipSuccess; ++r) e = sweep(prec, MODE_STEP, L, a, s);
        if (e == hipSuccess) e = hipEventRecord(ev[0], s);
        for (int r = 0; r < kReps && e == hipSuccess; ++r) {
            e = sweep(prec, MODE_STEP, L, a, s);
            if (e == hipSuccess) e = hipEventRecord(ev[r + 1], s);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[kReps]);
        double t[kReps];
        for (int r = 0; r < kReps && e == hipSuccess; ++r) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
            t[r] = 1e3 * ms;
        }
        if (e == hipSuccess) {
            std::sort(t, t + kReps);
            if (round)
                cd.rounds.push_back(t[kReps / 2]);
            else
                cd.us = std::min(cd.us, t[kReps / 2]);
        }
        return e;
    };
    // the first candidate also warms the device clocks up before anything is compared
    hipError_t e = cands.empty() ? hipSuccess : time_one(cands[0], 24, false);
    for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) e = time_one(cands[i], 1, false);
    // the closest candidates and the default choice are timed again in interleaved rounds;
    // a finalist's time is the median of its rounds (a single lucky round does not decide)
    int dv = 0, dx = 0;
    default_tile(lat, prec, dv, dx);
    size_t di = cands.size();
    for (size_t i = 0; i < cands.size(); ++i)
        if (cands[i].v == dv && cands[i].xc == dx) di = i;
    std::vector<size_t> order(cands.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cands[x].us < cands[y].us; });
    order.resize(std::min<size_t>(4, order.size()));
    if (di < cands.size() && std::find(order.begin(), order.end(), di) == order.end()) order.push_back(di);
    for (int round = 0; round < 3 && e == hipSuccess; ++round)
        for (size_t i = 0; i < order.size() && e == hipSuccess; ++i) e = time_one(cands[order[i]], 1, true);
    for (size_t i : order) {
        auto& r = cands[i].rounds;
        if (r.empty()) continue;
        std::sort(r.begin(), r.end());
        cands[i].us = r[r.size() / 2];
    }
    if (e != hipSuccess) {
        cleanup();
        return fail(SKYR_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
    }
    // the fastest candidate, unless it beats the default by less than the timing spread of
    // close shapes (a few percent between runs): then the default stays
    double best = INFINITY;
    int bv = dv, bx = dx;
    if (!order.empty()) {
        // among the finalists (timed in every round)
        size_t pick = order[0];
        for (size_t i : order)
            if (cands[i].us < cands[pick].us) pick = i;
        if (di < cands.size() && !(cands[pick].us < kAutotuneMargin * cands[di].us)) pick = di;
        best = cands[pick].us;
        bv = cands[pick].v;
        bx = cands[pick].xc;
    }
    cleanup();
    SKYR_HIP(fill(vel, 4 * sites(lat), prec, 0.0, s));
    SKYR_HIP(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> g(g_tile_mu);
        g_tiles[TileKey{lat->n[0], lat->n[1], lat->n[2], (int)prec}] = {bv, bx};
    }
    if (variant_out) *variant_out = bv;
    if (xchunk_out) *xchunk_out = bx;
    if (best_us_out) *best_us_out = best;
    return SKYR_OK;
}

}  // extern "C"

// ================================================================ batches
// A batch owns only its job table, the control blocks and the graph of its sweep slots;
// field, velocity and workspace memory stay with the caller.
struct skyr_batch {
    struct Job {
        bool active = false;
        skyr_lattice lat{};
        skyr_precision prec = SKYR_F64;
        Launch L{};
        void* phi = nullptr;
        void* phi_alt = nullptr;
        long long array_sites = 0;  // sites of the stored arrays (the padded rows included)
    };
    int max_jobs = 0;
    hipStream_t stream = nullptr;    // caller's stream (work is launched here)
    std::vector<Job> jobs;
    std::vector<SweepArgs> args;     // host mirror of d_args
    std::vector<Ctl> ctl;            // host mirror of d_ctl (valid after a run / poll)
    Ctl* d_ctl = nullptr;            // [max_jobs]
    SweepArgs* d_args = nullptr;     // [max_jobs]
    int* d_count = nullptr;          // [max_jobs] blocks of a job
    // Jobs are grouped by (precision, tile shape): group g < F64 shape count is F64 shape g,
    // the rest F32 shape g - (F64 shape count); one kernel serves a group.  A group's jobs
    // form one chain: one batched launch of its jobs per sweep slot (the sweep takes each
    // job's flow decision itself).  Chains share no field, so the graph holds them as
    // independent branches, where one chain's blocks fill the CUs another chain's last
    // blocks leave idle.
    static constexpr int kGroups = 16;
    static constexpr int kChains = kGroups;
    int nchains = 0;
    int chain_group[kChains] = {};
    int* d_map[kChains] = {};  // launch slots (job, block of the job) per chain
    int map_cap[kChains] = {};
    int grid[kChains] = {};
    int ext[kChains] = {};  // the highest kernel variant a job of the chain needs
    bool dirty = true;       // the job tables need rebuilding
    bool params_stale = true;  // the graph's launch parameters predate the job tables
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_sweeps = 0;
    int graph_chains = 0;
    const void* graph_fn[kChains] = {};     // the kernel of each chain in the graph
    std::vector<hipGraphNode_t> nodes;      // [chain][sweep slot]
};

namespace skyr {

static void batch_release_graph(skyr_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_sweeps = 0;
    b->graph_chains = 0;
    b->nodes.clear();
}

static int batch_group(skyr_precision prec, int variant)
{
    return prec == SKYR_F64 ? variant : shape_count(SKYR_F64) + variant;
}
static_assert(sizeof(kShapesF64) / sizeof(Shape) + sizeof(kShapesF32) / sizeof(Shape) <= skyr_batch::kGroups,
              "batch groups");

// upload `v` to a device array of at least v.size() ints, growing it when needed
static skyr_status upload_ints(const std::vector<int>& v, int*& d, int& cap)
{
    const int n = (int)v.size();
    if (n > cap) {
        if (d) SKYR_HIP(hipFree(d));
        d = nullptr;
        SKYR_HIP(hipMalloc((void**)&d, sizeof(int) * n));
        cap = n;
    }
    if (n) SKYR_HIP(hipMemcpy(d, v.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    return SKYR_OK;
}

// Sweep time of block `blk` of a job, in the units of a shape's cost factor: the planes
// of its item (the march's four extra included) times the item's output columns.
static double item_time(const Launch& L, int nx, int blk)
{
    const int tiles = L.tiles_y * L.tiles_z;
    const int slab = blk / tiles;
    const int planes = std::min(L.xchunk, nx - slab * L.xchunk);
    return (double)(planes + 4) * L.shape.oy() * L.shape.oz() * L.shape.cost;
}

// The launch slots of one chain.  Blocks go to the XCDs in pieces of at most one XCD's
// CUs from one job (a job's neighbouring tiles then march through the same planes on
// one L2), the piece of most work first, each to the XCD with the least work so far;
// on each XCD, the pieces with the longest blocks dispatch first.  Launch block p runs
// on XCD p mod 8 as the (p / 8)-th block there; XCDs with fewer blocks are padded with
// empty slots.
static std::vector<int> chain_slots(const skyr_batch* b, const std::vector<int>& jobs, const std::vector<int>& count)
{
    constexpr int kXcds = 8, kPiece = kCUs / kXcds;
    struct Piece {
        int job, first, n;
        double work, longest;
    };
    std::vector<Piece> pieces;
    for (int j : jobs) {
        const auto& J = b->jobs[j];
        const int nx = J.lat.n[0] - 4;
        for (int f = 0; f < count[j]; f += kPiece) {
            Piece pc{j, f, std::min(kPiece, count[j] - f), 0.0, 0.0};
            for (int k = f; k < f + pc.n; ++k) {
                const double t = item_time(J.L, nx, k);
                pc.work += t;
                pc.longest = std::max(pc.longest, t);
            }
            pieces.push_back(pc);
        }
    }
    std::stable_sort(pieces.begin(), pieces.end(), [](const Piece& x, const Piece& y) { return x.work > y.work; });
    std::vector<const Piece*> on[kXcds];
    double load[kXcds] = {};
    for (const Piece& pc : pieces) {
        const int x = (int)(std::min_element(load, load + kXcds) - load);
        load[x] += pc.work;
        on[x].push_back(&pc);
    }
    size_t longest = 0;
    std::vector<int> list[kXcds];
    for (int x = 0; x < kXcds; ++x) {
        std::stable_sort(on[x].begin(), on[x].end(), [](const Piece* p, const Piece* q) { return p->longest > q->longest; });
        for (const Piece* pc : on[x])
            for (int k = pc->first; k < pc->first + pc->n; ++k) {
                list[x].push_back(pc->job);
                list[x].push_back(k);
            }
        longest = std::max(longest, list[x].size() / 2);
    }
    std::vector<int> slots(2 * kXcds * longest, -1);
    for (int x = 0; x < kXcds; ++x)
        for (size_t k = 0; k < list[x].size() / 2; ++k) {
            slots[2 * (k * kXcds + x)] = list[x][2 * k];
            slots[2 * (k * kXcds + x) + 1] = list[x][2 * k + 1];
        }
    return slots;
}

// rebuild the device job tables, chains and launch slots from the host description
static skyr_status batch_rebuild(skyr_batch* b)
{
    std::vector<int> count(b->max_jobs, 0), of_group[skyr_batch::kGroups];
    for (int j = 0; j < b->max_jobs; ++j) {
        const auto& J = b->jobs[j];
        if (!J.active) continue;
        count[j] = J.L.blocks();
        of_group[batch_group(J.prec, J.L.variant)].push_back(j);
    }
    // one chain per group: a group's jobs in one launch per sweep slot, their blocks spread
    // over the XCDs by chain_slots (splitting a group into concurrent chains mixes their
    // blocks on the CUs, and neighbouring tiles of a field no longer march together)
    std::vector<int> list[skyr_batch::kChains];
    int nc = 0;
    for (int g = 0; g < skyr_batch::kGroups; ++g) {
        if (of_group[g].empty()) continue;
        list[nc] = of_group[g];
        b->chain_group[nc] = g;
        ++nc;
    }
    for (int c = 0; c < skyr_batch::kChains; ++c) {
        b->ext[c] = EXT_NONE;
        for (int j : list[c]) b->ext[c] = std::max(b->ext[c], ext_level(b->args[j]));
        const std::vector<int> slots = chain_slots(b, list[c], count);
        skyr_status rc = upload_ints(slots, b->d_map[c], b->map_cap[c]);
        if (rc != SKYR_OK) return rc;
        b->grid[c] = (int)slots.size() / 2;
    }
    b->nchains = nc;
    SKYR_HIP(hipMemcpy(b->d_count, count.data(), sizeof(int) * b->max_jobs, hipMemcpyHostToDevice));
    SKYR_HIP(hipMemcpy(b->d_args, b->args.data(), sizeof(SweepArgs) * b->max_jobs, hipMemcpyHostToDevice));
    b->dirty = false;
    b->params_stale = true;
    return SKYR_OK;
}

// launch parameters of chain c's batched sweep; argv (three entries) receives the
// addresses of its arguments, which live in the batch object
static hipKernelNodeParams chain_params(skyr_batch* b, int c, void** argv)
{
    const int g = b->chain_group[c];
    const bool f64 = g < shape_count(SKYR_F64);
    int threads = 0;
    const void* fn = batch_kernel(f64 ? SKYR_F64 : SKYR_F32_BULK, f64 ? g : g - shape_count(SKYR_F64), b->ext[c],
                                  threads);
    argv[0] = &b->d_args;
    argv[1] = &b->d_map[c];
    argv[2] = &b->d_count;
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(fn);
    p.gridDim = dim3(b->grid[c]);
    p.blockDim = dim3(threads);
    p.sharedMemBytes = 0;
    p.kernelParams = argv;
    p.extra = nullptr;
    return p;
}

// The graph of `sweeps` sweep slots: one kernel node per chain and slot, each chain a
// linear branch of its own.  When only the jobs changed (the same chains with the same
// kernels), the nodes of the instantiated graph get their new grids and tables in place;
// otherwise the graph is built and instantiated anew.
static skyr_status batch_graph(skyr_batch* b, int sweeps)
{
    const int nc = b->nchains;
    void* argv[skyr_batch::kChains][3];
    hipKernelNodeParams prm[skyr_batch::kChains];
    bool same = b->exec && b->graph_sweeps == sweeps && b->graph_chains == nc;
    for (int c = 0; c < nc; ++c) {
        prm[c] = chain_params(b, c, argv[c]);
        if (!prm[c].func) return fail(SKYR_E_INVAL, "no batched kernel for a job's tile shape");
        same = same && prm[c].func == b->graph_fn[c];
    }
    if (same) {
        hipError_t e = hipSuccess;
        for (int c = 0; c < nc && e == hipSuccess; ++c)
            for (int k = 0; k < sweeps && e == hipSuccess; ++k)
                e = hipGraphExecKernelNodeSetParams(b->exec, b->nodes[(size_t)c * sweeps + k], &prm[c]);
        if (e == hipSuccess) {
            b->params_stale = false;
            return SKYR_OK;
        }
        (void)hipGetLastError();  // rebuild below
    }
    batch_release_graph(b);
    hipGraph_t g = nullptr;
    SKYR_HIP(hipGraphCreate(&g, 0));
    b->graph = g;
    b->nodes.assign((size_t)nc * sweeps, nullptr);
    for (int c = 0; c < nc; ++c) {
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < sweeps; ++k) {
            hipGraphNode_t node = nullptr;
            SKYR_HIP(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &prm[c]));
            b->nodes[(size_t)c * sweeps + k] = node;
            prev = node;
        }
        b->graph_fn[c] = prm[c].func;
    }
    SKYR_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->graph_sweeps = sweeps;
    b->graph_chains = nc;
    b->params_stale = false;
    return SKYR_OK;
}

}  // namespace skyr

extern "C" {

skyr_status skyr_batch_create(int32_t max_jobs, void* stream, skyr_batch** out)
{
    if (!out || max_jobs < 1 || max_jobs > 4096) return fail(SKYR_E_INVAL, "max_jobs must be 1..4096, out non-null");
    *out = nullptr;
    skyr_batch* b = new (std::nothrow) skyr_batch();
    if (!b) return fail(SKYR_E_NOMEM, "host allocation failed");
    b->max_jobs = max_jobs;
    b->stream = (hipStream_t)stream;
    b->jobs.resize(max_jobs);
    b->args.assign(max_jobs, SweepArgs{});
    b->ctl.assign(max_jobs, Ctl{});
    for (auto& c : b->ctl) c.done = 1;  // empty slots do nothing
    auto cleanup = [&](hipError_t e) {
        (void)hipFree(b->d_ctl);
        (void)hipFree(b->d_args);
        (void)hipFree(b->d_count);
        delete b;
        return fail(SKYR_E_DEVICE, std::string("skyr_batch_create: ") + hipGetErrorString(e));
    };
    hipError_t e = hipMalloc((void**)&b->d_ctl, sizeof(Ctl) * max_jobs);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_args, sizeof(SweepArgs) * max_jobs);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_count, sizeof(int) * max_jobs);
    if (e == hipSuccess) e = hipMemcpy(b->d_ctl, b->ctl.data(), sizeof(Ctl) * max_jobs, hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(e);
    // every slot points at its own (done) control block
    for (int j = 0; j < max_jobs; ++j) b->args[j].ctl = b->d_ctl + j;
    *out = b;
    return SKYR_OK;
}

}  // extern "C"

namespace skyr {

// the argument checks of skyr_batch_add
static skyr_status batch_add_checks(const skyr_batch* b, const skyr_lattice* lat, skyr_precision prec,
                                    const skyr_model* model, const skyr_flow* flow, const void* phi,
                                    const void* phi_alt, const void* vel, void* work)
{
    if (!b) return fail(SKYR_E_INVAL, "batch is null");
    skyr_status rc = check_common(lat, prec, model, phi, work);
    if (rc != SKYR_OK) return rc;
    if (model->form != SKYR_FORM_EXACT) return fail(SKYR_E_INVAL, "batches run the exact-gradient sweep only");
    if (!flow || !phi_alt || !vel) return fail(SKYR_E_INVAL, "flow, phi_alt and vel must be non-null");
    if (!(flow->dt > 0.0) || !std::isfinite(flow->dt)) return fail(SKYR_E_INVAL, "dt must be positive");
    if (!(flow->tol >= 0.0) || flow->max_steps < 0 || flow->renorm64_every < 0)
        return fail(SKYR_E_INVAL, "tol, max_steps and renorm64_every must be >= 0");
    if (flow->mode < SKYR_ARREST_ENERGY || flow->mode > SKYR_GRADIENT_FLOW) return fail(SKYR_E_INVAL, "unknown flow mode");
    if (phi == phi_alt || phi == vel || phi_alt == vel) return fail(SKYR_E_INVAL, "phi, phi_alt and vel must differ");
    return SKYR_OK;
}

// skyr_batch_add after its argument checks, with the field's launch plan given; pitch > 0:
// the arrays hold rows of `pitch` elements with the lattice's z = 0 at element `lead`
static skyr_status batch_add_launch(skyr_batch* b, const skyr_lattice* lat, skyr_precision prec,
                                    const skyr_model* model, const skyr_flow* flow, void* phi, void* phi_alt,
                                    void* vel, void* work, const Launch& L, int32_t* slot, int lead = 0,
                                    int pitch = 0)
{
    int j = -1;
    for (int k = 0; k < b->max_jobs; ++k)
        if (!b->jobs[k].active) {
            j = k;
            break;
        }
    if (j < 0) return fail(SKYR_E_BUSY, "every batch slot is in use");
    SweepArgs a = make_args(lat, L, model, flow->dt);
    if (pitch > 0) use_padded_rows(a, lat, lead, pitch);
    a.gradient_flow = flow->mode == SKYR_GRADIENT_FLOW;
    a.phi0 = phi;
    a.phi1 = phi_alt;
    a.vel = vel;
    a.partials = (double*)((char*)work + CTL_BYTES + OBS_BYTES);
    a.ctl = b->d_ctl + j;
    const long long array_sites = pitch > 0 ? (long long)lat->n[0] * lat->n[1] * pitch : sites(lat);
    Ctl h{};
    h.target = flow->max_steps;
    h.renorm64_every = prec == SKYR_F32_BULK ? flow->renorm64_every : 0;
    h.flow_mode = flow->mode;
    h.nblocks = L.blocks();
    h.E_prev = INFINITY;
    h.E = NAN;
    h.max_force = NAN;
    h.tol = flow->tol;
    h.h3 = lat->h * lat->h * lat->h;
    h.done = flow->max_steps <= 0 ? 1 : 0;
    h.status = h.done ? 2 : 0;
    hipStream_t s = b->stream;
    SKYR_HIP(hipMemcpyAsync(b->d_ctl + j, &h, sizeof h, hipMemcpyHostToDevice, s));
    if (pitch > 0) {
        // the frozen layers and the padding of phi in phi_alt: the whole arrays
        SKYR_HIP(hipMemcpyAsync(phi_alt, phi, 4 * array_sites * elem_bytes(prec), hipMemcpyDeviceToDevice, s));
    } else {
        const long long N3 = sites(lat);
        const int blocks = (int)std::min<long long>((N3 + 255) / 256, 8192);
        if (prec == SKYR_F64)
            hipLaunchKernelGGL(copy_frozen_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)phi,
                               (double*)phi_alt, lat->n[0], lat->n[1], lat->n[2]);
        else
            hipLaunchKernelGGL(copy_frozen_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)phi,
                               (float*)phi_alt, lat->n[0], lat->n[1], lat->n[2]);
        SKYR_HIP(hipGetLastError());
    }
    SKYR_HIP(hipStreamSynchronize(s));
    auto& J = b->jobs[j];
    J.active = true;
    J.lat = *lat;
    J.prec = prec;
    J.L = L;
    J.phi = phi;
    J.phi_alt = phi_alt;
    J.array_sites = array_sites;
    b->args[j] = a;
    b->ctl[j] = h;
    b->dirty = true;
    if (slot) *slot = j;
    return SKYR_OK;
}

}  // namespace skyr

extern "C" {

skyr_status skyr_batch_add(skyr_batch* b, const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                           const skyr_flow* flow, void* phi, void* phi_alt, void* vel, void* work, int32_t* slot)
{
    skyr_status rc = skyr::batch_add_checks(b, lat, prec, model, flow, phi, phi_alt, vel, work);
    if (rc != SKYR_OK) return rc;
    // tile shape and slab length of the lattice's fields in batches
    return skyr::batch_add_launch(b, lat, prec, model, flow, phi, phi_alt, vel, work, skyr::plan_batch(lat, prec), slot);
}

skyr_status skyr_batch_layout(const skyr_lattice* lat, skyr_precision prec, int32_t* lead, int32_t* pitch)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (!lead || !pitch) return fail(SKYR_E_INVAL, "lead and pitch must be non-null");
    // the first tile column of the lattice's batch tile on a 128-byte line
    const int line = 128 / (int)elem_bytes(prec);
    const Launch L = plan_batch(lat, prec);
    *lead = (line - L.zstart % line) % line;
    *pitch = (*lead + lat->n[2] + line - 1) / line * line;
    return SKYR_OK;
}

skyr_status skyr_batch_add_padded(skyr_batch* b, const skyr_lattice* lat, skyr_precision prec,
                                  const skyr_model* model, const skyr_flow* flow, void* phi, void* phi_alt, void* vel,
                                  void* work, int32_t lead, int32_t pitch, int32_t* slot)
{
    skyr_status rc = skyr::batch_add_checks(b, lat, prec, model, flow, phi, phi_alt, vel, work);
    if (rc != SKYR_OK) return rc;
    rc = skyr::check_padded_rows(lat, prec, lead, pitch);
    if (rc != SKYR_OK) return rc;
    return skyr::batch_add_launch(b, lat, prec, model, flow, phi, phi_alt, vel, work, skyr::plan_batch(lat, prec), slot,
                                  lead, pitch);
}

skyr_status skyr_batch_run(skyr_batch* b, int32_t sweeps)
{
    if (!b || sweeps < 1) return fail(SKYR_E_INVAL, "batch must be non-null and sweeps >= 1");
    if (b->dirty) {
        skyr_status rc = batch_rebuild(b);
        if (rc != SKYR_OK) return rc;
    }
    int blocks = 0;
    for (int c = 0; c < b->nchains; ++c) blocks += b->grid[c];
    if (blocks > 0) {
        if (!b->exec || b->graph_sweeps != sweeps || b->params_stale) {
            skyr_status rc = batch_graph(b, sweeps);
            if (rc != SKYR_OK) return rc;
        }
        SKYR_HIP(hipGraphLaunch(b->exec, b->stream));
    }
    SKYR_HIP(hipMemcpyAsync(b->ctl.data(), b->d_ctl, sizeof(Ctl) * b->max_jobs, hipMemcpyDeviceToHost, b->stream));
    SKYR_HIP(hipStreamSynchronize(b->stream));
    return SKYR_OK;
}

static void state_from_ctl(const Ctl& h, skyr_anf_state* st)
{
    st->steps = h.steps;
    st->arrests = h.arrests;
    st->redo_sweeps = h.redo_sweeps;
    st->sweeps = h.sweeps;
    st->E_prev = h.E_prev;
    st->E = h.E;
    st->max_force = h.max_force;
    st->converged = h.status == 1;
    st->redo_pending = h.redo;
    st->nonfinite = h.status == 3;
    st->_pad = 0;
}

// once a field has stopped, make sure its result sits in phi and, after convergence in the
// last sweep slot of a run, that its velocity is v_k again (a restore sweep of its own)
static skyr_status batch_settle(skyr_batch* b, int j)
{
    Ctl& h = b->ctl[j];
    if (h.restore) {
        const auto& J = b->jobs[j];
        const SweepArgs& a = b->args[j];
        SKYR_HIP(sweep(J.prec, MODE_STEP, J.L, a, b->stream));
        SKYR_HIP(hipMemcpyAsync(&h, a.ctl, sizeof h, hipMemcpyDeviceToHost, b->stream));
        SKYR_HIP(hipStreamSynchronize(b->stream));
    }
    if (h.cur == 1) {
        const auto& J = b->jobs[j];
        SKYR_HIP(hipMemcpyAsync(J.phi, J.phi_alt, 4 * J.array_sites * elem_bytes(J.prec), hipMemcpyDeviceToDevice,
                                b->stream));
        h.cur = 0;
        SKYR_HIP(hipMemcpyAsync(&b->d_ctl[j].cur, &h.cur, sizeof h.cur, hipMemcpyHostToDevice, b->stream));
        SKYR_HIP(hipStreamSynchronize(b->stream));
    }
    return SKYR_OK;
}

skyr_status skyr_batch_poll(skyr_batch* b, int32_t slot, skyr_anf_state* st)
{
    if (!b || !st || slot < 0 || slot >= b->max_jobs || !b->jobs[slot].active)
        return fail(SKYR_E_INVAL, "no such active batch slot");
    const Ctl& h = b->ctl[slot];
    if (h.done) {
        skyr_status rc = batch_settle(b, slot);
        if (rc != SKYR_OK) return rc;
    }
    state_from_ctl(h, st);
    if (st->nonfinite) return fail(SKYR_E_NONFINITE, "energy or force is not finite");
    return SKYR_OK;
}

skyr_status skyr_batch_remove(skyr_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_jobs || !b->jobs[slot].active)
        return fail(SKYR_E_INVAL, "no such active batch slot");
    skyr_status rc = batch_settle(b, slot);
    if (rc != SKYR_OK) return rc;
    b->jobs[slot].active = false;
    Ctl h{};
    h.done = 1;
    b->ctl[slot] = h;
    b->args[slot] = SweepArgs{};
    b->args[slot].ctl = b->d_ctl + slot;
    // from the host mirror (it outlives the copy), in order on the batch's stream
    SKYR_HIP(hipMemcpyAsync(b->d_ctl + slot, &b->ctl[slot], sizeof h, hipMemcpyHostToDevice, b->stream));
    b->dirty = true;
    return SKYR_OK;
}

int32_t skyr_batch_active(const skyr_batch* b)
{
    if (!b) return 0;
    int n = 0;
    for (const auto& J : b->jobs) n += J.active ? 1 : 0;
    return n;
}

skyr_status skyr_batch_destroy(skyr_batch* b)
{
    if (!b) return SKYR_OK;
    (void)hipStreamSynchronize(b->stream);
    batch_release_graph(b);
    (void)hipFree(b->d_ctl);
    (void)hipFree(b->d_args);
    (void)hipFree(b->d_count);
    for (int c = 0; c < skyr_batch::kChains; ++c) (void)hipFree(b->d_map[c]);
    delete b;
    return SKYR_OK;
}

// The batch autotuner: every candidate slab length (the even splits of x into 1 ..
// kMaxSlabs slabs of at least kMinChunk planes, with the batch shape, which keeps the
// fields of one precision in one launch) is given to all the copies in one batch, which
// runs kWarm sweep slots and then kReps timed runs of kSweeps slots; a candidate's time is
// the median of its runs per slot.  The fastest is kept unless it beats the batch default
// by less than kAutotuneMargin.
skyr_status skyr_batch_autotune(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                const skyr_flow* flow, int32_t copies, void* const* phi, void* const* phi_alt,
                                void* const* vel, void* const* work, int32_t lead, int32_t pitch, void* stream,
                                int32_t* variant_out, int32_t* xchunk_out, double* best_us_out)
{
    if (copies < 1 || !phi || !phi_alt || !vel || !work) return fail(SKYR_E_INVAL, "copies >= 1 and buffer arrays required");
    if (!flow) return fail(SKYR_E_INVAL, "flow must be non-null");
    for (int i = 0; i < copies; ++i) {
        skyr_status rc = check_common(lat, prec, model, phi[i], work[i]);
        if (rc != SKYR_OK) return rc;
        if (!phi_alt[i] || !vel[i]) return fail(SKYR_E_INVAL, "phi_alt and vel must be non-null");
        if (phi[i] == phi_alt[i] || phi[i] == vel[i] || phi_alt[i] == vel[i])
            return fail(SKYR_E_INVAL, "phi, phi_alt and vel must differ");
    }
    if (pitch != 0) {
        skyr_status prc = check_padded_rows(lat, prec, lead, pitch);
        if (prc != SKYR_OK) return prc;
    }
    if (model->form != SKYR_FORM_EXACT) return fail(SKYR_E_INVAL, "batches run the exact-gradient sweep only");
    if (!(flow->dt > 0.0) || !std::isfinite(flow->dt)) return fail(SKYR_E_INVAL, "dt must be positive");
    if (flow->mode < SKYR_ARREST_ENERGY || flow->mode > SKYR_GRADIENT_FLOW) return fail(SKYR_E_INVAL, "unknown flow mode");
    hipStream_t s = (hipStream_t)stream;
    // the timed flows never stop: no tolerance, no step limit
    skyr_flow fl = *flow;
    fl.tol = 0.0;
    fl.max_steps = INT64_MAX / 2;
    constexpr int kWarm = 4, kSweeps = 6, kReps = 3;
    skyr_batch* b = nullptr;
    skyr_status rc = skyr_batch_create(copies, stream, &b);
    if (rc != SKYR_OK) return rc;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto done = [&](skyr_status r) {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        (void)skyr_batch_destroy(b);
        return r;
    };
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
        return done(fail(SKYR_E_DEVICE, "batch autotune: event creation failed"));
    struct Cand {
        int v, xc;
        double us;
    };
    std::vector<Cand> cands;
    const int nx = lat->n[0] - 4;
    {
        int prev = -1;
        for (int sl = 1; sl <= kMaxSlabs; ++sl) {
            const int xc = std::max(std::min(kMinChunk, nx), (nx + sl - 1) / sl);
            if (xc == prev) continue;
            prev = xc;
            cands.push_back({kBatchShape, xc, INFINITY});
        }
    }
    int dv = 0, dx = 0;
    batch_default_tile(lat, prec, dv, dx);
    size_t di = cands.size();
    for (size_t i = 0; i < cands.size(); ++i)
        if (cands[i].v == dv && cands[i].xc == dx) di = i;
    const long long array_sites = pitch > 0 ? (long long)lat->n[0] * lat->n[1] * pitch : sites(lat);
    for (Cand& cd : cands) {
        const Launch L = plan_with(lat, prec, cd.v, cd.xc);
        for (int i = 0; i < copies; ++i) {
            if (b->jobs[i].active && (rc = skyr_batch_remove(b, i)) != SKYR_OK) return done(rc);
            SKYR_HIP_OR(fill(vel[i], 4 * array_sites, prec, 0.0, s), done);
            if ((rc = batch_add_launch(b, lat, prec, model, &fl, phi[i], phi_alt[i], vel[i], work[i], L, nullptr, lead,
                                       pitch)) != SKYR_OK)
                return done(rc);
        }
        if ((rc = skyr_batch_run(b, kWarm)) != SKYR_OK) return done(rc);
        double t[kReps];
        for (int r = 0; r < kReps; ++r) {
            SKYR_HIP_OR(hipEventRecord(ev[0], s), done);
            if ((rc = skyr_batch_run(b, kSweeps)) != SKYR_OK) return done(rc);
            SKYR_HIP_OR(hipEventRecord(ev[1], s), done);
            SKYR_HIP_OR(hipEventSynchronize(ev[1]), done);
            float ms = 0.0f;
            SKYR_HIP_OR(hipEventElapsedTime(&ms, ev[0], ev[1]), done);
            t[r] = 1e3 * ms / kSweeps;
        }
        std::sort(t, t + kReps);
        cd.us = t[kReps / 2];
    }
    size_t pick = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (cands[i].us < cands[pick].us) pick = i;
    if (di < cands.size() && !(cands[pick].us < kAutotuneMargin * cands[di].us)) pick = di;
    for (int i = 0; i < copies; ++i)
        if (b->jobs[i].active && (rc = skyr_batch_remove(b, i)) != SKYR_OK) return done(rc);
    for (int i = 0; i < copies; ++i) SKYR_HIP_OR(fill(vel[i], 4 * array_sites, prec, 0.0, s), done);
    SKYR_HIP_OR(hipStreamSynchronize(s), done);
    {
        std::lock_guard<std::mutex> g(g_tile_mu);
        g_batch_tiles[TileKey{lat->n[0], lat->n[1], lat->n[2], (int)prec}] = {cands[pick].v, cands[pick].xc};
    }
    if (variant_out) *variant_out = cands[pick].v;
    if (xchunk_out) *xchunk_out = cands[pick].xc;
    if (best_us_out) *best_us_out = cands[pick].us;
    return done(SKYR_OK);
}

void skyr_timing_enable(int32_t on)
{
    Timing& t = g_timing;
    t.on = on != 0;
    t.used = 0;
    if (t.on) {
        t.ms = 0.0;
        t.launches = 0;
    }
}

skyr_status skyr_timing_read(double* sweep_ms, int64_t* sweep_launches)
{
    Timing& t = g_timing;
    if (t.used > 0) {  // pairs recorded by calls that returned without waiting for them
        SKYR_HIP(hipEventSynchronize(t.ev[t.used - 1]));
        SKYR_HIP(timing_collect());
    }
    if (sweep_ms) *sweep_ms = g_timing.ms;
    if (sweep_launches) *sweep_launches = g_timing.launches;
    return SKYR_OK;
}

}  // extern "C"

// ------------------------------------------------------------ field files
// The program's text and binary formats (Sec. 7.4).  Host code; the device
// variants stage the field through a host buffer.
namespace {
constexpr int32_t kFileMagic = 1234;
constexpr double kFileSentinel = -123456789.0;
constexpr int kMaxExtraParams = 64;

struct FileHeader {
    double xmin[3];
    int32_t n[3];
    double m[4];
    double c6;
};

struct FileCloser {
    FILE* f;
    ~FileCloser()
    {
        if (f) std::fclose(f);
    }
};

bool read_exact(FILE* f, void* p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }

// binary header up to and including the sentinel (extra parameters skipped)
bool read_binary_header(FILE* f, FileHeader& h)
{
    int32_t magic = 0;
    if (!read_exact(f, &magic, 4) || magic != kFileMagic) return false;
    if (!read_exact(f, h.xmin, sizeof h.xmin) || !read_exact(f, h.n, sizeof h.n) || !read_exact(f, h.m, sizeof h.m) ||
        !read_exact(f, &h.c6, sizeof h.c6))
        return false;
    for (int k = 0; k <= kMaxExtraParams; ++k) {
        double v;
        if (!read_exact(f, &v, sizeof v)) return false;
        if (v == kFileSentinel) return true;
    }
    return false;
}

// text header: eleven numbers on the first line
bool read_text_header(FILE* f, FileHeader& h)
{
    char line[4096];
    if (!std::fgets(line, sizeof line, f)) return false;
    double v[11];
    const char* p = line;
    for (int k = 0; k < 11; ++k) {
        char* end = nullptr;
        v[k] = std::strtod(p, &end);
        if (end == p) return false;
        p = end;
    }
    for (int i = 0; i < 3; ++i) h.xmin[i] = v[i];
    for (int i = 0; i < 3; ++i) {
        if (v[3 + i] != std::floor(v[3 + i]) || v[3 + i] < 1.0 || v[3 + i] > 1e9) return false;
        h.n[i] = (int32_t)v[3 + i];
    }
    for (int i = 0; i < 4; ++i) h.m[i] = v[6 + i];
    h.c6 = v[10];
    return true;
}

// open, detect the format, read the header; leaves f after the header
skyr_status open_field_file(const char* path, FILE** out, FileHeader& h, bool& binary)
{
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SKYR_E_IO, std::string("cannot open ") + path);
    int32_t magic = 0;
    binary = read_exact(f, &magic, 4) && magic == kFileMagic;
    std::rewind(f);
    const bool ok = binary ? read_binary_header(f, h) : read_text_header(f, h);
    if (!ok) {
        std::fclose(f);
        return fail(SKYR_E_IO, std::string("malformed field file header: ") + path);
    }
    *out = f;
    return SKYR_OK;
}

// one lattice spacing for all three axes
bool header_lattice(const FileHeader& h, skyr_lattice* lat)
{
    double hs[3];
    for (int i = 0; i < 3; ++i) {
        if (h.n[i] < 2) return false;
        hs[i] = -2.0 * h.xmin[i] / (h.n[i] - 1);
        if (!(hs[i] > 0.0) || !std::isfinite(hs[i])) return false;
    }
    for (int i = 1; i < 3; ++i)
        if (std::fabs(hs[i] - hs[0]) > 1e-12 * hs[0]) return false;
    lat->n[0] = h.n[0];
    lat->n[1] = h.n[1];
    lat->n[2] = h.n[2];
    lat->_pad = 0;
    lat->h = hs[0];
    return true;
}

void header_model(const FileHeader& h, skyr_model* m)
{
    std::memset(m, 0, sizeof *m);
    m->m = h.m[0];
    m->m_y = h.m[1];
    m->m_z = h.m[2];
    m->m_w = h.m[3];
    m->c6 = h.c6;
}
}  // namespace

skyr_status skyr_write_field_host(const char* path, int32_t format, const skyr_lattice* lat, const skyr_model* model,
                                  const double* phi)
{
    skyr_status st = check_lattice(lat, SKYR_F64);
    if (st != SKYR_OK) return st;
    if (!path || !model || !phi) return fail(SKYR_E_INVAL, "path, model and phi must be non-null");
    if (format != SKYR_FILE_BINARY && format != SKYR_FILE_TEXT) return fail(SKYR_E_INVAL, "unknown file format");
    const size_t N3 = (size_t)sites(lat);
    double xmin[3];
    for (int i = 0; i < 3; ++i) xmin[i] = -0.5 * (lat->n[i] - 1) * lat->h;
    const double m[4] = {model->m, model->m_y, model->m_z, model->m_w};
    FileCloser fc{std::fopen(path, format == SKYR_FILE_BINARY ? "wb" : "w")};
    if (!fc.f) return fail(SKYR_E_IO, std::string("cannot create ") + path);
    bool ok = true;
    if (format == SKYR_FILE_BINARY) {
        ok = std::fwrite(&kFileMagic, 4, 1, fc.f) == 1 && std::fwrite(xmin, 8, 3, fc.f) == 3 &&
             std::fwrite(lat->n, 4, 3, fc.f) == 3 && std::fwrite(m, 8, 4, fc.f) == 4 &&
             std::fwrite(&model->c6, 8, 1, fc.f) == 1 && std::fwrite(&kFileSentinel, 8, 1, fc.f) == 1;
        std::vector<double> buf;
        const size_t chunk = 1 << 16;
        for (size_t s0 = 0; ok && s0 < N3; s0 += chunk) {
            const size_t s1 = std::min(N3, s0 + chunk);
            buf.resize(4 * (s1 - s0));
            for (size_t s = s0; s < s1; ++s)
                for (int A = 0; A < 4; ++A) buf[4 * (s - s0) + A] = phi[A * N3 + s];
            ok = std::fwrite(buf.data(), 8, buf.size(), fc.f) == buf.size();
        }
    } else {
        ok = std::fprintf(fc.f, "%.17g\t%.17g\t%.17g\t%d\t%d\t%d\t%.17g\t%.17g\t%.17g\t%.17g\t%.17g\n", xmin[0], xmin[1],
                          xmin[2], lat->n[0], lat->n[1], lat->n[2], m[0], m[1], m[2], m[3], model->c6) > 0;
        for (size_t s = 0; ok && s < N3; ++s)
            ok = std::fprintf(fc.f, "%.17g\t%.17g\t%.17g\t%.17g\n", phi[s], phi[N3 + s], phi[2 * N3 + s],
                              phi[3 * N3 + s]) > 0;
    }
    if (!ok) return fail(SKYR_E_IO, std::string("write failed: ") + path);
    const int rc = std::fclose(fc.f);
    fc.f = nullptr;
    if (rc != 0) return fail(SKYR_E_IO, std::string("write failed: ") + path);
    return SKYR_OK;
}

skyr_status skyr_file_info(const char* path, skyr_lattice* lat_out, skyr_model* model_out)
{
    if (!path) return fail(SKYR_E_INVAL, "path must be non-null");
    FILE* f = nullptr;
    FileHeader h{};
    bool binary = false;
    skyr_status st = open_field_file(path, &f, h, binary);
    if (st != SKYR_OK) return st;
    std::fclose(f);
    skyr_lattice lat{};
    if (!header_lattice(h, &lat)) return fail(SKYR_E_IO, "the file's lattice has unequal or invalid spacings");
    if (lat_out) *lat_out = lat;
    if (model_out) header_model(h, model_out);
    return SKYR_OK;
}

skyr_status skyr_read_field_host(const char* path, const skyr_lattice* lat, skyr_model* model_out, double* phi)
{
    skyr_status st = check_lattice(lat, SKYR_F64);
    if (st != SKYR_OK) return st;
    if (!path || !phi) return fail(SKYR_E_INVAL, "path and phi must be non-null");
    FILE* f = nullptr;
    FileHeader h{};
    bool binary = false;
    st = open_field_file(path, &f, h, binary);
    if (st != SKYR_OK) return st;
    FileCloser fc{f};
    skyr_lattice fl{};
    if (!header_lattice(h, &fl) || fl.n[0] != lat->n[0] || fl.n[1] != lat->n[1] || fl.n[2] != lat->n[2] ||
        std::fabs(fl.h - lat->h) > 1e-12 * lat->h)
        return fail(SKYR_E_INVAL, "the file's lattice differs from the given lattice");
    const size_t N3 = (size_t)sites(lat);
    if (binary) {
        std::vector<double> buf;
        const size_t chunk = 1 << 16;
        for (size_t s0 = 0; s0 < N3; s0 += chunk) {
            const size_t s1 = std::min(N3, s0 + chunk);
            buf.resize(4 * (s1 - s0));
            if (!read_exact(f, buf.data(), 8 * buf.size())) return fail(SKYR_E_IO, "field data truncated");
            for (size_t s = s0; s < s1; ++s)
                for (int A = 0; A < 4; ++A) phi[A * N3 + s] = buf[4 * (s - s0) + A];
        }
    } else {
        for (size_t s = 0; s < N3; ++s) {
            double v[4];
            if (std::fscanf(f, "%lf %lf %lf %lf", &v[0], &v[1], &v[2], &v[3]) != 4)
                return fail(SKYR_E_IO, "field data truncated or malformed");
            for (int A = 0; A < 4; ++A) phi[A * N3 + s] = v[A];
        }
    }
    if (model_out) header_model(h, model_out);
    return SKYR_OK;
}

skyr_status skyr_save_field(const char* path, int32_t format, const skyr_lattice* lat, skyr_precision prec,
                            const skyr_model* model, const void* phi, void* stream)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (!phi) return fail(SKYR_E_INVAL, "phi must be non-null");
    const size_t n = 4 * (size_t)sites(lat);
    std::vector<double> host(n);
    hipStream_t s = (hipStream_t)stream;
    if (prec == SKYR_F64) {
        SKYR_HIP(hipMemcpyAsync(host.data(), phi, n * sizeof(double), hipMemcpyDeviceToHost, s));
        SKYR_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<float> tmp(n);
        SKYR_HIP(hipMemcpyAsync(tmp.data(), phi, n * sizeof(float), hipMemcpyDeviceToHost, s));
        SKYR_HIP(hipStreamSynchronize(s));
        for (size_t k = 0; k < n; ++k) host[k] = tmp[k];
    }
    return skyr_write_field_host(path, format, lat, model, host.data());
}

skyr_status skyr_load_field(const char* path, const skyr_lattice* lat, skyr_precision prec, skyr_model* model_out,
                            void* phi, void* stream)
{
    skyr_status st = check_lattice(lat, prec);
    if (st != SKYR_OK) return st;
    if (!phi) return fail(SKYR_E_INVAL, "phi must be non-null");
    const size_t n = 4 * (size_t)sites(lat);
    std::vector<double> host(n);
    st = skyr_read_field_host(path, lat, model_out, host.data());
    if (st != SKYR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (prec == SKYR_F64) {
        SKYR_HIP(hipMemcpyAsync(phi, host.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
        SKYR_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<float> tmp(n);
        for (size_t k = 0; k < n; ++k) tmp[k] = (float)host[k];
        SKYR_HIP(hipMemcpyAsync(phi, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, s));
        SKYR_HIP(hipStreamSynchronize(s));
    }
    return SKYR_OK;
}

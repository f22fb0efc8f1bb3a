/*
 * skyr.h -- C ABI of the MI355X arrested-Newton-flow library for the 3D Skyrme
 * model in the sigma-model (unit 4-vector) form, arXiv:2604.25876.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Field layout.  A field is four real components per lattice site stored as
 *   structure of arrays  phi[A][x][y][z],  A = 0..3,  z fastest,
 * n[0] x n[1] x n[2] sites per component, contiguous, in double (SKYR_F64) or
 * float (SKYR_F32_BULK).  U = phi^0 + i phi^a tau^a (Sec. 2.1).
 * Coordinates x_i = (i - (n-1)/2) h.  The two outer layers of every face are
 * frozen boundary values (vacuum (1,0,0,0) after skyr_init_field) and are never
 * written by the flow; the interior I = {2..n-3}^3 carries energy, charge and
 * the update.
 *
 * Discrete energy (Sec. 2.1 energy density at one half of the printed
 * normalisation, discretised with the two fourth-order stencils of Sec. 3):
 *   E_h = h^3 sum_{x in I} [ -1/2 phi.Lap_h phi + 1/4 (S^2 - sum_ij G_ij^2)
 *                            + m^2 (1 - phi^0) ]
 * with a_i = D_i phi (first-difference stencil), G_ij = a_i.a_j, S = tr G and
 * Lap_h the sum of the five-point second differences.  The gradient returned
 * and used by the flow is the exact derivative of E_h, in density units
 * (g = h^-3 dE_h/dphi).
 *
 * Memory.  Every field, velocity, gradient and workspace pointer is DEVICE
 * memory owned by the caller; the library never allocates or frees it.  Host
 * structs are borrowed for the duration of a call.  `stream` is a hipStream_t
 * (NULL = the default stream); device work is enqueued on it, and calls with
 * host outputs synchronise it before returning.
 *
 * Errors.  Every entry point returns a skyr_status.  Arguments are validated
 * before any device work: null required pointers, any n < 5, h <= 0, dt <= 0,
 * or a lattice whose component exceeds 2^31 sites give SKYR_E_INVAL with no
 * side effect.  HIP failures give SKYR_E_DEVICE.  skyr_last_error() returns a
 * thread-local message describing the last failure of the calling thread.
 * Calls are re-entrant on distinct buffers, workspaces and streams.
 */
#ifndef SKYR_H
#define SKYR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* exported symbols of libskyr.so */
#define SKYR_API __attribute__((visibility("default")))

typedef enum {
    SKYR_OK = 0,
    SKYR_E_INVAL = -1,     /* invalid argument; nothing was done            */
    SKYR_E_NOMEM = -2,     /* workspace too small / host allocation failed  */
    SKYR_E_DEVICE = -3,    /* a HIP call failed                              */
    SKYR_E_NONFINITE = -4, /* energy or force stopped being finite           */
    SKYR_E_BUSY = -5,      /* batch slot table full                          */
    SKYR_E_IO = -6         /* a file could not be opened, read or written    */
} skyr_status;

/* The precision crosses the ABI as an argument: in C++ its type has a fixed 32-bit
 * representation, so that every int32_t a caller passes is a value of it and an unknown
 * one can be checked and rejected (C enums are int-sized already). */
#ifdef __cplusplus
#define SKYR_ENUM_INT32 : int32_t
#else
#define SKYR_ENUM_INT32
#endif
typedef enum SKYR_ENUM_INT32 {
    SKYR_F64 = 0,      /* fields, velocities and stencils in double                        */
    SKYR_F32_BULK = 1  /* fields, velocities and stencils in float; energy and charge sums,
                          the arrest comparison and a periodic renormalisation in double  */
} skyr_precision;

/* Uniform cubic lattice (Sec. 3): n sites per axis (frozen layers included), spacing h. */
typedef struct {
    int32_t n[3];
    int32_t _pad;
    double h;
} skyr_lattice;

/* Model couplings (Sec. 2.1 and the program's four potentials and sextic term, Sec. 7.7),
 * in this library's energy normalisation (one half of the printed density):
 *   V(phi0) = m^2 (1 - phi0) + m_y^2 (1 - phi0^2)/2 + m_z^2 (1 - phi0)^2/2 + m_w^2 (1 - phi0)^4/4
 *   e6      = (c6 / 2) det[phi, a_1, a_2, a_3]^2        (a_i the derivatives of phi)
 * m is the rescaled pion mass (m = 2 m_pi / (F_pi e)); m_y, m_z, m_w are the modified
 * pion mass, loosely bound and lightly bound potential masses; c6 >= 0 weighs the sextic
 * (BPS-Skyrme) term, the squared baryon density up to (2 pi^2)^2.  0 = absent. */
typedef struct {
    double m;
    double m_y;
    double m_z;
    double m_w;
    double c6;
    int32_t form;  /* a skyr_gradient_form */
    int32_t _pad;
} skyr_model;

/* Form of the force (Sec. 3).
 *   SKYR_FORM_EXACT    the exact derivative of the discrete energy E_h (default;
 *                      the flow descends E_h and its fixed points are those of E_h)
 *   SKYR_FORM_PRINTED  the paper's printed Euler-Lagrange expression, halved, with
 *                      the five-point second difference and D_i D_j mixed
 *                      derivatives on every interior site (a one-stage stencil);
 *                      agrees with the exact form to O(h^4).  The energy, charge
 *                      and arrest test are unchanged.  Not available with the
 *                      sextic term (c6 != 0), in batches or for the autotuner. */
typedef enum { SKYR_FORM_EXACT = 0, SKYR_FORM_PRINTED = 1 } skyr_gradient_form;

/* Flow mode (Sec. 3; the program's flow modes, Sec. 7.5).
 *   SKYR_ARREST_ENERGY  arrested Newton flow with the paper's rule: arrest at step k
 *                       when E_k > E_{k-1} (strict; E_{-1} = +inf).
 *   SKYR_ARREST_POWER   arrested Newton flow, arresting when the power
 *                       P_k = h^3 sum_I F_k . v_k is negative (dE/dt = -F . v: the
 *                       instantaneous form of "the energy starts to rise").  P needs
 *                       no difference of two total energies; in single precision the
 *                       rounding noise of E_k exceeds the per-step energy decrease
 *                       well before the force reaches its floor, and the energy rule
 *                       then fires on noise.  Recommended with SKYR_F32_BULK.
 *   SKYR_NEWTON_FLOW    Newton flow: the same kick-drift steps, never arrested (it
 *                       does not converge to a minimum by itself).
 *   SKYR_GRADIENT_FLOW  first-order gradient flow phi_{k+1} = normalise(phi_k + dt F_k);
 *                       the velocity stays zero.
 * An arrest keeps phi_k and restarts from it with v_k = 0. */
typedef enum {
    SKYR_ARREST_ENERGY = 0,
    SKYR_ARREST_POWER = 1,
    SKYR_NEWTON_FLOW = 2,
    SKYR_GRADIENT_FLOW = 3
} skyr_flow_mode;

/* Flow controls (Sec. 3).
 *   dt             fictitious time step (kick-drift step; gradient flow: phi += dt F)
 *   tol            stop when max over I of |F| < tol, F the projected force
 *   max_steps      total cap on accepted steps across calls
 *   renorm64_every SKYR_F32_BULK only: every this many steps the renormalisation
 *                  phi <- phi/|phi| is done in double (0 = never; default 16)
 *   mode           a skyr_flow_mode (0 = arrested Newton flow, the paper's rule) */
typedef struct {
    double dt;
    double tol;
    int64_t max_steps;
    int32_t renorm64_every;
    int32_t mode;
} skyr_flow;

/* Initial data (Sec. 4). */
typedef enum {
    SKYR_INIT_HEDGEHOG = 0,       /* B = 1 at the origin, R(z) = z                           */
    SKYR_INIT_RATIONAL_MAP = 1,   /* c[0]: one rational map constituent                      */
    SKYR_INIT_PRODUCT = 2,        /* c[0..count): product ansatz, left to right               */
    SKYR_INIT_RANDOM_PRODUCT = 3  /* B unit charges drawn from `seed` (skyr_random_constituents) */
} skyr_init_kind;

/* One constituent of a product (Sec. 4.1, 4.2): the degree-`degree` rational
 * map R = p/q (p(z) = sum_k p[k] z^k, complex coefficients as (re, im)),
 * profile f(r) = prof_a exp(-r / prof_lambda), centre X, isorotation by the
 * unit quaternion quat = (a0, a1, a2, a3), A = a0 + i a.tau, U -> A U A^dagger,
 * and spatial orientation by the unit quaternion orient = B (Sec. 5.3): the
 * constituent is A U_R(D(B)^T (x - X)) A^dagger with D(B)_ij =
 * (1/2) Tr(tau^i B tau^j B^dagger), i.e. turned by the rotation D(B) about its
 * centre; orient = (0, 0, 0, 0) means no rotation. */
typedef struct {
    int32_t degree; /* 1..8 */
    int32_t _pad;
    double p[9][2];
    double q[9][2];
    double X[3];
    double quat[4];
    double prof_a;
    double prof_lambda;
    double orient[4];
} skyr_constituent;

typedef struct {
    int32_t kind;                /* skyr_init_kind                                          */
    int32_t count;               /* SKYR_INIT_PRODUCT: number of constituents in c (1..64)  */
    const skyr_constituent* c;   /* host array; RATIONAL_MAP uses c[0]                      */
    int32_t B;                   /* SKYR_INIT_RANDOM_PRODUCT: number of unit charges (1..64) */
    int32_t _pad;
    uint64_t seed;               /* SKYR_INIT_RANDOM_PRODUCT                                */
    double ball_radius;          /* SKYR_INIT_RANDOM_PRODUCT: centres uniform in this ball  */
    double prof_a;               /* HEDGEHOG, RANDOM_PRODUCT profile amplitude (pi)         */
    double prof_lambda;          /* HEDGEHOG, RANDOM_PRODUCT profile length                  */
} skyr_init_spec;

/* Observables (Sec. 2.1, 5.6): E = E2 + E4 + E0 + E6; B = h^3 sum_I b with
 * b = -(1/2 pi^2) det[phi, a_1, a_2, a_3] (the sign that gives the hedgehog with
 * f(0) = pi charge +1); virial = E2 - E4 + 3 E0 - 3 E6 (dE/dlambda under
 * x -> lambda x; zero for a Derrick-stationary field); max_force = max over I of
 * |F|, F = -(g - (g.phi) phi); E6 = the sextic energy (0 when c6 = 0). */
typedef struct {
    double E, E2, E4, E0, B, virial, max_force, E6;
} skyr_obs;

/* State of an arrested Newton flow, carried across skyr_anf_step calls.
 * Initialise with skyr_anf_state_init (E_prev = +inf, counters 0) and start
 * from zero velocity. */
typedef struct {
    int64_t steps;        /* accepted updates                                        */
    int64_t arrests;      /* velocity resets (E(phi_k) > E(phi_{k-1}))                */
    int64_t redo_sweeps;  /* sweeps recomputed with zero velocity after an arrest     */
    int64_t sweeps;       /* all sweeps run (accepted + redone + final check)         */
    double E_prev;        /* E(phi_{steps-1}); +inf before the first update           */
    double E;             /* energy of the field at the last evaluated sweep          */
    double max_force;     /* max |F| at the last evaluated sweep                      */
    int32_t converged;    /* 1 once max_force < tol; the returned field is that one   */
    int32_t redo_pending; /* the next sweep re-runs the last field with zero velocity */
    int32_t nonfinite;    /* 1 if E or max_force stopped being finite                  */
    int32_t _pad;
} skyr_anf_state;

/* Library version string. */
SKYR_API const char* skyr_version(void);

/* Thread-local description of the last error of the calling thread ("" if none). */
SKYR_API const char* skyr_last_error(void);

/* Bytes of device workspace needed by skyr_energy_gradient, skyr_anf_step,
 * skyr_observables and skyr_moments for this lattice and precision (0 on
 * invalid arguments).
 * The workspace holds the flow's control block and one block of partial sums
 * per thread block; it must be 256-byte aligned and not shared by calls that
 * overlap in time. */
SKYR_API size_t skyr_workspace_bytes(const skyr_lattice* lat, skyr_precision prec);

/* The B unit-charge constituents of SKYR_INIT_RANDOM_PRODUCT, drawn on the
 * host (smorgasbord-style data, Sec. 4.2): SplitMix64 (Steele, Lea, Flood 2014)
 * seeded with `seed`; per constituent, centre by rejection from the cube
 * [-R, R]^3 until |X| <= R (three uniforms per attempt), then a Haar-random
 * quaternion by Shoemake's method from three more uniforms,
 * (sqrt(1-u1) sin 2pi u2, sqrt(1-u1) cos 2pi u2, sqrt(u1) sin 2pi u3, sqrt(u1) cos 2pi u3);
 * uniforms are the top 53 bits times 2^-53.  out: host array of B entries. */
SKYR_API skyr_status skyr_random_constituents(uint64_t seed, int32_t B, double radius, double prof_a, double prof_lambda,
                                     skyr_constituent* out);

/* Orientation quaternion B for the Euler angles of the program's configuration
 * files (Sec. 7.3.1: a rotation about z, then about y, then about z, in radians):
 * D(B) = R_z(a[0]) R_y(a[1]) R_z(a[2]), with R_n(t) the right-handed rotation by
 * t about axis n and D as in skyr_constituent.  out: 4 doubles, b0 >= 0. */
SKYR_API void skyr_orientation_zyz(const double angles[3], double out[4]);

/* Fill phi (device, layout above) with initial data (Sec. 4): the product
 * U = prod_k A_k U_k(x - X_k) A_k^dagger (eq. Product ansatz) of rational-map
 * fields U_k = exp(i f(r) n_R . tau) (Sec. 4.1), evaluated in double and
 * rounded to the field precision; frozen layers set to vacuum.  Enqueued on
 * `stream`; returns without waiting. */
SKYR_API skyr_status skyr_init_field(const skyr_lattice* lat, skyr_precision prec, const skyr_init_spec* spec, void* phi,
                            void* stream);

/* Discrete gradient of E_h at phi (Sec. 3, eq. Newton_flow and the
 * Euler-Lagrange expression it projects; here the exact derivative of E_h).
 *   grad       nullable device output, layout of phi: g (projected = 0) or the
 *              tangential part g - (g.phi) phi (projected = 1); zero on the
 *              frozen layers
 *   parts      nullable host output: E, E2, E4, E0, virial and max_force
 *              (B is not computed here and is set to 0)
 *   work       device workspace of skyr_workspace_bytes(lat, prec) bytes
 * Synchronises `stream` when parts is non-null. */
SKYR_API skyr_status skyr_energy_gradient(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                 const void* phi, void* grad, int32_t projected, skyr_obs* parts, void* work,
                                 void* stream);

/* Reset a flow state: counters 0, E_prev = +inf, no redo pending. */
SKYR_API void skyr_anf_state_init(skyr_anf_state* st);

/* Advance the arrested Newton flow (Sec. 3) by up to nsteps accepted steps.
 * Step k, from (phi_k, v_k):
 *   E_k = E_h(phi_k); if E_k > E_{k-1} the velocity is reset (arrest, v_k := 0)
 *   F_k = -(g - (g.phi) phi); stop if max over I of |F_k| < tol
 *   v_{k+1} = v_k + dt F_k;  phi_{k+1} = (phi_k + dt v_{k+1}) / |phi_k + dt v_{k+1}|
 * The device evaluates E_k in the same sweep that computes the speculative
 * update; an arrest re-runs that sweep with v_k = 0, so the trajectory is the
 * one above.  Runs until st->steps reaches min(st->steps + nsteps,
 * flow->max_steps), convergence, or a non-finite value.
 *   phi      in/out; holds the result on return
 *   phi_alt  scratch field of the same size (its frozen layers are overwritten)
 *   vel      in/out velocity, same layout; zero at the start of a flow.  On
 *            return it is v_k, the velocity belonging to the returned phi_k,
 *            also after convergence: the sweep that finds max|F_k| < tol has
 *            already kicked vel to v_k + dt F_k in place, and one more sweep
 *            over phi_k writes (v_k + dt F_k) - dt F_k back (within one rounding
 *            of v_k; exactly zero when v_k was reset by an arrest)
 *   st       in/out state (skyr_anf_state_init before the first call)
 * Returns SKYR_E_NONFINITE if the energy or force stops being finite (field
 * contents then unspecified).  Synchronises `stream`. */
SKYR_API skyr_status skyr_anf_step(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                          const skyr_flow* flow, void* phi, void* phi_alt, void* vel, skyr_anf_state* st,
                          int64_t nsteps, void* work, void* stream);

/* skyr_anf_step for fields stored in padded rows with the four components of a
 * row one after the other (the layout of skyr_batch_add_padded: component A,
 * site (x, y, z) at element ((x n1 + y) 4 + A) pitch + lead + z; lead >= 0,
 * pitch >= lead + n2, the elements outside [lead, lead + n2) of a row finite
 * and never written; skyr_batch_layout gives lead and pitch that put the
 * first tile column on a 128-byte line).  phi, phi_alt and vel all take that
 * layout; the exact-gradient form only.  Results are bitwise those of
 * skyr_anf_step on the same field stored densely; on a lattice whose rows are
 * not whole 128-byte lines the sweep runs faster. */
SKYR_API skyr_status skyr_anf_step_padded(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                          const skyr_flow* flow, void* phi, void* phi_alt, void* vel,
                                          skyr_anf_state* st, int64_t nsteps, void* work, int32_t lead,
                                          int32_t pitch, void* stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses
 * that forbid hipMalloc / hipFree, callers without a workspace of their own):
 * skyr_anf_step with the same arguments except `work`.  The control block and
 * the per-block partial sums live in a fixed device array of
 * SKYR_NOALLOC_SCRATCH_BYTES inside the library, one per device (its address
 * is taken on the first call on a device, with that device current, and the
 * array is held until the process ends).  The call allocates nothing and runs
 * the same kernels as skyr_anf_step, so its results are the same bit for bit.
 * A flow whose sweep needs more workspace than the array holds (the control
 * block, 512 bytes of observables and 64 bytes per sweep block: room for 4084
 * blocks, which the default tiles of every lattice fit; a tile setting with
 * many short slabs on a large lattice may not) gives SKYR_E_INVAL before any
 * device work.  Every call on one
 * device shares that device's array and leaves its last contents there (each
 * call initialises what it reads): calls that overlap in time on one device,
 * from any stream or thread, race and give undefined results.  Synchronises
 * `stream`. */
#define SKYR_NOALLOC_SCRATCH_BYTES (1u << 18)
SKYR_API skyr_status skyr_anf_step_noalloc(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                           const skyr_flow* flow, void* phi, void* phi_alt, void* vel,
                                           skyr_anf_state* st, int64_t nsteps, void* stream);

/* ---- One block of a 3D block decomposition (the one-device share of a lattice that is
 * split over devices; Sec. 3 stencils) ----
 * The block owns the sites origin[d] .. origin[d] + extent[d] - 1 of the whole lattice
 * `lattice` (frozen layers included) and stores each of its fields padded: extent[d] + 8
 * sites per axis, in the field layout above, own site g at padded index g - origin + 4.
 * The shell four sites deep around the own box holds neighbouring blocks' sites: the
 * exact gradient at a site reads phi up to four sites away along the axes (the quartic
 * flux needs phi within two sites, its divergence the flux within two), so one exchange
 * of the shell per sweep is all a block needs from its neighbours.
 * Shell buffer: the shell's sites in the row-major order of the padded box with the own
 * box left out, component-major (4 x skyr_block_shell_sites elements of the field
 * precision): the data the neighbouring blocks send.  Entries for sites outside the
 * lattice are ignored; such shell sites are filled with the nearest lattice site, the
 * value a sweep over the whole lattice reads there. */
typedef struct {
    skyr_lattice lattice; /* the whole lattice */
    int32_t origin[3];    /* its site of the block's first own site, per axis */
    int32_t extent[3];    /* own sites per axis, >= 1; origin + extent <= lattice.n */
} skyr_block;

/* Sites per component of a padded block field, and of its shell (0 on an invalid block;
 * a padded block obeys the size limit of a lattice). */
SKYR_API int64_t skyr_block_sites(const skyr_block* blk);
SKYR_API int64_t skyr_block_shell_sites(const skyr_block* blk);

/* Bytes of device workspace skyr_block_sweep needs (0 on invalid arguments); 256-byte
 * aligned, not shared by calls that overlap in time. */
SKYR_API size_t skyr_block_workspace_bytes(const skyr_block* blk, skyr_precision prec);

/* The block's share of the sums of one sweep, over its own sites in I: added over all
 * blocks (maximum for max_force) they are the sums of the whole lattice. */
typedef struct {
    double E;         /* energy (both modes)                                        */
    double E2, E4, E0, E6; /* its parts (gradient mode; 0 in step mode)             */
    double power;     /* h^3 sum F . v of the incoming velocity (step mode)          */
    double max_force; /* max |F|                                                    */
} skyr_block_sums;

typedef enum { SKYR_BLOCK_GRADIENT = 0, SKYR_BLOCK_STEP = 1 } skyr_block_mode;

/* One sweep over the block's own sites in the lattice's interior I:
 *   1. the shell of phi is written from `shell` (as described above); the block's own
 *      sites of phi are only read;
 *   2. SKYR_BLOCK_GRADIENT: out = g, the exact gradient of E_h (skyr_energy_gradient's
 *      values, bit for bit), or its tangential part g - (g.phi) phi when projected != 0;
 *      SKYR_BLOCK_STEP: one kick-drift step of Sec. 3 from (phi, vel):
 *      vel <- v + dt F, out <- (phi + dt vel) / |phi + dt vel|, with v = 0 when
 *      redo != 0 (the restart after an arrest); renorm64 != 0 makes a SKYR_F32_BULK
 *      step normalise in double, as skyr_anf_step does every renorm64_every steps (it is
 *      ignored for SKYR_F64, which computes in double throughout).  The values are those
 *      of the corresponding step of skyr_anf_step, bit for bit.  The flow's
 *      decision (arrest, convergence) belongs to the caller, from every block's sums.
 * out and vel are padded block fields written (and vel read) at the block's own sites
 * in I only; the model must use the exact form.
 *   sums   nullable host output; the call synchronises `stream` when it is non-null
 *   work   device workspace of skyr_block_workspace_bytes(blk, prec) bytes
 * A block with no site in I does nothing (sums zero). */
SKYR_API skyr_status skyr_block_sweep(const skyr_block* blk, skyr_precision prec, const skyr_model* model,
                                      int32_t mode, int32_t projected, double dt, int32_t redo, int32_t renorm64,
                                      void* phi, const void* shell, void* out, void* vel, skyr_block_sums* sums,
                                      void* work, void* stream);

/* The block sweep on block fields stored in padded rows with the four components
 * of a row one after the other: component A at padded site (x, y, z) (the
 * indices of skyr_block_sites' box, P0 x P1 x P2) at element
 * ((x P1 + y) 4 + A) pitch + lead + z, with lead >= 0 and pitch >= lead + P2
 * (4 P0 P1 pitch elements within 4 GiB).  phi, out and vel take that layout;
 * the shell buffer is as for skyr_block_sweep.  The elements outside
 * [lead, lead + P2) of a row must be finite (zero, for instance) and are never
 * written.  Results are bitwise those of skyr_block_sweep.  skyr_block_layout
 * gives a lead and pitch that put the first tile column of the block's sweep on
 * a 128-byte line, rows of whole lines (the padded rows of P2 = extent + 8
 * elements otherwise straddle lines). */
SKYR_API skyr_status skyr_block_sweep_padded(const skyr_block* blk, skyr_precision prec, const skyr_model* model,
                                             int32_t mode, int32_t projected, double dt, int32_t redo,
                                             int32_t renorm64, void* phi, const void* shell, void* out, void* vel,
                                             skyr_block_sums* sums, void* work, int32_t lead, int32_t pitch,
                                             void* stream);
SKYR_API skyr_status skyr_block_layout(const skyr_block* blk, skyr_precision prec, int32_t* lead, int32_t* pitch);

/* Energy parts, baryon number, virial and largest projected force of phi
 * (Sec. 2.1 eq. B0_components, Sec. 5.6 eq. Virial).  Synchronises `stream`. */
SKYR_API skyr_status skyr_observables(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                             const void* phi, skyr_obs* out, void* work, void* stream);

/* Kinetic energy of a flow's velocity field (Sec. 3: the quantity whose growth
 * the arrest criterion watches), T = (1/2) h^3 sum over I of |v|^2, in this
 * library's normalisation (one half of the printed one, like skyr_obs.E).
 * vel: device field of precision prec; out: host double.  FP64 sums in a
 * fixed order.  Synchronises `stream`. */
SKYR_API skyr_status skyr_kinetic_energy(const skyr_lattice* lat, skyr_precision prec, const void* vel, double* out,
                                         void* work, void* stream);

/* Moment observables of a field (Sec. 5), in the printed (un-halved)
 * normalisation of the Lagrangian, integrals as h^3 sums over the interior I
 * with a_i the fourth-order first differences, coordinates x = (idx - (n-1)/2) h:
 *   B       h^3 sum b (charge density b as in skyr_obs)
 *   E       the total static energy in the printed normalisation (2 x skyr_obs.E)
 *   X       centre of mass, (1/B) h^3 sum x b (eq. CoM); r = x - X below
 *   R       RMS radius, ((1/B) h^3 sum |r|^2 b)^(1/2) (eq. RMS radius)
 *   U, V, W isospin, spin and mixed inertia tensors (eqs. U, V, W inertia tensor),
 *           with L_i = U^dagger d_i U, T_j = (i/2) U^dagger [tau^j, U]; row-major
 *   Q       isospin-0 quadrupole, rho = b/2 (eq. Q tensor); row-major
 *   D       monopole D-term (eq. D-term) with the static stress tensor of eq. Stress tensor
 * The tensors contain the quadratic and quartic terms of the printed formulas
 * only (the sextic term and potentials of Sec. 7.7 do not enter them). */
typedef struct {
    double B, E;
    double X[3];
    double R;
    double U[9], V[9], W[9], Q[9];
    double D;
} skyr_moment_obs;

/* Compute skyr_moment_obs of phi: one observables sweep for E, then two FP64
 * passes over I (the charge and its first moments, then the tensor densities in
 * the centre-of-mass frame), reduced in a fixed order on the device.
 *   work  device workspace of skyr_workspace_bytes(lat, prec) bytes
 * Returns SKYR_E_NONFINITE, with *out filled, when |B| < 1e-6 (no centre of
 * mass) or a result is not finite.  Synchronises `stream`. */
SKYR_API skyr_status skyr_moments(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                  const void* phi, skyr_moment_obs* out, void* work, void* stream);

/* Batches: many independent flows (uneven lattices, charges, masses and
 * precisions) advanced together.  Fields of one precision and tile shape share
 * a kernel and form one chain; per sweep slot a chain is one launch over its
 * fields' tiles, whose blocks also take each field's flow decision (the last
 * block of a field to finish reads its partial sums).  The launch's blocks are
 * laid out for the device: a field's blocks in pieces of at most one XCD's
 * compute units, the pieces spread over the XCDs by estimated work and the
 * longest blocks dispatched first.  Chains share no field: skyr_batch_run
 * replays a captured hipGraph of `sweeps` slots that runs the chains as
 * independent branches.  A field's blocks, partial sums and decisions are
 * those of the same field flowing alone with its lattice's batch tile (see
 * skyr_get_batch_tile), so a field's result does not depend on the other
 * fields in the batch, and equals that of skyr_anf_step when skyr_set_tile
 * gives the lattice the same tile.  A batch object owns only its job table,
 * control blocks and graph; field, velocity and workspace memory stay with
 * the caller and must stay valid while the field is in the batch.  A batch is
 * used by one thread at a time.
 *   skyr_batch_create  max_jobs slots; work is enqueued on `stream`
 *   skyr_batch_add     a fresh flow (state as after skyr_anf_state_init, zero
 *                      velocity); runs until max|F| < flow->tol or
 *                      flow->max_steps accepted steps; returns its slot
 *   skyr_batch_run     `sweeps` sweep slots for every active field; waits for
 *                      them; SKYR_E_BUSY never; errors as skyr_anf_step
 *   skyr_batch_poll    state of a slot after the last run; once the field has
 *                      stopped, its result is (copied if needed) in phi
 *   skyr_batch_remove  frees the slot (phi then holds the field's last state)
 *   skyr_batch_active  number of occupied slots */
typedef struct skyr_batch skyr_batch;
SKYR_API skyr_status skyr_batch_create(int32_t max_jobs, void* stream, skyr_batch** out);
SKYR_API skyr_status skyr_batch_add(skyr_batch* b, const skyr_lattice* lat, skyr_precision prec,
                                    const skyr_model* model, const skyr_flow* flow, void* phi, void* phi_alt,
                                    void* vel, void* work, int32_t* slot);

/* Padded rows for batch fields.  A field whose rows are not whole 128-byte
 * lines (n2 x element size) has its tiles' rows straddle lines, which costs
 * the sweep up to a quarter of its speed; and the four component arrays of a
 * field are four separate memory streams.  skyr_batch_layout gives a layout of
 * phi, phi_alt and vel in which the four components of a lattice row follow
 * each other, each padded so that the first tile column of the lattice's
 * batch tile starts a line: component A, site (x, y, z) at element
 * ((x n1 + y) 4 + A) pitch + lead + z, with lead < 128 bytes and pitch the
 * least whole number of lines >= lead + n2 (a tensor of shape
 * (n0, n1, 4, pitch)).  skyr_batch_add_padded takes fields in any such layout
 * (lead >= 0, pitch >= lead + n2, 4 n0 n1 pitch elements within 4 GiB; the
 * elements outside [lead, lead + n2) of a row must be finite, zero for
 * instance, and are never written); it is skyr_batch_add otherwise, and a
 * field's results are bitwise those of the same field stored densely.
 * skyr_anf_step_padded is the single-field flow on such fields; the other
 * entry points take dense fields only. */
SKYR_API skyr_status skyr_batch_layout(const skyr_lattice* lat, skyr_precision prec, int32_t* lead, int32_t* pitch);
SKYR_API skyr_status skyr_batch_add_padded(skyr_batch* b, const skyr_lattice* lat, skyr_precision prec,
                                           const skyr_model* model, const skyr_flow* flow, void* phi,
                                           void* phi_alt, void* vel, void* work, int32_t lead, int32_t pitch,
                                           int32_t* slot);
SKYR_API skyr_status skyr_batch_run(skyr_batch* b, int32_t sweeps);
SKYR_API skyr_status skyr_batch_poll(skyr_batch* b, int32_t slot, skyr_anf_state* st);
SKYR_API skyr_status skyr_batch_remove(skyr_batch* b, int32_t slot);
SKYR_API int32_t skyr_batch_active(const skyr_batch* b);
SKYR_API skyr_status skyr_batch_destroy(skyr_batch* b);

/* Tile shapes of the fused sweep.  A few shapes (interior waves, halo waves,
 * halo positions per halo lane, output columns) are compiled per precision;
 * skyr_tile_variant_info gives a shape's threads per block and its output
 * rows and columns.  x is cut into slabs of `xchunk` (>= 16) planes and one
 * block marches one (y, z) tile of one slab.  The choice is kept per (lattice
 * dimensions, precision) for the whole process and applies to every later
 * sweep on such a lattice; results are deterministic for a given choice.
 * Default for a field flowing alone (a lattice never set or tuned): the shape
 * and even split of x into 1..8 slabs of least estimated time, that is the
 * rounds of the device its blocks take times the padded work of one block,
 * each shape priced by a factor measured at 256^3.  Fields in batches have a
 * tile setting of their own (skyr_set_batch_tile, skyr_batch_autotune) whose
 * default is the precision's first shape (variant 0: the fields of one
 * precision then share one launch per sweep slot) with x split evenly into the
 * fewest slabs of at most 64 planes: in a batch the other fields fill the
 * device.  The getters report the setting in force, the default included. */
SKYR_API int32_t skyr_tile_variants(skyr_precision prec);
SKYR_API skyr_status skyr_tile_variant_info(skyr_precision prec, int32_t variant, int32_t info[3]);
SKYR_API skyr_status skyr_set_tile(const skyr_lattice* lat, skyr_precision prec, int32_t variant, int32_t xchunk);
SKYR_API skyr_status skyr_get_tile(const skyr_lattice* lat, skyr_precision prec, int32_t* variant, int32_t* xchunk);
SKYR_API skyr_status skyr_set_batch_tile(const skyr_lattice* lat, skyr_precision prec, int32_t variant,
                                         int32_t xchunk);
SKYR_API skyr_status skyr_get_batch_tile(const skyr_lattice* lat, skyr_precision prec, int32_t* variant,
                                         int32_t* xchunk);

/* Autotuner: time every compiled shape with the slab lengths that split the
 * interior x-extent evenly into 1..8 slabs (at least 16 planes each) on this
 * lattice (flow sweeps, phi read, phi_alt and vel written; a candidate's time
 * is the median of five sweeps; the four fastest and the default choice are
 * then timed in three more interleaved rounds, and a finalist's time is the
 * median of its rounds), keep the fastest finalist with skyr_set_tile -- the
 * default choice unless the fastest beats it by 3% or more, about the spread
 * of such timings between runs -- and return it
 * (outputs nullable; best_us is its sweep time in microseconds).  phi is
 * unchanged; phi_alt is scratch and vel is zero on return.  Synchronises
 * `stream`. */
SKYR_API skyr_status skyr_autotune(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                   const skyr_flow* flow, const void* phi, void* phi_alt, void* vel, void* work,
                                   void* stream, int32_t* variant, int32_t* xchunk, double* best_us);

/* Batch autotuner: the slab length of fields on this lattice in batches.
 * `copies` independent fields (arrays of `copies` device pointers: phi[i]
 * initial data, phi_alt[i] and vel[i] field-sized, work[i] of
 * skyr_workspace_bytes; dense when pitch = 0, else in the padded,
 * row-interleaved layout (lead, pitch) of skyr_batch_add_padded, the padding
 * zero) run together in
 * one batch for each even split of x
 * into 1..8 slabs (at least 16 planes each), with the batch shape (variant 0,
 * which keeps a precision's fields in one launch): four sweep slots, then
 * three timed runs of six slots each; a candidate's time per slot is the
 * median of its runs.  The fastest is kept with skyr_set_batch_tile -- the batch default
 * unless the fastest beats it by 3% or more -- and returned (outputs nullable;
 * best_us is its time per sweep slot of the whole batch, in microseconds).  The
 * flows run with no tolerance and no step limit, so phi[i] and phi_alt[i] end
 * with unspecified (advanced) fields and vel[i] zero: pass scratch copies.
 * Give enough copies that their blocks fill the device several times over.
 * Synchronises `stream`. */
SKYR_API skyr_status skyr_batch_autotune(const skyr_lattice* lat, skyr_precision prec, const skyr_model* model,
                                         const skyr_flow* flow, int32_t copies, void* const* phi,
                                         void* const* phi_alt, void* const* vel, void* const* work, int32_t lead,
                                         int32_t pitch, void* stream, int32_t* variant, int32_t* xchunk,
                                         double* best_us);

/* Kernel timing for measurement tools.  skyr_timing_enable(1) resets and
 * starts recording a pair of HIP events around every sweep-kernel launch made
 * by skyr_anf_step and skyr_block_sweep on the calling thread (on the caller's
 * stream; skyr_anf_step then launches every sweep directly instead of replaying
 * graphs); (0) stops.  skyr_timing_read waits for the launches recorded so far
 * and returns their summed event time in milliseconds and their count (either
 * pointer may be null). */
SKYR_API void skyr_timing_enable(int32_t on);
SKYR_API skyr_status skyr_timing_read(double* sweep_ms, int64_t* sweep_launches);

/* Field files in the program's two formats (Sec. 7.4).
 *   SKYR_FILE_BINARY  (int32) 1234, (double) xmin, ymin, zmin, (int32) XLEN, YLEN, ZLEN,
 *                     (double) m.x, m.y, m.z, m.w, (double) c6, (double) -123456789.0
 *                     (sentinel), then the field as XLEN*YLEN*ZLEN records of four
 *                     doubles (phi0..phi3), z fastest, then y, then x; little-endian,
 *                     fields written one after another without padding (88 header bytes)
 *   SKYR_FILE_TEXT    a header line of the eleven parameters above (from xmin to c6,
 *                     tab-separated), then one line of four tab-separated numbers per
 *                     site in the same order; doubles printed with 17 significant digits
 * A lattice of n sites and spacing h spans [xmin, -xmin] with xmin = -(n-1) h / 2 on
 * every axis; m.x..m.w and c6 are skyr_model's m, m_y, m_z, m_w, c6.  Reading
 * detects the format from the leading 1234, skips extra parameters that a
 * modified program stores before the sentinel (at most 64), checks that the
 * file's lattice equals `lat` (SKYR_E_INVAL otherwise; the spacing to 1e-12
 * relative, the same on all three axes) and fills model_out (nullable; form = 0).
 * I/O failures and malformed files give SKYR_E_IO. */
typedef enum { SKYR_FILE_BINARY = 0, SKYR_FILE_TEXT = 1 } skyr_file_format;

/* Host-memory variants: phi is a host array of 4 * N3 doubles in this library's
 * layout ([4][n0][n1][n2]). */
SKYR_API skyr_status skyr_write_field_host(const char* path, int32_t format, const skyr_lattice* lat,
                                           const skyr_model* model, const double* phi);
SKYR_API skyr_status skyr_read_field_host(const char* path, const skyr_lattice* lat, skyr_model* model_out,
                                          double* phi);

/* The lattice and model stored in a field file (either format), for sizing
 * buffers before skyr_load_field; lat_out and model_out nullable. */
SKYR_API skyr_status skyr_file_info(const char* path, skyr_lattice* lat_out, skyr_model* model_out);

/* Device variants: phi is a device field of precision prec (layout above);
 * the field goes through a host buffer (allocated and freed by the call).
 * Synchronise `stream`. */
SKYR_API skyr_status skyr_save_field(const char* path, int32_t format, const skyr_lattice* lat, skyr_precision prec,
                                     const skyr_model* model, const void* phi, void* stream);
SKYR_API skyr_status skyr_load_field(const char* path, const skyr_lattice* lat, skyr_precision prec,
                                     skyr_model* model_out, void* phi, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SKYR_H */

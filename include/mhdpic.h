/*
 * mhdpic.h -- C ABI of the MI355X cosmic-ray particle step of the MHD-PIC
 * method (Bai, Caprioli, Sironi & Spitkovsky 2015).
 *
 * One call of mhdpic_step advances every CR particle by one or more steps
 * through fields held fixed during the call:
 *   - gather: the cell-centred B and E = E0 - F_CR/n_g (E0 = -v_g x B, the
 *     CR-Hall correction of Sec. 2.1, eq. emfcr2, optional) are interpolated to
 *     the particle at x^(n+1/2) with TSC (quadratic-spline) weights (Sec. 3);
 *   - push: drift-kick-rotate-kick-drift relativistic Boris step at the
 *     reduced speed of light C, with the parallel electric field removed at
 *     the particle (App. A.2);
 *   - deposit: -dM = -m(v^(n+1)-v^(n)) and -dE_k = -m(E_k^(n+1)-E_k^(n)) at
 *     x^(n+1/2) (App. A.3, corrector), and n_CR = (q/mc) m, J_CR = (q/mc) m u
 *     at x^(n+1) (App. A.1 eq. nJCR; the predictor input of the next step).
 *
 * Deposits are exact 64-bit fixed-point amounts in units of 2^-frac_bits:
 * a stencil cell k other than the particle's own receives
 * round-half-even(W_k * V) of the exact product, and the particle's own cell
 * receives round-half-even(V) minus the others, so sums are exact and do not
 * depend on the order in which particles are processed.  Integers wrap
 * modulo 2^64.  Divide an amount by 2^frac_bits and by the cell volume to get
 * a density.
 *
 * Conventions for every entry point:
 *   - Array pointers named "device" are HIP device pointers.  Arrays are
 *     structure-of-arrays with the component outermost: a [3][N] array holds
 *     all x-components, then y, then z.  Grid arrays are [comp][cells] with the
 *     cells of box 0 first, then box 1, ...; within a box x is fastest:
 *     cell = (iz*ny + iy)*nx + ix.  Particle arrays hold box 0's particles
 *     first, then box 1's, ...
 *   - The caller owns all memory, including the workspace.  The library keeps
 *     only descriptors into it; the workspace must stay allocated and untouched
 *     until mhdpic_destroy.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it and the call returns without waiting, except where a
 *     function says otherwise.  Inputs must stay valid until the stream has
 *     passed the call's work.
 *   - Errors are returned as the codes below; nothing is thrown across the
 *     ABI.  mhdpic_last_error() gives a message for the last failure of the
 *     calling thread.  A condition found by a kernel (non-finite velocity,
 *     an amount too large for the fixed point) is latched on the device and
 *     returned by mhdpic_check, or by the next mhdpic_step once the earlier
 *     work has finished.
 */
#ifndef MHDPIC_H
#define MHDPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MHDPIC_OK = 0,
    MHDPIC_EINVAL = -1,     /* bad argument */
    MHDPIC_ENOMEM = -2,     /* workspace too small */
    MHDPIC_EDEVICE = -3,    /* a HIP call failed */
    MHDPIC_ERANGE = -4,     /* time step over the move limit, a deposit amount
                               |V| >= 2^51 quanta, a position whose (x-x0)/dx lies
                               outside [-2^31, 2^31), or a grid/particle count
                               beyond the library's index limits */
    MHDPIC_ENONFINITE = -5, /* a position or velocity is not finite */
    MHDPIC_ESTATE = -6,     /* internal consistency check failed */
    MHDPIC_ENOTSUP = -7     /* a configuration the compiled library does not cover */
};

enum { MHDPIC_FP64 = 0, MHDPIC_FP32_MIXED = 1 };

/* Particle boundary of one face of a box (Sec. 5: a conducting wall at x = 0
 * and an inflow boundary at x = L_x; periodic otherwise).  A particle that
 * crosses a reflecting face in a half drift is mirrored back (its offset and
 * that axis's velocity change sign; one landing exactly on the upper face
 * stays at the largest offset below 1/2 of the last cell); one that crosses
 * an absorbing face leaves the box (crossed in the first half drift it
 * deposits nothing, in the second it deposits -dM, -dE_k but no n_CR,
 * J_CR).  Stencil cells beyond a non-periodic face are their mirror images
 * inside (cell -1-k is cell k, cell n+k is cell n-1-k), for gathers and
 * deposits alike. */
enum { MHDPIC_PERIODIC = 0, MHDPIC_REFLECT = 1, MHDPIC_ABSORB = 2 };

/* One box of the grid (units: the paper's code units, Sec. 5). */
typedef struct {
    int32_t ndim;           /* 2 or 3; every box of one context has the same ndim */
    int32_t n[3];           /* cells per dimension; n[2] must be 1 in 2D.
                               Limits: 3D nx,ny <= 2048, nz <= 1024; 2D nx,ny <= 65536 */
    double dx[3];           /* cell size per dimension (> 0) */
    double x0[3];           /* lower corner */
    double C;               /* reduced particle speed of light (Sec. 2.2), > 0 */
    double qomc_gas;        /* (q/mc)_g of the gas ions: n_g = qomc_gas * rho (App. A.1, eq. ng) */
    int32_t hall;           /* 1: E = E0 - F_CR/n_g (Sec. 2.1, eq. emfcr2); 0: E = E0 */
    int32_t frac_bits;      /* fixed-point quantum 2^-frac_bits, 0..60 (40 is the usual value) */
    int32_t max_move_cells; /* 1 or 2: a particle crosses at most this many cells per step
                               (App. A.4); mhdpic_step rejects C*|dt|/dx above it */
    int32_t tile[3];        /* cells per tile per dimension for the LDS-staged kernels
                               (the boxes of one context may differ);
                               0 = library default (2D: 32x16; 3D: 8x4x4, or
                               4x4x4 for a box given 24 or more particles per
                               cell).  tile[2] is ignored in 2D */
    int32_t boundary[3][2]; /* per axis, low and high face: MHDPIC_PERIODIC (both faces or
                               neither), MHDPIC_REFLECT or MHDPIC_ABSORB; all zero =
                               periodic.  A non-periodic axis needs at least 2 cells */
    int64_t capacity;       /* particle slots reserved for this box, for mhdpic_inject;
                               0 or less than its initial count: the initial count */
} mhdpic_box;

typedef struct mhdpic_ctx mhdpic_ctx;

/* Bytes of device workspace a context needs for these boxes, particle counts
 * (n_particles[b] for box b) and precision (MHDPIC_FP64 or MHDPIC_FP32_MIXED). */
int mhdpic_workspace_size(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                          int32_t precision, size_t* bytes);

/* Creates a context: converts the particles' global positions to (cell index,
 * offset from the cell centre) form, and deposits n_CR and J_CR at the initial
 * positions (App. A.3 predictor).  The accumulated -dM, -dE_k start at zero.
 *   x, v   device, [3][N] doubles: global positions (2D ignores z) and spatial
 *          four-velocities v = gamma*u (Sec. 2.2, eq. 4vel)
 *   m, qm  device, [N] doubles: the CR mass carried by each particle and its
 *          (q/mc) (App. A.1)
 *   workspace  device, at least mhdpic_workspace_size bytes, 256-byte aligned
 * N is the sum of n_particles.  The call waits for the stream before it
 * returns (it checks the converted input). */
int mhdpic_init(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                int32_t precision, const double* x, const double* v, const double* m,
                const double* qm, void* workspace, size_t ws_bytes, void* hip_stream,
                mhdpic_ctx** out);

/* One call without a context: the particles of mhdpic_init are set up in
 * `workspace` (at least mhdpic_workspace_size bytes for the same boxes,
 * counts and precision, 256-byte aligned), advanced n_steps steps of n_sub
 * particle sub-steps each through fixed fields as mhdpic_step_sub does, and
 * written back; nothing is kept after the call.  The same results, bit for
 * bit, as mhdpic_init + mhdpic_step_sub + mhdpic_particles_read +
 * mhdpic_deposit_read on a new context.
 *   x, v, m, qm      device inputs as for mhdpic_init
 *   B, vg, rho, dt   fields and host time steps as for mhdpic_step
 *   n_steps >= 0, 1 <= n_sub <= 1024
 *   x_out, v_out     device, [3][N] doubles: final global positions and
 *                    four-velocities, in the input particle order
 *   deposits_out     device, [8][cells] int64: n_CR, J_CR at the final
 *                    positions, then -dM, -dE_k accumulated over the call
 * The workspace is scratch: its contents are undefined afterwards and it may
 * be reused as soon as the call returns.  Waits for the stream; device
 * errors (ENONFINITE, ERANGE) are returned by this call.  Other errors as for
 * mhdpic_init and mhdpic_step. */
int mhdpic_advance(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                   int32_t precision, const double* x, const double* v, const double* m,
                   const double* qm, const double* B, const double* vg, const double* rho,
                   const double* dt, int32_t n_steps, int32_t n_sub, double* x_out, double* v_out,
                   int64_t* deposits_out, void* workspace, size_t ws_bytes, void* hip_stream);

/* mhdpic_advance for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments without the workspace, and the same results bit for
 * bit.  The call's scratch is a static device array of 64 MiB per GPU, held
 * from the library's first use on that GPU until the process ends; the call
 * itself calls no allocating routine.  Boxes and particles whose workspace
 * (mhdpic_workspace_size) exceeds 64 MiB are rejected with MHDPIC_ENOMEM
 * before any device work.  Every call on one GPU uses the same scratch, so
 * calls that overlap on one GPU (other threads, other streams) race: the
 * caller must serialise them.  Waits for the stream. */
int mhdpic_advance_noalloc(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                           int32_t precision, const double* x, const double* v, const double* m,
                           const double* qm, const double* B, const double* vg, const double* rho,
                           const double* dt, int32_t n_steps, int32_t n_sub, double* x_out,
                           double* v_out, int64_t* deposits_out, void* hip_stream);

/* Advances all particles n_steps steps (App. A.2, A.3) through fixed fields.
 * Waits for the stream only when dt differs from the previous call (the new
 * step constants are uploaded).  The call may be captured into a HIP graph if
 * dt equals the previous call's and n_steps is even, so that each replay
 * leaves the context's buffers as it found them; calls made between replays
 * of such a graph must keep n_steps even for the same reason (see also
 * mhdpic_step_graph, which tracks this itself).
 *   B, vg  device, [3][cells] doubles: cell-centred magnetic field and gas velocity
 *   rho    device, [cells] doubles: gas density (read only where hall = 1)
 *   dt     host, [n_boxes] doubles: time step of each box (may be negative)
 * Before each step the cell-centred E is formed from the current n_CR, J_CR
 * (Sec. 2.1); -dM and -dE_k accumulate over steps; n_CR and J_CR are replaced
 * by their values at the new positions.  Returns MHDPIC_ERANGE if
 * C*|dt|/dx > max_move_cells for any box.  Does not wait for the stream. */
int mhdpic_step(mhdpic_ctx* ctx, const double* B, const double* vg, const double* rho,
                const double* dt, int32_t n_steps, void* hip_stream);

/* mhdpic_step with particle sub-cycling (App. A, "Timestepping and Code
 * Performance"): each of the n_steps steps of dt forms the cell-centred E
 * once, from the n_CR, J_CR present at its start, and then advances the
 * particles n_sub times by dt/n_sub with that E and the given B.  -dM and
 * -dE_k of every sub-step accumulate; n_CR and J_CR are deposited only after
 * the last sub-step, at the particles' final positions.  n_sub = 1 is
 * mhdpic_step.  1 <= n_sub <= 1024, else MHDPIC_EINVAL; the move limit
 * applies to C*|dt/n_sub|/dx.  Other arguments and waits as for mhdpic_step. */
int mhdpic_step_sub(mhdpic_ctx* ctx, const double* B, const double* vg, const double* rho,
                    const double* dt, int32_t n_steps, int32_t n_sub, void* hip_stream);

/* Cell-centred CR feedback of the predictor step (App. A.3: computed at cell
 * centres from the n_CR, J_CR deposited at the particles' current positions,
 * R from the gas density, E0 = -v_g x B and B).  Code units: c = 1 and no
 * factors of 4 pi (as in App. B); n_CR = D0 2^-frac_bits / dV, J_CR likewise.
 *   B, vg  device, [3][cells] doubles; rho device, [cells] doubles, > 0
 *   out    device, [10][cells] doubles, written:
 *     0-2  -F_CR, F_CR = (1-R)(n_CR E0 + J_CR x B)   (Sec. 2.2 eq. lorentz2): the
 *          momentum source of the gas (eq. gasmotion)
 *     3    -(1-R) J_CR . E0 = -v_g . F_CR (eqs. engeq, eng): its energy source
 *     4-6  (E - E0) x B with E = E0 - F_CR/n_g (eq. emfcr2): the CR-Hall part
 *          of the energy flux (eq. engeq; times c/4pi in Gaussian units)
 *     7-9  Lambda = R (u_CR - v_g) / v_A, u_CR = J_CR/n_CR, v_A = |B|/sqrt(rho)
 *          (eq. lambda); 0 where n_CR = 0 or B = 0
 * R = n_CR/(n_g + n_CR), n_g = qomc_gas rho.  In a box with hall = 0, R is
 * taken as 0 in channels 0-6 (the particles feel E0), so 4-6 are 0; Lambda
 * keeps the physical R.  Enqueued on the stream; does not wait. */
int mhdpic_feedback(mhdpic_ctx* ctx, const double* B, const double* vg, const double* rho,
                    double* out, void* hip_stream);

/* mhdpic_step through a HIP graph.  The first call (and any call whose
 * B, vg, rho, dt or n_steps differ from the cached ones, or that finds the
 * context's buffers in another state than at capture) captures the n_steps
 * steps into a graph owned by the context; every call then launches that
 * graph, so one launch advances all boxes n_steps steps.  n_steps must be even
 * (the step's buffer swaps then return to the captured state after each
 * launch) and hip_stream must not be the default stream.  Waits for the stream
 * when it captures.  Does not wait otherwise. */
int mhdpic_step_graph(mhdpic_ctx* ctx, const double* B, const double* vg, const double* rho,
                      const double* dt, int32_t n_steps, void* hip_stream);

/* mhdpic_step_graph with particle sub-cycling (see mhdpic_step_sub): each of
 * the n_steps steps (n_steps even) takes n_sub particle steps of dt/n_sub.
 * The cached graph is also recaptured when n_sub changes, or when eager calls
 * in between left the context's buffers in another state. */
int mhdpic_step_graph_sub(mhdpic_ctx* ctx, const double* B, const double* vg, const double* rho,
                          const double* dt, int32_t n_steps, int32_t n_sub, void* hip_stream);

/* Picks the tile shape (cells per tile, the LDS staging unit of the push
 * kernel) with the shortest step time for this workload: for every compiled
 * shape it builds a context in `workspace` from the given particles, runs two
 * warm-up steps and times n_steps steps with HIP events.  Arguments as for
 * mhdpic_init and mhdpic_step (the particle arrays are read, not changed);
 * workspace needs mhdpic_autotune_workspace_size bytes.  Writes the shape to
 * tile_out[3] (use it as mhdpic_box.tile) and, if not NULL, its time per step
 * in ms.  Waits for the stream. */
int mhdpic_autotune_workspace_size(const mhdpic_box* boxes, int32_t n_boxes,
                                   const int64_t* n_particles, int32_t precision, size_t* bytes);
int mhdpic_autotune(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                    int32_t precision, const double* x, const double* v, const double* m,
                    const double* qm, const double* B, const double* vg, const double* rho,
                    const double* dt, int32_t n_steps, void* workspace, size_t ws_bytes,
                    void* hip_stream, int32_t* tile_out, double* ms_per_step);

/* The batched form's autotuner (the independent boxes of uneven size of the
 * batching workload): a tile shape per box-size class.  The tile is both the
 * unit the binning sorts particles into and the LDS staging unit of the push,
 * so one shape sets both.  A box's size class is k for 4^k <= its cell count <
 * 4^(k+1).  For every compiled shape it times n_steps steps of a context in
 * which all boxes take that shape, with the push launched once per size
 * class, and takes for each class the shape of the shortest push.  The mix is
 * then timed as a whole and kept only if its step is shorter than that of the
 * best single shape (which is used for all boxes otherwise).  Boxes of one
 * context may have different tile shapes (mhdpic_box.tile); each shape is one
 * push launch per step.  Arguments as for mhdpic_autotune; workspace needs
 * mhdpic_autotune_classes_workspace_size bytes.  Writes the shape of box b to
 * tiles_out[3b .. 3b+2] and, if not NULL, the chosen step time in ms.  Waits
 * for the stream. */
int mhdpic_autotune_classes_workspace_size(const mhdpic_box* boxes, int32_t n_boxes,
                                           const int64_t* n_particles, int32_t precision,
                                           size_t* bytes);
int mhdpic_autotune_classes(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                            int32_t precision, const double* x, const double* v, const double* m,
                            const double* qm, const double* B, const double* vg, const double* rho,
                            const double* dt, int32_t n_steps, void* workspace, size_t ws_bytes,
                            void* hip_stream, int32_t* tiles_out, double* ms_per_step);

/* Copies the deposits to out (device, [8][cells] int64): channels
 * 0..3 = n_CR, J_CR x,y,z at the current positions; 4..6 = accumulated
 * -dM x,y,z; 7 = accumulated -dE_k.  If reset_accumulated is nonzero,
 * channels 4..7 are cleared after the copy.  Does not wait. */
int mhdpic_deposit_read(mhdpic_ctx* ctx, int64_t* out, int32_t reset_accumulated,
                        void* hip_stream);

/* Copies particle states to x, v (device, [3][N] doubles, N the particles
 * given to mhdpic_init) in the original particle order: global positions
 * x0 + dx*((i + 1/2) + offset) (z = 0 in 2D) and four-velocities.  Columns
 * of particles that have left their box (absorbing faces, mhdpic_remove_tagged)
 * read NaN.  MHDPIC_ESTATE once particles were added (mhdpic_inject): use
 * mhdpic_particles_read_ids.  Does not wait. */
int mhdpic_particles_read(mhdpic_ctx* ctx, double* x, double* v, void* hip_stream);

/* Particles in their boxes (Sec. 5 runs add and remove particles): writes
 * the *n_out current particles, compacted in an unspecified order, to x, v
 * (device, [3][n_max] doubles, positions and four-velocities as for
 * mhdpic_particles_read), ids (device, [n_max] int32: the index of a particle
 * in mhdpic_init's arrays, then numbered on by mhdpic_inject in call order
 * and array order) and, if not NULL, tags (device, [n_max] doubles: the tags
 * given to mhdpic_inject, +infinity for particles without one).  Returns
 * MHDPIC_ENOMEM if more than n_max particles exist (*n_out still holds their
 * number; the first n_max found are written).  Waits for the stream. */
int mhdpic_particles_read_ids(mhdpic_ctx* ctx, double* x, double* v, int32_t* ids, double* tags,
                              int64_t n_max, int64_t* n_out, void* hip_stream);

/* Current particles per box: counts (host, [n_boxes] int64).  Waits. */
int mhdpic_counts(mhdpic_ctx* ctx, int64_t* counts, void* hip_stream);

/* Adds particles (Sec. 5: CRs injected at the shock front each step): n_new
 * (host, [n_boxes]) particles per box, box 0's first, from global positions
 * x and four-velocities v (device, [3][sum n_new] doubles), m, qm (device,
 * [sum n_new] doubles) and tags (device, [sum n_new] doubles, may be NULL:
 * +infinity), for instance the injection time.  The new particles join n_CR,
 * J_CR at once (the next step's cell-centred E sees them); the caller takes
 * their mass, momentum and energy from the gas (the paper's compensation).
 * A position must lie inside its box along non-periodic axes (MHDPIC_ERANGE
 * otherwise, returned after the particles were added).  MHDPIC_ENOMEM if the
 * context's slots (the sum of the boxes' capacity, or of their initial counts)
 * cannot hold them.  Waits for the stream. */
int mhdpic_inject(mhdpic_ctx* ctx, const int64_t* n_new, const double* x, const double* v,
                  const double* m, const double* qm, const double* tags, void* hip_stream);

/* Removes the particles whose tag is below t_cut once t_now is at least twice
 * their tag (Sec. 5: particles injected before t_cut are removed at twice
 * their injection time); their n_CR, J_CR leave the current deposits.  Needs
 * a context with a capacity (tags).  Waits for the stream. */
int mhdpic_remove_tagged(mhdpic_ctx* ctx, double t_cut, double t_now, void* hip_stream);

/* Waits for the stream and returns the latched device error (then clears it):
 * MHDPIC_OK, MHDPIC_ENONFINITE, MHDPIC_ERANGE or MHDPIC_ESTATE. */
int mhdpic_check(mhdpic_ctx* ctx, void* hip_stream);

/* Frees the context's host-side state.  The workspace is the caller's. */
int mhdpic_destroy(mhdpic_ctx* ctx);

/* Message for the last non-OK code returned on the calling thread. */
const char* mhdpic_last_error(void);

/* Per-phase kernel timing with HIP events recorded on the launch stream.
 * Phases: 0 = binning (rekey, scan, scatter), 1 = cell-centred field
 * preparation (which also clears the next n_CR, J_CR buffer), 2 = fused
 * gather/push/deposit, 3 = separate buffer clears (the step has none now;
 * the slot is kept so that the arrays keep their size).
 * mhdpic_timing_enable(ctx, phases) starts recording an event pair around
 * every later launch of the phases whose bit (1 << phase) is set in phases
 * (MHDPIC_TIMING_ALL: all four); 0 stops; other values are EINVAL.  Each
 * recorded event costs some microseconds of stream time, so time only the
 * phases you need.  Launches inside a graph capture are never timed.
 * mhdpic_timing_read waits for the recorded events, writes the summed
 * milliseconds and the number of timed launches of each phase (ms[4],
 * launches[4]) and clears the record. */
#define MHDPIC_TIMING_ALL 15
int mhdpic_timing_enable(mhdpic_ctx* ctx, int32_t phases);
int mhdpic_timing_read(mhdpic_ctx* ctx, double* ms, int64_t* launches);

/* Where the particles of a step move to their new slots.  Before each push
 * the particles are binned by the tile of the cell they have reached.
 *   MHDPIC_MOVES_IN_PUSH: the binning moves only the ids (and tags) and
 *     leaves a map from new slots to old ones; the push reads each particle
 *     through it and writes it, updated, to its new slot.  This saves a pass
 *     over the particle data, but the push's reads become gathers, whose
 *     cost grows the more the particles of a tile change cells in different
 *     ways from one step to the next;
 *   MHDPIC_MOVES_IN_BINNING: the binning moves every particle to its slot in
 *     the other particle buffer (a read and a write of all its data), and the
 *     push updates the particles in place;
 *   MHDPIC_MOVES_AUTO (the default): in the push.
 * Positions, velocities and deposits are the same either way, bit for bit.
 * Takes effect at the next step call.  EINVAL for another value. */
enum { MHDPIC_MOVES_AUTO = 0, MHDPIC_MOVES_IN_BINNING = 1, MHDPIC_MOVES_IN_PUSH = 2 };
int mhdpic_set_particle_moves(mhdpic_ctx* ctx, int32_t where);

/* Arithmetic self-test: out[0][i] = sqrt(a[i]), out[1][i] = a[i]/b[i],
 * out[2][i] = fma(a[i], b[i], c[i]), out[3][i] = (double)(int64)bits of c[i]
 * reinterpreted, computed by the device with the rounding the step kernels
 * use.  a, b, c device [n] doubles; out device [4][n].  Waits for the stream. */
int mhdpic_selftest_arith(const double* a, const double* b, const double* c, double* out,
                          int64_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif

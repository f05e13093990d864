/*
 * lb.h - C ABI of liblb: the two-component D3Q19 Shan-Chen lattice-Boltzmann
 * step on one AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv:2112.08264):
 *   - D3Q19 lattice: the rest velocity, 6 axis neighbours and 12 face
 *     diagonals (Sec. 2); weights 1/3, 1/18, 1/36 (Appendix, D3Q19 table).
 *   - Two population sets f_i^k, k in {A, B}; rho_k = sum_i f_i^k and the
 *     mixture momentum sum_k sum_i f_i^k c_i (Appendix, two-component LBE).
 *   - BGK relaxation f* = (1 - omega_k) f + omega_k f^eq, omega_k = 1/tau_k
 *     (Sec. 2, Eq. 1), viscosity c_s^2 (tau - 1/2) (Eq. 2), with the
 *     second-order equilibrium of Eq. LEQ (Appendix), c_s^2 = 1/3.
 *   - Streaming f_i(x + c_i, t + 1) = f*_i(x, t) (Eq. 1), periodic box, and
 *     halfway bounce-back at solid nodes at rest (Appendix, Eq. LADDFLBE
 *     with zero wall velocity).
 *   - Inter-component Shan-Chen force (not in the paper, which uses colour
 *     gradient): F_k(x) = -G psi_k(x) sum_{i=1..18} w_i psi_kbar(x + c_i) c_i,
 *     psi = rho_ref (1 - exp(-rho / rho_ref)), applied by shifting the
 *     equilibrium velocity of component k to
 *       v_k = u' + tau_k F_k / rho_k,
 *       u'  = (sum_k m_k / tau_k) / (sum_k rho_k / tau_k),  m_k = sum_i f_i^k c_i.
 *
 * Conventions shared by every call:
 *   - Node index n = x + nx * (y + ny * z), x fastest.  N = nx * ny * nz.
 *   - Population index order i = 0..18:
 *       0 (0,0,0); 1 (+1,0,0); 2 (-1,0,0); 3 (0,+1,0); 4 (0,-1,0);
 *       5 (0,0,+1); 6 (0,0,-1); 7 (+1,+1,0); 8 (-1,-1,0); 9 (+1,-1,0);
 *       10 (-1,+1,0); 11 (+1,0,+1); 12 (-1,0,-1); 13 (+1,0,-1);
 *       14 (-1,0,+1); 15 (0,+1,+1); 16 (0,-1,-1); 17 (0,+1,-1); 18 (0,-1,+1).
 *   - Population arrays exchanged through this ABI are float64
 *     [k][i][n] (k = A then B), 2 * 19 * N values, no padding; they hold the
 *     pre-collision state f(t) (the state the next step starts from).
 *   - Field arrays are float64 [n]; velocity arrays are float64 [3][n]
 *     (u_x plane, then u_y, then u_z); the solid mask is uint8 [n], nonzero
 *     meaning solid.
 *   - on_device != 0: the pointer is device memory of the context's device;
 *     on_device == 0: host memory.  The caller owns every array it passes;
 *     the library copies what it needs before returning (host inputs) or
 *     before the enqueued work completes (device inputs, stream-ordered).
 *   - Every call returns an lb_status and never aborts the process.
 *   - Work is enqueued on the context's stream.  lb_step returns without
 *     waiting; lb_set_fields, lb_set_populations, lb_moments,
 *     lb_get_populations and lb_totals return after their results are
 *     complete.  One context must not be used from two threads at once.
 */
#ifndef LB_H
#define LB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_ABI_VERSION 1

typedef struct lb_ctx lb_ctx; /* opaque; owned by the library */

typedef enum {
  LB_OK = 0,
  LB_EINVAL = -1,     /* bad argument: NULL pointer, size, tau <= 1/2, non-finite or negative input */
  LB_ENOMEM = -2,     /* device allocation failed */
  LB_EDEVICE = -3,    /* a HIP runtime call failed, or no usable device */
  LB_ESTATE = -4,     /* call out of order: no fields set yet */
  LB_ENONFINITE = -5  /* the state holds NaN or Inf */
} lb_status;

typedef enum {
  LB_F64 = 0,          /* populations stored as float64, float64 arithmetic */
  LB_F32 = 1,          /* stored as float32, float32 arithmetic */
  LB_F16_SHIFTED = 2   /* stored as float16 h = f - w_i rho0_k, float32 arithmetic */
} lb_storage;

typedef struct {
  int32_t nx, ny, nz;   /* periodic box, each >= 1; no tile-size restriction */
  double tau[2];        /* relaxation time per component, > 1/2 (Eq. 2: 0 < omega < 2) */
  double G;             /* Shan-Chen coupling; G > 0 pushes the components apart */
  double psi_ref;       /* rho_ref of the pseudopotential, > 0 (1.0 in the standard form) */
  double rho0[2];       /* reference density per component for LB_F16_SHIFTED; ignored otherwise */
  int32_t storage;      /* lb_storage */
  int32_t device;       /* HIP device ordinal */
  void* stream;         /* hipStream_t the work is enqueued on; NULL = the null stream */
} lb_params;

/* Fill *p with defaults: 1^3 box, tau = 1, G = 0, psi_ref = 1, rho0 = 1,
 * LB_F64, device 0, null stream. */
void lb_params_default(lb_params* p);

/* Validate *params, allocate the two population grids (A/B ping-pong) and
 * the work buffers on params->device, and return a context in *out.
 * Errors: LB_EINVAL (NULL, nx/ny/nz < 1, tau <= 1/2 or non-finite,
 * psi_ref <= 0, unknown storage, N * 38 overflowing 2^62), LB_EDEVICE (bad
 * device), LB_ENOMEM.  On error *out is set to NULL. */
lb_status lb_create(const lb_params* params, lb_ctx** out);

/* Wait for the context's work, free its device memory and the context.
 * NULL is accepted and ignored. */
lb_status lb_destroy(lb_ctx* ctx);

/* Replace the stream later calls enqueue on (NULL = null stream). */
lb_status lb_set_stream(lb_ctx* ctx, void* stream);

/* Initial state f_i^k(x) = f_i^eq(rho_k(x), u(x)) (Eq. LEQ), zero at solid
 * nodes.  rho_a, rho_b: [N], finite and >= 0.  u: [3][N] finite, or NULL
 * for a fluid at rest.  solid: [N] mask or NULL for none; the mask is kept
 * for every later step.  Errors: LB_EINVAL, LB_EDEVICE, LB_ENOMEM. */
lb_status lb_set_fields(lb_ctx* ctx, const double* rho_a, const double* rho_b,
                        const double* u, const uint8_t* solid, int on_device);

/* Advance n >= 0 steps.  One step: densities rho_k and pseudopotentials,
 * force, velocity-shifted BGK collision, pull streaming with bounce-back at
 * solid neighbours.  Enqueued; returns before completion.
 * Where nx is a multiple of 64 and ny of 4, the fused steps keep the
 * populations in a tile-major order inside the library (one contiguous
 * block per 64 x 4 tile and plane; float64 without fixed solid nodes,
 * float storage with or without, and the steps with moving particles):
 * the first step after lb_set_fields, lb_set_populations,
 * lb_restore_state, lb_set_particles or a call that needs the structure of
 * arrays (lb_save_state to host memory, the two-pass kernel) reorders the
 * grid once, and those calls reorder it back (one read and one write of
 * the grid each).  lb_moments, lb_totals, lb_get_populations and
 * lb_save_state to device memory read either order and reorder nothing.
 * Results do not depend on the order.
 * Errors: LB_EINVAL (n < 0), LB_ESTATE (no lb_set_fields /
 * lb_set_populations yet), LB_EDEVICE. */
lb_status lb_step(lb_ctx* ctx, int32_t n);

/* Moments of the current state: rho_a, rho_b [N] and the barycentric
 * velocity u = (m_A + m_B + (F_A + F_B) / 2) / (rho_A + rho_B) as [3][N]
 * (zero at solid nodes).  Any output pointer may be NULL to skip it.
 * Errors: LB_EINVAL, LB_ESTATE, LB_EDEVICE. */
lb_status lb_moments(lb_ctx* ctx, double* rho_a, double* rho_b, double* u, int on_device);

/* Copy out / replace the pre-collision populations, float64 [2][19][N].
 * lb_set_populations encodes into the context's storage format and zeroes
 * solid nodes.  Errors: LB_EINVAL, LB_ESTATE (get before any state),
 * LB_EDEVICE. */
lb_status lb_get_populations(lb_ctx* ctx, double* f, int on_device);
lb_status lb_set_populations(lb_ctx* ctx, const double* f, int on_device);

/* Conserved totals of the current state, accumulated in float64 on the
 * device with a fixed reduction order (bitwise repeatable):
 * out[0] = sum_x rho_A, out[1] = sum_x rho_B, out[2..4] = sum_x sum_k m_k.
 * *nonfinite = 1 if any population is NaN or Inf (and the call then returns
 * LB_ENONFINITE), else 0.  Errors: LB_EINVAL, LB_ESTATE, LB_EDEVICE. */
lb_status lb_totals(lb_ctx* ctx, double out[5], int* nonfinite);

/* Per-kernel timing with HIP events recorded around every launch on the
 * context's stream.  lb_timing(ctx, 1) starts a fresh record, 0 stops
 * recording.  lb_timing_read waits for the stream and returns, for kernel
 * slot k (0 <= k < lb_timing_slots()), the summed duration in milliseconds
 * and the launch count; lb_timing_name gives the slot's kernel name. */
lb_status lb_timing(lb_ctx* ctx, int enable);
lb_status lb_timing_read(lb_ctx* ctx, int32_t slot, double* total_ms, int64_t* launches);
int32_t lb_timing_slots(void);
const char* lb_timing_name(int32_t slot);

/* Step implementation.  LB_KERNEL_FUSED reads and writes every population
 * once per step: one kernel marches z-columns and keeps the pseudopotential
 * of three planes in LDS.  LB_KERNEL_FUSED_STAGED (the default;
 * LB_KERNEL_AUTO picks it) is the same march for LB_F64 with nx a multiple
 * of 32 and no solid nodes, where the populations of the plane two ahead are
 * copied into LDS by direct-to-LDS loads while the current plane is
 * collided; other storages, shapes and lattices with solids run
 * LB_KERNEL_FUSED.  LB_KERNEL_TWO_PASS computes the
 * pseudopotential field in a first kernel and collides and streams in a
 * second.  All give bitwise identical results for LB_F64.
 * Errors: LB_EINVAL (unknown value). */
typedef enum {
  LB_KERNEL_AUTO = 0,
  LB_KERNEL_FUSED = 1,
  LB_KERNEL_TWO_PASS = 2,
  LB_KERNEL_FUSED_STAGED = 3
} lb_kernel;
lb_status lb_set_kernel(lb_ctx* ctx, int32_t kernel);

/* Change the Shan-Chen coupling G of later steps (and adjoint steps).
 * Errors: LB_EINVAL (NULL, non-finite G). */
lb_status lb_set_coupling(lb_ctx* ctx, double G);

/* ---- Colour-gradient model (the paper's two-component model, Appendix;
 * case 2 of Sec. 5) ----------------------------------------------------------
 * lb_set_model switches the context's collision between
 *   LB_MODEL_SHAN_CHEN (the default): the pseudopotential force by velocity
 *     shift, as described at lb_create;
 *   LB_MODEL_COLOUR_GRADIENT: per component, BGK towards f^eq(rho_k, u) at
 *     the mixture velocity u = (m_A + m_B) / rho with one effective
 *     omega = 2 / (6 nu_bar + 1), 1/nu_bar = (rho_A/rho)/nu_A +
 *     (rho_B/rho)/nu_B, nu_k = (tau_k - 1/2)/3 (Appendix, Eq. 1coll; Eq. 2),
 *     plus the perturbation (A/2)|g|(w_i (c_i.n)^2 - B_i) with
 *     A = (9/4) sigma omega (Eq. 2coll, Eq. sigmaA); the sum of the two
 *     components is then split by the recolouring
 *     f_i^A = (rho_A/rho) f*_i + beta (rho_A rho_B / rho^2) cos(phi_i) w_i rho
 *     and f_i^B = (rho_B/rho) f*_i - (the same term) (Eq. 3coll), where
 *     g = 3 sum_i w_i Theta(x + c_i) c_i is the gradient of the phase field
 *     Theta = (rho_A - rho_B)/(rho_A + rho_B), n = g/|g| and
 *     cos(phi_i) = c_i.n / |c_i|.  The perturbation and the recolouring act
 *     only where |g|^2 > 1e-16 (float32: 1e-10).  Streaming is periodic.
 * sigma (surface tension, >= 0) and beta (recolouring, >= 0) are used by the
 * colour-gradient model only; G and psi_ref by the Shan-Chen model only.
 * The model applies to later lb_step calls; lb_moments then reports
 * u = (m_A + m_B) / rho.  The colour-gradient model takes LB_F64 or LB_F32
 * storage, no solid nodes, and every node needs rho_A + rho_B > 0
 * (lb_set_fields checks this); lb_step with LB_KERNEL_TWO_PASS, the
 * adjoint calls, lb_step_record and lb_step_between return LB_EINVAL in it.
 * Errors: LB_EINVAL (NULL ctx, unknown model, non-finite or negative sigma
 * or beta, LB_F16_SHIFTED storage or solid nodes with the colour-gradient
 * model). */
typedef enum {
  LB_MODEL_SHAN_CHEN = 0,
  LB_MODEL_COLOUR_GRADIENT = 1
} lb_model;
lb_status lb_set_model(lb_ctx* ctx, int32_t model, double sigma, double beta);

/* ---- Raw state snapshots (checkpointing) -------------------------------
 * A snapshot is the current population grid in the library's storage
 * format: lb_state_bytes() bytes, structure of arrays (plane k * 19 + i at
 * offset (k * 19 + i) * Npad elements, Npad = N rounded up to 128), whatever
 * order lb_step keeps internally (lb_save_state to device memory writes it
 * straight from that order).  It is meant only for lb_restore_state,
 * lb_step_between and lb_adjoint_step of a context with the same parameters.
 * lb_save_state copies the current state to dst; lb_restore_state makes src
 * the current state.  on_device selects device or host memory.
 * Errors: LB_EINVAL, LB_ESTATE (save before any state), LB_EDEVICE. */
lb_status lb_state_bytes(const lb_ctx* ctx, int64_t* bytes);
lb_status lb_save_state(lb_ctx* ctx, void* dst, int on_device);
lb_status lb_restore_state(lb_ctx* ctx, const void* src, int on_device);

/* One step from the snapshot at fin to the snapshot at fout, both device
 * memory of lb_state_bytes() bytes, fin != fout; the context's own state is
 * untouched.  Solid-node entries of fout are not written.  Enqueued on the
 * context's stream.  Errors: LB_EINVAL, LB_EDEVICE. */
lb_status lb_step_between(lb_ctx* ctx, const void* fin, void* fout);

/* ---- Discrete adjoint (reverse-mode gradient of a final-state objective) --
 * For an objective J of the densities after T steps, the caller
 *   1. seeds lam(T) = dJ/df(T) from dJ/drho_A and dJ/drho_B at step T
 *      (lb_adjoint_begin; float64 [N] each, NULL = zero), which also zeroes
 *      the dJ/dG accumulator;
 *   2. calls lb_adjoint_step once per step, last step first, each time with
 *      the device snapshot of the pre-collision state f(t) that step started
 *      from (t = T-1 down to 0), which maps lam(t+1) to lam(t) and adds the
 *      step's part of dJ/dG: the transposed streaming (with bounce-back),
 *      the transposed collision Jacobian including the velocity shift, and
 *      the transposed Shan-Chen stencil;
 *   3. reads dJ/drho_k(x, 0) = sum_i w_i lam_i^k(x, 0), the gradient with
 *      respect to the densities of an initial state at rest (f = w_i rho_k,
 *      Appendix Eq. LEQ with u = 0), and dJ/dG (lb_adjoint_result; any
 *      output may be NULL).
 * The adjoint's arithmetic type is the context's (float64 for LB_F64,
 * float32 otherwise).  lb_adjoint_lambda exports lam as float64 [2][19][N].
 * Errors: LB_EINVAL, LB_ESTATE (step or result before begin), LB_ENOMEM,
 * LB_EDEVICE. */
lb_status lb_adjoint_begin(lb_ctx* ctx, const double* dJ_drho_a, const double* dJ_drho_b, int on_device);
lb_status lb_adjoint_step(lb_ctx* ctx, const void* state);
lb_status lb_adjoint_result(lb_ctx* ctx, double* dJ_drho_a0, double* dJ_drho_b0, double* dJ_dG, int on_device);
lb_status lb_adjoint_lambda(lb_ctx* ctx, double* lam, int on_device);

/* The adjoint needs, per step, only the moments of f(t): rho_A, rho_B,
 * m_A (3), m_B (3), psi_A, psi_B, each [N] in the context's arithmetic type
 * (a "record" of lb_record_bytes() bytes, zero at solid nodes).
 * lb_step_record advances the context's own state by one step, exactly as
 * lb_step(ctx, 1), and writes the record of the state it started from into
 * device memory; lb_adjoint_step_record is lb_adjoint_step with that record
 * in place of the snapshot.  A checkpointed backward pass restores a
 * checkpoint, records the segment's steps and runs the adjoint over the
 * records in reverse.  Errors: LB_EINVAL, LB_ESTATE, LB_EDEVICE. */
lb_status lb_record_bytes(const lb_ctx* ctx, int64_t* bytes);
lb_status lb_step_record(lb_ctx* ctx, void* record);
lb_status lb_adjoint_step_record(lb_ctx* ctx, const void* record);

/* Bytes of device memory the context holds. */
lb_status lb_device_bytes(const lb_ctx* ctx, int64_t* bytes);

/* ---- Single-fluid step (the paper's case 1, Sec. 5) ----------------------
 * One population set: rho = sum_i f_i, u = m / rho, BGK relaxation towards
 * f^eq(rho, u) (Sec. 2, Eq. 1; Appendix, Eq. LEQ), push streaming with
 * halfway bounce-back at solid nodes at rest (Appendix, Eq. LADDFLBE with
 * the wall velocity set to zero), periodic box.  No inter-component force.
 * Parameters come from lb_params: nx, ny, nz, tau[0] (> 1/2), rho0[0] (the
 * float16 offset w_i rho0), storage, device and stream; the other fields
 * are ignored.  Storage per step: 19 values read and 19 written per node.
 * Ownership, streams and on_device flags work as for the two-component
 * calls above; populations are [19][N] float64, u is [3][N], rho is [N].
 * lb1_totals writes (M, P_x, P_y, P_z).  Errors as for the corresponding
 * two-component calls. */
typedef struct lb1_ctx lb1_ctx; /* opaque; owned by the library */
lb_status lb1_create(const lb_params* params, lb1_ctx** out);
lb_status lb1_destroy(lb1_ctx* ctx);
lb_status lb1_set_stream(lb1_ctx* ctx, void* stream);
lb_status lb1_set_fields(lb1_ctx* ctx, const double* rho, const double* u, const uint8_t* solid, int on_device);
lb_status lb1_step(lb1_ctx* ctx, int32_t n);
lb_status lb1_moments(lb1_ctx* ctx, double* rho, double* u, int on_device);
lb_status lb1_get_populations(lb1_ctx* ctx, double* f, int on_device);
lb_status lb1_totals(lb1_ctx* ctx, double out[4], int* nonfinite);

/* ---- Moving particles in the single-fluid step (the paper's particle
 * solver: Sec. 2, Eq. PARDYN; Sec. 3; Appendix, Eqs. UPI, LADDFLBE,
 * FORCEPP, FORCEPARTEQ, TORQUEPARTEQ) ---------------------------------------
 * lb1_set_particles places `count` rigid spheres of one radius and mass in
 * the current fluid state (call it after lb1_set_fields, which drops any
 * particles).  Host arrays [count][3], float64:
 *   pos   centres, each coordinate in [0, L) (x, y, z);
 *   vel   velocities (NULL = 0), each component below 0.5 in magnitude;
 *   omega angular velocities (NULL = 0).
 * A node belongs to a particle when its distance d from the centre meets
 * (d_x d_x + d_y d_y) + d_z d_z <= radius^2.  A node inside two particles
 * belongs to the lower index.  The populations of particle nodes are
 * discarded.  mass may be +inf (the particle then keeps its velocities);
 * the moment of inertia is (2/5) mass radius^2.  Particles already placed
 * are removed first: their nodes turn to fluid at rest, f_i = w_i rho0[0]
 * (count = 0 only removes).
 * lb1_step then advances fluid and particles together.
 *   - Links from a fluid node into a particle bounce back with
 *     f_ibar = f*_i - 2 rho w_i (u_b . c_i) / c_s^2, where rho is the fluid
 *     node's density and u_b = v + omega x r_b at the link midpoint r_b.
 *   - The particle receives c_i (f*_i + f_ibar) per link, and r_b x that as
 *     torque.  These are summed in float64 in a fixed order.
 *   - Leap-frog: v += F / m, omega += T / I, then the centre moves by v.
 *   - Nodes covered by the move give their momentum to the particle.  Nodes
 *     uncovered start at f^eq(rho0[0], u_b) and take that momentum from it.
 *   - Total momentum, fluid plus particles, is conserved to rounding.
 * lb1_get_particles copies the particle state to host arrays [count][3]
 * (any may be NULL): positions, velocities, angular velocities, and the
 * force and torque of the last step.
 * Storage LB_F64 or LB_F32.  Not with fixed solids from lb1_set_fields.
 * Each particle's box, floor(2 radius) + 4 nodes, must fit the lattice on
 * every axis.
 * Errors: LB_EINVAL (NULL ctx or pos, bad radius, mass, position or speed;
 * fixed solids; LB_F16_SHIFTED; box larger than the lattice), LB_ESTATE
 * (lb1_set_particles before lb1_set_fields; lb1_get_particles without
 * particles), LB_ENOMEM, LB_EDEVICE. */
lb_status lb1_set_particles(lb1_ctx* ctx, int32_t count, double radius, double mass, const double* pos,
                            const double* vel, const double* omega);
lb_status lb1_get_particles(lb1_ctx* ctx, double* pos, double* vel, double* omega, double* force, double* torque);

/* ---- Moving particles in the colour-gradient fluid (the paper's case 3:
 * two immiscible fluids with colloidal particles, Sec. 5; particle solver
 * of Sec. 2, Eq. PARDYN; Sec. 3; Appendix, Eqs. UPI, LADDFLBE, FORCEPP,
 * FORCEPARTEQ, TORQUEPARTEQ) -------------------------------------------------
 * lb_set_particles places spheres in a context switched to
 * LB_MODEL_COLOUR_GRADIENT, with the arguments, node ownership, mass,
 * removal and limits of lb1_set_particles.  Per step: the colour-gradient
 * collision at fluid nodes, where a neighbour inside a particle contributes
 * the node's own phase field Theta to the gradient (neutral, 90 degree
 * wetting); then, per component k, bounce-back at each link from a fluid
 * node x into a particle node with the moving-wall term
 *   f^k_ibar(x, t+1) = f^k*_i(x) - 2 rho^k(x) w_i (u_b . c_i) / c_s^2,
 * u_b = v + omega x r_b at the link midpoint; the particle receives
 * c_i (f^k*_i(x) + f^k_ibar(x, t+1)) from each component of each link,
 * summed in float64; leap-frog; nodes a particle covers hand the momentum
 * of both components to it, nodes it uncovers start at
 * f^eq(rho0[k], u_b) per component and take that momentum from it.
 * Removed particles leave fluid at rest, f^k_i = w_i rho0[k].
 * Storage LB_F64 or LB_F32; lb_set_fields drops the particles; with
 * particles lb_restore_state returns LB_EINVAL, lb_moments reports zeros
 * at particle nodes and lb_totals sums the fluid only.
 * lb_get_particles works as lb1_get_particles.
 * Errors: LB_EINVAL (NULL ctx or pos; not the colour-gradient model; bad
 * radius, mass, position or speed; LB_F16_SHIFTED; box larger than the
 * lattice), LB_ESTATE (before lb_set_fields; lb_get_particles without
 * particles), LB_ENOMEM, LB_EDEVICE.  lb_set_model back to
 * LB_MODEL_SHAN_CHEN returns LB_EINVAL while particles are placed. */
lb_status lb_set_particles(lb_ctx* ctx, int32_t count, double radius, double mass, const double* pos,
                           const double* vel, const double* omega);
lb_status lb_get_particles(lb_ctx* ctx, double* pos, double* vel, double* omega, double* force, double* torque);

/* ---- Conserved totals of a snapshot, without allocating -----------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * totals of lb_totals computed from a caller-owned device snapshot, with no
 * context.  Nothing is allocated: the per-workgroup partial sums live in a
 * fixed device array inside the library (131,136 bytes per device, held
 * until the process ends; the reduction grid is capped at 2048 workgroups,
 * so every lattice fits).  The call calls no hipMalloc or hipFree.
 *   params    nx, ny, nz, storage, rho0 (LB_F16_SHIFTED decoding), device
 *             and stream are used; the other fields are ignored.
 *   snapshot  device memory in the snapshot format of lb_save_state:
 *             storage-typed, plane k * 19 + i at (k * 19 + i) * Npad
 *             elements, Npad = N rounded up to 128.  Read only.
 *   solid     device uint8 [N] (non-zero = solid, skipped), or NULL.
 *   out       6 doubles: M_A, M_B, P_x, P_y, P_z (as lb_totals, same
 *             reduction order, bitwise the same) and the count of
 *             non-finite populations.  on_device = 1: device memory; the
 *             call only enqueues on params->stream and returns LB_OK (the
 *             caller reads out[5] for the non-finite count).  on_device = 0:
 *             host memory; the call waits for the stream and returns
 *             LB_ENONFINITE when out[5] != 0.
 * Calls that overlap on one device share its array and race: issue them on
 * one stream, or wait for one before the next.  The array keeps the last
 * call's partial sums; each call writes the partials it reads first.
 * Errors: LB_EINVAL (NULL params, snapshot or out; a size below 1; an
 * unknown storage; non-finite rho0 with LB_F16_SHIFTED; more than
 * 2^31 - 4097 nodes), LB_EDEVICE (bad device ordinal or a HIP failure),
 * LB_ENONFINITE (host out only). */
lb_status lb_snapshot_totals(const lb_params* params, const void* snapshot, const uint8_t* solid, double* out,
                             int32_t on_device);

/* Human-readable text for a status code. */
const char* lb_strerror(lb_status status);

/* LB_ABI_VERSION of the built library. */
int32_t lb_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */

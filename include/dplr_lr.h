/*
 * dplr_lr.h - C ABI of the MI355X (gfx950) DPLR long-range electrostatic step.
 *
 * The library evaluates the Gaussian-charge long-range energy of Deep Potential
 * Long-Range (paper: DPLR background section, the energy E_Gt and structure
 * factor S(m) equations) by particle-particle particle-mesh (PPPM) with
 * ik-differentiation ("Poisson-IK", Optimization section, hardware-offloaded
 * 3D FFT: one forward and three inverse 3D FFTs), times the Coulomb constant:
 *
 *   E = k_e/(2 pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2,
 *   S(m) = sum_i q_i exp(-2 pi i m.R_i) + sum_n q_n exp(-2 pi i m.W_n),
 *
 * where R_i are ion (atom) positions and W_n Wannier-centroid (WC) positions.
 * It returns E, the forces on ions and on WCs separately (the two derivative
 * terms dE_Gt/dR_i and dE_Gt/dW_n of the force chain-rule equations), and the
 * virial.  Every step runs in the library's own HIP kernels; callers provide
 * device memory and a HIP stream.
 *
 * Conventions
 *   - Units: Angstrom, elementary charge, eV (k_e = 14.399645 eV A gives eV).
 *   - Box: orthorhombic, edge lengths L[3]; positions may lie anywhere (they
 *     are wrapped into the box).  A non-finite coordinate (NaN or +-Inf) is
 *     taken as 0 on its axis, so no input position leads outside the mesh;
 *     non-finite charges give non-finite outputs.  The m = 0 term is excluded
 *     (tin-foil boundary); a non-neutral input is computed as given.
 *   - Arrays: positions and forces are contiguous [n][3] (x, y, z), charges
 *     [n]; element type float for DPLR_LR_FP32 plans and double for
 *     DPLR_LR_FP64 plans.  Energy and virial are always double.
 *   - Virial order: xx, yy, zz, xy, xz, yz; W_ab = -dE/d(strain_ab).
 *   - Every call is asynchronous on the plan's stream (no host
 *     synchronisation, no device-to-host copy).  Device pointers must stay
 *     valid until the stream has executed the call.  The library never frees
 *     or keeps caller memory.
 *   - One plan must not be used from two host threads, or on two streams, at
 *     the same time (its workspace is shared by its calls).
 *
 * Errors
 *   Every entry point validates its arguments on the host before it enqueues
 *   any device work; on an error it returns a status code, leaves all outputs
 *   untouched and records a message for dplr_lr_last_error().
 */
#ifndef DPLR_LR_H
#define DPLR_LR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPLR_LR_ABI_VERSION 1

typedef struct dplr_lr_plan_s* dplr_lr_plan;

typedef enum {
  DPLR_LR_OK = 0,
  DPLR_LR_E_INVALID = 1,      /* bad argument (null pointer, negative size, ...) */
  DPLR_LR_E_UNSUPPORTED = 2,  /* valid request outside what the library supports */
  DPLR_LR_E_NO_BOX = 3,       /* compute before set_box                          */
  DPLR_LR_E_CAPACITY = 4,     /* more particles than the plan's capacity         */
  DPLR_LR_E_DEVICE = 5,       /* a HIP runtime call failed                       */
  DPLR_LR_E_NOMEM = 6         /* device or host allocation failed                */
} dplr_lr_status;

typedef enum { DPLR_LR_FP32 = 0, DPLR_LR_FP64 = 1 } dplr_lr_precision;

/* flags */
#define DPLR_LR_ACCUMULATE 0x1u   /* add forces into the output arrays instead of overwriting */
#define DPLR_LR_NO_VIRIAL  0x2u   /* skip the virial reduction (virial6 may be NULL)         */
/* Forces by analytic differentiation of the B-spline assignment weights
 * instead of ik: the potential phi(g) = sum_n G(n) Q^(n) exp(2 pi i n.g/K)
 * takes one inverse FFT (instead of three), and
 *   F_ja = -(k_e q_j / (V h_a)) sum_g phi(g) dW(u_j - g)/du_a
 * is the exact gradient of the returned energy (same E and virial as ik).
 * Not the paper's choice (it uses Poisson-IK); the adjacent textbook
 * variant.  The net force is not exactly zero. */
#define DPLR_LR_DIFF_AD    0x4u

typedef struct {
  int32_t mesh[3];     /* Kx, Ky, Kz, each at most 512 with no prime factor but 2, 3, 5.
                          Powers of two from 16 up run on the plane/pencil kernels; any
                          other mesh (e.g. the paper's 8x12x8, 10x15x10 and 12x18x12
                          precision-study grids, Evaluation section) on the mixed-radix
                          kernels, which need every size >= order and take no
                          DPLR_LR_DIFF_AD                                               */
  int32_t order;       /* B-spline assignment order p (points per axis), 2..8             */
  double beta;         /* Gaussian width parameter beta of the E_Gt equation (1/A), > 0  */
  double coulomb_k;    /* Coulomb constant k_e (eV A); E is returned in its units         */
  int32_t precision;   /* dplr_lr_precision of spreading, FFTs and gather; the influence
                          table and the energy/virial reductions are FP64 in both modes  */
  int32_t alias_range; /* |m_a| <= alias_range in the influence-function alias sums, 0..4 */
  int64_t capacity;    /* maximum n_ion + n_wc per call, 0 .. 2^31 - 1                    */
  uint32_t flags;      /* DPLR_LR_ACCUMULATE | DPLR_LR_NO_VIRIAL | DPLR_LR_DIFF_AD        */
} dplr_lr_config;

/* Version of this ABI (DPLR_LR_ABI_VERSION of the built library). */
int32_t dplr_lr_abi_version(void);

/* Fill *cfg with the defaults: mesh 32^3, order 5, beta 0.4, k_e 14.399645,
 * FP32, alias range 2, capacity 0, no flags. */
void dplr_lr_config_default(dplr_lr_config* cfg);

/* Host-only validation of a configuration (no device call).  On failure a
 * message is written to msg (NUL-terminated, at most msg_len bytes) when msg
 * is not NULL. */
dplr_lr_status dplr_lr_config_validate(const dplr_lr_config* cfg, char* msg, int64_t msg_len);

/* Create a plan: validates cfg, then allocates the device workspace on the
 * current HIP device.  hip_stream is a hipStream_t (NULL = the null stream).
 * On success *out owns the workspace until dplr_lr_plan_destroy.  On failure
 * *out is set to NULL and dplr_lr_last_error(NULL) holds the message. */
dplr_lr_status dplr_lr_plan_create(const dplr_lr_config* cfg, void* hip_stream, dplr_lr_plan* out);

/* Rebind the plan to another stream (hipStream_t). */
dplr_lr_status dplr_lr_set_stream(dplr_lr_plan p, void* hip_stream);

/* The paper's Mixed-Int32 transforms (Optimization section, int32
 * quantisation of the FFT reduction chains; Evaluation section, precision
 * configurations), for mixed-radix plans with every mesh size <= 256.  Each
 * 1D transform of every 3D transform (x, then y, then z) is formed as the sum
 * over nodes[a] consecutive blocks of K_a / nodes[a] points of the blocks'
 * partial DFTs; each partial value (real and imaginary part) is multiplied by
 * scale, rounded to the nearest integer and clamped to the int32 range, the
 * integers are added exactly and the sum is divided by scale (the paper uses
 * scale = 1e7).  The charge spectrum is transformed in charge units and the
 * field spectra carry k_e / V, so the inverse transforms produce the field
 * (eV/A per unit charge), values of order one.  nodes (host, 3 ints) must
 * divide the mesh sizes; scale in (0, 2^31].  nodes = NULL switches the mode
 * off.  Returns E_UNSUPPORTED on plans whose mesh runs on the plane/pencil
 * kernels (powers of two from 16 to 512).  Takes effect from the
 * next compute; energy and virial come from the quantised charge spectrum. */
dplr_lr_status dplr_lr_set_fft_int32(dplr_lr_plan p, const int32_t nodes[3], double scale);

/* Set the orthorhombic box (host array of 3 positive lengths, Angstrom) and
 * enqueue the FP64 influence-function table for it: the optimal ik influence
 * function of Hockney and Eastwood for the Gaussian-screened Coulomb kernel
 * 4 pi exp(-k^2/4 beta^2)/k^2 (the Fourier form of the E_Gt summand) with
 * B-spline assignment of the plan's order. */
dplr_lr_status dplr_lr_set_box(dplr_lr_plan p, const double box_len[3]);

/* The long-range step.  Device inputs: ion_pos [n_ion][3], ion_q [n_ion],
 * wc_pos [n_wc][3], wc_q [n_wc] (plan precision).  Device outputs:
 * ion_force [n_ion][3] and wc_force [n_wc][3] (F = -dE/dr, eV/A, plan
 * precision), energy (1 double, eV) and virial6 (6 doubles, eV).  Without
 * DPLR_LR_NO_VIRIAL, virial6 must not be NULL (E_INVALID); with it the virial
 * is not computed, virial6 is not written and may be NULL.  Pointers of an
 * empty set (n = 0) may be NULL.  Requires set_box first and
 * n_ion + n_wc <= capacity. */
dplr_lr_status dplr_lr_compute_energy_forces_virial(
    dplr_lr_plan p,
    int64_t n_ion, const void* ion_pos, const void* ion_q,
    int64_t n_wc, const void* wc_pos, const void* wc_q,
    void* ion_force, void* wc_force, double* energy, double* virial6);

/* Backward of the energy with respect to positions (the derivative the
 * force chain-rule equations take of E_Gt): ion_grad = -g * ion_force and
 * wc_grad = -g * wc_force, with g = *grad_energy (a device double, the
 * incoming gradient of E).  Arrays as in compute; outputs may alias their
 * inputs. */
dplr_lr_status dplr_lr_scale_grad(dplr_lr_plan p, const double* grad_energy,
                                  int64_t n_ion, const void* ion_force, void* ion_grad,
                                  int64_t n_wc, const void* wc_force, void* wc_grad);

/* ------------------------------------------------------------------------
 * The same step without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It needs no plan: cfg and box_len (host) describe what
 * dplr_lr_plan_create and dplr_lr_set_box would (cfg->capacity is not used),
 * and the arguments after them are those of
 * dplr_lr_compute_energy_forces_virial, with the same meaning, layout and
 * results; hip_stream is a hipStream_t (NULL = the null stream).
 *
 * Working memory is one library-owned device array of
 * DPLR_LR_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load until
 * the process ends; the call allocates nothing.  A request that does not fit
 * returns DPLR_LR_E_CAPACITY before any device work (the 128^3 FP32 mesh
 * leaves room for about 2.5 million particles, 64^3 for about 5 million).
 * Only power-of-two meshes from 16 to 512 are taken (E_UNSUPPORTED
 * otherwise).  The first call on a device looks up the array's address and
 * writes the FFT twiddle tables into it with synchronous copies, so a caller
 * that captures graphs makes one call before capturing.  The influence table
 * is recomputed only when the mesh, order, alias range, beta or box differ
 * from the previous call on that device.
 *
 * Every call on a GPU shares that GPU's array and leaves its contents there:
 * calls that overlap on one GPU (two host threads, or two streams whose work
 * can run at the same time) race and give wrong results; serialise them.
 * Errors are reported by dplr_lr_last_error(NULL). */
#define DPLR_LR_NOALLOC_SCRATCH_BYTES (128LL << 20)
dplr_lr_status dplr_lr_compute_noalloc(const dplr_lr_config* cfg, const double box_len[3],
                                       int64_t n_ion, const void* ion_pos, const void* ion_q,
                                       int64_t n_wc, const void* wc_pos, const void* wc_q,
                                       void* ion_force, void* wc_force, double* energy, double* virial6,
                                       void* hip_stream);

/* Release the plan and its workspace (synchronises the plan's stream). NULL is accepted. */
dplr_lr_status dplr_lr_plan_destroy(dplr_lr_plan p);

/* Message of the last failed call on p (p = NULL: the last failed plan
 * creation or validation of this thread).  Valid until the next call on p. */
const char* dplr_lr_last_error(dplr_lr_plan p);

/* Device bytes held by the plan's workspace. */
int64_t dplr_lr_workspace_bytes(dplr_lr_plan p);

/* Intermediate buffers of the most recent compute (for kernel-level tests):
 *   DPLR_LR_BUF_SPECTRUM  the charge mesh transformed along x (real to
 *                         complex) and y; the z transform is done inside
 *                         the Poisson pass.  complex [Kx/2+1][Kz][Ky]
 *                         (kx slowest, y fastest);
 *   DPLR_LR_BUF_INFLUENCE FP64 influence table G(|nx|,|ny|,|nz|),
 *                         [Kx/2+1][Ky/2+1][Kz/2+1];
 *   DPLR_LR_BUF_FIELD_SPECTRA the field spectra after the inverse z
 *                         transform, complex [3][Kx/2+1][Kz][Ky] (plans
 *                         whose z planes do not fit in LDS also apply the
 *                         inverse y transform here; DPLR_LR_DIFF_AD plans
 *                         fill only the first, the potential).
 * Mixed-radix plans (meshes outside the powers of two from 16 to 512) keep
 * only DPLR_LR_BUF_INFLUENCE: debug_size returns -1 for the others and
 * debug_copy E_INVALID.
 * Copies `bytes` bytes (at most the buffer size, else E_INVALID) into the
 * device pointer dst, stream-ordered. */
#define DPLR_LR_BUF_SPECTRUM 0
#define DPLR_LR_BUF_INFLUENCE 1
#define DPLR_LR_BUF_FIELD_SPECTRA 2
/* Mixed-radix plans: the number of partial values (real and imaginary parts
 * counted separately) that the int32-quantised transforms of the last compute
 * clamped to the int32 range, one uint64.  A partial value saturates when
 * |value| * scale >= 2^31, i.e. above about 214.7 at the paper's scale 1e7
 * (charge units in the forward transform, eV/A per unit charge in the
 * inverse ones); a non-zero count means the forces of that call are not the
 * rounded transforms of the header's dplr_lr_set_fft_int32 description. */
#define DPLR_LR_BUF_Q32_CLAMPED 3
dplr_lr_status dplr_lr_debug_copy(dplr_lr_plan p, int32_t which, void* dst, int64_t bytes);
int64_t dplr_lr_debug_size(dplr_lr_plan p, int32_t which);

/* One axis of the int32-quantised transform of dplr_lr_set_fft_int32 (for
 * element-wise kernel tests): transforms, in place on the plan's stream, the
 * device array data of ncomp (1..3) complex meshes [ncomp][Kz][Ky][Kx] (plan
 * precision, x fastest) along axis (0 = x, 1 = y, 2 = z) with exp(sign 2 pi
 * i n k / K_axis), sign = -1 or +1, using the plan's node counts and scale.
 * E_UNSUPPORTED unless int32 transforms are enabled on a mixed-radix plan. */
dplr_lr_status dplr_lr_debug_dft_q32(dplr_lr_plan p, int32_t axis, int32_t sign, void* data, int32_t ncomp);

/* Instrumentation (not part of the method).  When enabled, compute records a
 * HIP event pair on the plan's stream around each of its kernels.
 * profile_read synchronises the plan's stream, adds the elapsed times of all
 * recorded pairs to per-stage totals and writes, for stage i < max, the
 * summed milliseconds ms[i] and the number of launches calls[i]; *n (may be
 * NULL) receives the number of stages; reset != 0 clears the totals after
 * reading.  profile_stage_name(i) names stage i ("" when out of range). */
dplr_lr_status dplr_lr_profile_enable(dplr_lr_plan p, int32_t enable);
dplr_lr_status dplr_lr_profile_read(dplr_lr_plan p, double* ms, int64_t* calls, int32_t max, int32_t* n,
                                    int32_t reset);
const char* dplr_lr_profile_stage_name(int32_t i);

/* ------------------------------------------------------------------------
 * Learned coarse-mesh correction.  A plan on a mesh twice as coarse computes
 * PPPM forces; this network adds a per-particle correction dF_i predicted from
 * the particle's charge neighbourhood, trained on fine-minus-coarse PPPM force
 * residuals the method itself generates.  The structure follows the paper's
 * Deep Potential / Deep Wannier description (DPLR background section):
 * a descriptor D_i built from the neighbour list, then a three-hidden-layer
 * fitting net, here predicting a vector per particle as the Deep Wannier
 * model does.  Definitions:
 *   T_i[k, a] = sum_{j: r_ij < cutoff} q_j T_k(2 r_ij / cutoff - 1) s(r_ij) u_a,
 *     T_k Chebyshev (k < 32), s(r) = (1 + cos(pi r / cutoff)) / 2,
 *     u = (1, unit vector from i to j);
 *   D_i[4k + l] = sum_a T_i[k, a] T_i[l, a] (l < 4); x_i = (D_i - mu) * inv_sigma;
 *   h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), h3 = silu(h2 W3 + b3),
 *   c = h3 W4 + b4 (128 -> 64 -> 64 -> 64 -> 32; BF16 MFMA, FP32 accumulate);
 *   dF_i = out_scale * q_i * sum_k c_ik T_i[k, 1:4].
 * Packed FP32 parameters: W1[128][64] b1[64] W2[64][64] b2[64] W3[64][64]
 * b3[64] W4[64][32] b4[32] mu[128] inv_sigma[128] (W stored [in][out]).
 * Positions, charges, forces and targets are FP32 device arrays [n][3] / [n];
 * the box is orthorhombic (host double[3]) and at least 3 cutoffs long.
 * ---------------------------------------------------------------------- */
typedef struct dplr_lr_mlp_s* dplr_lr_mlp;

typedef struct {
  double cutoff;     /* neighbour cutoff (A), default 4 */
  double out_scale;  /* fixed output scale of the force head, default 0.01 */
  int64_t capacity;  /* maximum n_ion + n_wc */
  uint32_t flags;    /* reserved, 0 */
} dplr_lr_mlp_config;

void dplr_lr_mlp_config_default(dplr_lr_mlp_config* cfg);
int64_t dplr_lr_mlp_param_count(void);
/* Allocates the network's workspace for `capacity` particles; parameters start at zero. */
dplr_lr_status dplr_lr_mlp_create(const dplr_lr_mlp_config* cfg, void* hip_stream, dplr_lr_mlp* out);
dplr_lr_status dplr_lr_mlp_destroy(dplr_lr_mlp m);
dplr_lr_status dplr_lr_mlp_set_stream(dplr_lr_mlp m, void* hip_stream);
/* Host copies of the packed parameters (synchronous); set_params resets the Adam state. */
dplr_lr_status dplr_lr_mlp_set_params(dplr_lr_mlp m, const float* host_params, int64_t count);
dplr_lr_status dplr_lr_mlp_get_params(dplr_lr_mlp m, float* host_params, int64_t count);
/* Checkpoint and resume of training: the whole training state as one byte
 * blob of dplr_lr_mlp_state_bytes() bytes in caller-owned host memory
 * (header with a magic, version and sizes; the packed parameters; the Adam
 * first and second moments and step count; the normalisation sums being
 * accumulated; the set of training charges).  Both calls are synchronous on
 * the network's stream.  set_state returns E_INVALID, changing nothing, for a
 * blob of another size, magic or version, or from a network with another
 * cutoff or output scale.  A step after set_state continues exactly (bitwise)
 * the training that get_state saved. */
int64_t dplr_lr_mlp_state_bytes(void);
dplr_lr_status dplr_lr_mlp_get_state(dplr_lr_mlp m, void* host_state, int64_t bytes);
dplr_lr_status dplr_lr_mlp_set_state(dplr_lr_mlp m, const void* host_state, int64_t bytes);
/* dF for every particle, written (accumulate = 0) or added (accumulate != 0)
 * to ion_dF / wc_dF.  The first call for a larger box grows the cell list
 * (device allocation); later calls allocate nothing.  Neighbours are taken in
 * a fixed order (cells in order, particles of a cell in original-index
 * order), so repeated calls give bitwise equal results.  Each call also
 * records, for dplr_lr_mlp_read_stats, the largest |dF_i|, the largest |F_i|
 * of the arrays it adds to (accumulate != 0; the forces being corrected) and
 * the smallest and largest neighbour count within the cutoff. */
dplr_lr_status dplr_lr_mlp_forward(dplr_lr_mlp m, const double box[3], int64_t n_ion, const float* ion_pos,
                                   const float* ion_q, int64_t n_wc, const float* wc_pos, const float* wc_q,
                                   float* ion_dF, float* wc_dF, int32_t accumulate);
/* One training step on the mean-squared error between dF and the targets:
 * forward, backward (BF16 MFMA, FP32 accumulate), deterministic gradient sum
 * and, when lr > 0, an Adam update (beta 0.9 / 0.999, eps 1e-8).  The target
 * of particle i is target_i - base_i when the base arrays are given (pass
 * the fine-mesh forces as target and the coarse-mesh forces as base to train
 * on the residual), else target_i; both base pointers NULL or both set.
 * *loss (device double) receives the loss before the update; grad_out
 * (device float[count of trainable parameters], may be NULL) the gradient. */
dplr_lr_status dplr_lr_mlp_train_step(dplr_lr_mlp m, const double box[3], int64_t n_ion, const float* ion_pos,
                                      const float* ion_q, int64_t n_wc, const float* wc_pos, const float* wc_q,
                                      const float* ion_target, const float* wc_target, const float* ion_base,
                                      const float* wc_base, float lr, double* loss, float* grad_out);
/* Input normalisation from training configurations: norm_accumulate adds
 * the invariants D_i of one configuration to FP64 sums (sum D, sum D^2, max
 * |D|, count; fixed-order reductions); norm_finish sets mu = mean and
 * inv_sigma = 1 / (std + 1e-6 (max |D| + 1)) in the parameters (device) and
 * clears the sums.  Stream-ordered, no host synchronisation. */
dplr_lr_status dplr_lr_mlp_norm_accumulate(dplr_lr_mlp m, const double box[3], int64_t n_ion, const float* ion_pos,
                                           const float* ion_q, int64_t n_wc, const float* wc_pos,
                                           const float* wc_q);
dplr_lr_status dplr_lr_mlp_norm_finish(dplr_lr_mlp m);
/* The descriptor T (device float [n][128], index 4k + a) in the network's
 * cell order, and that order (device int [n], original particle indices;
 * ions first).  Either output may be NULL. */
dplr_lr_status dplr_lr_mlp_descriptor(dplr_lr_mlp m, const double box[3], int64_t n_ion, const float* ion_pos,
                                      const float* ion_q, int64_t n_wc, const float* wc_pos, const float* wc_q,
                                      float* T_sorted, int32_t* order);
const char* dplr_lr_mlp_last_error(dplr_lr_mlp m);

/* Fallback guard.  The learned form is used only while the inputs look
 * like the training data and periodic audits (a fine-mesh recomputation
 * compared with the learned result) stay within tolerance; otherwise the
 * caller runs the fine plan.  The statistics come from the device:
 *   set_train_charges  the charges present in training (host, at most 16);
 *   check_charges      counts particles whose charge is not one of them;
 *   audit              sum |F - F_ref|^2 and sum |F_ref|^2 over both sets
 *                      (FP64, fixed order), replacing (accumulate = 0) or
 *                      adding to (accumulate != 0) the previous audit sums;
 *   read_stats         synchronises the network's stream and fills
 *                      max_correction, max_force and the neighbour range of
 *                      the last forward (min_neighbours = HUGE_VAL and
 *                      max_neighbours = 0 when it saw no particle, a range
 *                      no bound rejects), unseen_charges of the last check,
 *                      and audit_valid / audit_rel_rmse = sqrt(sum / sum) of
 *                      the audit sums; steps_since_audit is left to the
 *                      caller.
 * dplr_lr_guard_decide is host-only. */
dplr_lr_status dplr_lr_mlp_set_train_charges(dplr_lr_mlp m, const float* host_charges, int32_t count);
dplr_lr_status dplr_lr_mlp_check_charges(dplr_lr_mlp m, int64_t n_ion, const float* ion_q, int64_t n_wc,
                                         const float* wc_q);
dplr_lr_status dplr_lr_mlp_audit(dplr_lr_mlp m, int64_t n_ion, const float* ion_force, const float* ion_ref,
                                 int64_t n_wc, const float* wc_force, const float* wc_ref, int32_t accumulate);
#define DPLR_LR_GUARD_LEARNED 0
#define DPLR_LR_GUARD_FINE 1
#define DPLR_LR_GUARD_AUDIT 2
typedef struct {
  double max_audit_rel_rmse;    /* relative force RMSE allowed at an audit            */
  double max_correction_ratio;  /* max |dF| allowed as a fraction of max |F| (0: off)  */
  int64_t audit_interval;       /* steps between audits (0: only the first)          */
  double min_neighbours, max_neighbours;  /* neighbour-count range seen in training (0: off) */
} dplr_lr_guard_config;
typedef struct {
  int32_t audit_valid;          /* an audit has been taken                           */
  double audit_rel_rmse;        /* its relative force RMSE                           */
  int64_t steps_since_audit;
  double max_correction, max_force;
  double min_neighbours, max_neighbours;
  int32_t unseen_charges;       /* particles whose charge was absent from training   */
} dplr_lr_guard_stats;
dplr_lr_status dplr_lr_mlp_read_stats(dplr_lr_mlp m, dplr_lr_guard_stats* out);
/* *decision = DPLR_LR_GUARD_LEARNED, _FINE or _AUDIT (run both and compare). */
dplr_lr_status dplr_lr_guard_decide(const dplr_lr_guard_config* cfg, const dplr_lr_guard_stats* stats,
                                    int32_t* decision);

#ifdef __cplusplus
}
#endif

#endif /* DPLR_LR_H */

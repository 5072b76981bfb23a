/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector gate engine.
 *
 * The engine holds the state of an n-qubit register as a dense array of 2^n
 * complex amplitudes alpha_j in device memory (Niwa, Matsumoto, Imai,
 * "General-Purpose Parallel Simulator for Quantum Computing", sec. 2.1
 * Registers) and evolves it in place by one-qubit gates and controlled
 * one-qubit gates (sec. 2.2.1 and 2.2.2), never forming the 2^n x 2^n matrix.
 *
 * Conventions used by every entry point:
 *   - Layout: amplitude j (the basis index) is stored at element j, real and
 *     imaginary parts interleaved: double2 for SV_C128, float2 for SV_C64.
 *   - Qubit 0 is the most significant bit of the basis index (sec. 2.2.1), so
 *     qubit q is index bit n-1-q.  sv_qubit_bit() gives its mask.
 *   - Masks (ctrl_mask, mask, value) are masks over basis-index bits.
 *   - A 2x2 matrix U is 8 doubles, row-major, (re, im) interleaved:
 *     u11re, u11im, u12re, u12im, u21re, u21im, u22re, u22im.  It is always
 *     FP64 on the host, read only during the call, and rounded once to FP32
 *     for an SV_C64 state.  It is not checked for unitarity; non-finite
 *     entries are rejected.
 *   - Streams: every state carries a HIP stream (hipStream_t passed as void*;
 *     NULL is the default stream).  Apply calls are enqueued on it and return
 *     at once; calls that return host values (sv_prob, sv_inner, sv_store to
 *     host, sv_sync) wait for the stream.
 *   - Errors: every call returns SV_OK (0) or a negative code; nothing aborts
 *     and no C++ exception crosses the ABI.  Arguments are validated before
 *     any device work is enqueued, so a rejected call leaves the state
 *     unchanged.  An error raised by an earlier asynchronous launch is
 *     reported as SV_EDEVICE by the next call that waits for the stream.
 *   - A handle must not be used from two host threads at once.
 */
#ifndef SV_H
#define SV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SV_OK = 0, SV_EINVAL = -1, SV_ENOMEM = -2, SV_EDEVICE = -3, SV_ENOTSUP = -4 };
/* Element type of a state, given as bytes per amplitude. */
enum { SV_C64 = 8, SV_C128 = 16 };
/* Largest register the ABI accepts (2^36 complex64 amplitudes = 512 GiB,
 * beyond one MI355X's 288 GB; larger n needs the registers split over GPUs). */
enum { SV_MAX_QUBITS = 36 };

typedef struct sv_state sv_state;

/* Basis-index mask of qubit q of an n-qubit register (qubit 0 = MSB). */
static inline uint64_t sv_qubit_bit(int n, int q) { return (uint64_t)1 << (n - 1 - q); }

/* Human-readable text for a status code.  Never NULL. */
const char *sv_strerror(int status);
/* Detail of the calling thread's last device failure ("call: HIP error
 * name"), or "" if none was recorded.  Never NULL. */
const char *sv_last_error(void);

/* ---------------------------------------------------------------- a1 ----
 * Register allocation and set-up (sec. 2.1: 2^n complex amplitudes).
 *
 * sv_create: allocates 2^n * dtype bytes of device memory on the current HIP
 *   device, owned by the handle, and sets the state to |0...0> (alpha_0 = 1).
 *   n in [1, SV_MAX_QUBITS]; dtype SV_C64 or SV_C128.
 *   SV_EINVAL on bad n/dtype/out, SV_ENOMEM if the allocation fails.
 * sv_wrap: makes a handle over caller-owned device memory of 2^n * dtype
 *   bytes at dev_ptr (at least 16-byte aligned).  The caller keeps ownership
 *   and must keep the memory alive until sv_destroy.  The contents are
 *   not touched.
 * sv_destroy: frees the handle and, for sv_create handles, the state memory.
 *   NULL is accepted.
 * sv_set_stream: changes the stream later calls are enqueued on.
 * sv_reset: sets the state to the basis state |basis_index>.
 * sv_load / sv_store: copy 2^n amplitudes of the state's dtype from/to host
 *   memory (on_device = 0) or device memory (on_device = 1).  sv_store to
 *   host waits for the copy.
 */
int sv_create(int n, int dtype, void *hip_stream, sv_state **out);
int sv_wrap(int n, int dtype, void *dev_ptr, void *hip_stream, sv_state **out);
int sv_destroy(sv_state *s);
int sv_set_stream(sv_state *s, void *hip_stream);
int sv_reset(sv_state *s, uint64_t basis_index);
int sv_load(sv_state *s, const void *src, int src_on_device);
int sv_store(const sv_state *s, void *dst, int dst_on_device);
/* Number of qubits, dtype and device pointer of a state (any may be NULL). */
int sv_info(const sv_state *s, int *n, int *dtype, void **dev_ptr);

/* ---------------------------------------------------------------- a2 ----
 * One-qubit gate (sec. 2.2.1): for every pair of basis indices (i0, i1) that
 * differ only in qubit q's bit, with that bit 0 in i0,
 *   alpha_i0 <- u11 alpha_i0 + u12 alpha_i1,
 *   alpha_i1 <- u21 alpha_i0 + u22 alpha_i1   (both from the old values).
 * An exact NOT matrix ([[0,1],[1,0]]) moves amplitudes without arithmetic,
 * so permutation gates are bit-exact.  A diagonal U touches only the
 * amplitudes it changes.  SV_EINVAL: q not in [0,n), NULL or non-finite U.
 */
int sv_apply_1q(sv_state *s, int q, const double U[8]);

/* ---------------------------------------------------------------- a3 ----
 * Controlled one-qubit gate (sec. 2.2.2): rows whose basis index has every
 * bit of ctrl_mask set are transformed as in sv_apply_1q; all other rows are
 * left alone (CTX[j] = I[j]).  Several control bits give the many-controlled
 * gate the same passage mentions.  ctrl_mask = 0 equals sv_apply_1q.
 * SV_EINVAL also when ctrl_mask has bits >= n or contains qubit q's bit.
 */
int sv_apply_ctrl(sv_state *s, uint64_t ctrl_mask, int q, const double U[8]);

/* Exchange of qubits q1 and q2 (a permutation; bit-exact).  q1 == q2 is a
 * no-op.  Used for the final swaps of the QFT circuit (sec. 2.3.2). */
int sv_apply_swap(sv_state *s, int q1, int q2);

/* ---------------------------------------------------------------- a6 ----
 * Reductions (sec. 2.2.3: measurement weights are |alpha_j|^2).  Both
 * accumulate in FP64 for either dtype with a fixed two-stage tree, so the
 * result is bitwise reproducible for a given n and mask.  They wait for the
 * stream.
 * sv_prob: *out = sum over j with (j & mask) == value of |alpha_j|^2.
 *   mask = value = 0 gives the squared norm.  SV_EINVAL if mask has bits
 *   >= n or value has bits outside mask.
 * sv_inner: out[0] + i out[1] = <a|b> = sum_j conj(a_j) b_j.  a and b must
 *   have the same n; their dtypes may differ (mixed c64/c128 fidelity).
 *   b's stream is used after a's pending work is ordered before it.
 */
int sv_prob(sv_state *s, uint64_t mask, uint64_t value, double *out);
int sv_inner(sv_state *a, sv_state *b, double out[2]);

/* ---------------------------------------------------------------- f1 ----
 * Measurement (sec. 2.2.3: draw r in [0, 1), take the integer i with
 * sum_{j<i} |alpha_j|^2 <= r < sum_{j<=i} |alpha_j|^2; the register is then
 * the basis state |i>).
 * sv_measure: *index = that i for the given r (r >= 0 and finite; it is
 *   compared with the unnormalised running sum, so for a normalised register
 *   r is the uniform draw).  If r is not below the total weight, the last
 *   index of nonzero weight; 0 for an all-zero register.  The register is
 *   not modified (sv_reset(s, i) gives the post-measurement state).  The
 *   running sums are FP64 over chunk sums (at most 1024 chunks per level,
 *   down to 4096 amplitudes scanned in order), so only an r within rounding
 *   of a boundary can pick a neighbour of the sequential answer.  Blocking.
 * sv_collapse: projection onto the outcome value of the qubits in mask (a
 *   basis-index mask): amplitudes with (j & mask) == value are scaled by
 *   1/sqrt(p), p = sv_prob(s, mask, value) in FP64, and the rest become 0;
 *   *prob (may be NULL) receives p.  SV_EINVAL for bad masks or p == 0 (the
 *   register is then unchanged).  Blocking.
 * A measurement of the qubits in mask samples i = sv_measure(s, r) and
 * collapses onto value = i & mask, which has probability p.
 */
int sv_measure(sv_state *s, double r, uint64_t *index);
int sv_collapse(sv_state *s, uint64_t mask, uint64_t value, double *prob);

/* Fidelity |<a|b>|^2 / (<a|a> <b|b>) from three FP64 reductions (the
 * fidelity of sec. 5.2, squared and normalised); a and b may differ in
 * dtype.  SV_EINVAL for different n or a zero state.  Waits. */
int sv_fidelity(sv_state *a, sv_state *b, double *fid);

/* Overlap loss 1 - |<phi|psi>|^2 and, if A is not NULL, A = <phi|psi>.
 * Waits. */
int sv_overlap_loss(sv_state *phi, sv_state *psi, double *loss, double A[2]);

/* Waits for the state's stream; reports asynchronous launch errors. */
int sv_sync(sv_state *s);

/* ---------------------------------------------------------------- a9 ----
 * Serialized gate record (88 bytes) and gate-matrix construction.
 * Kinds and parameters (sec. 3.2: one-qubit gates are U_R(theta) U_P1(phi)
 * with U_R(theta) = [[cos, -sin], [sin, cos]], U_P1(phi) = diag(1, e^{i phi});
 * H = U_R(pi/4) U_P1(pi), NOT = U_R(pi/2) U_P1(pi); errors are added to the
 * angles):
 *   SV_G_U    p[0..7] = the matrix
 *   SV_G_H    U_R(pi/4 + p[0]) U_P1(pi + p[1]); exact 1/sqrt(2)[[1,1],[1,-1]]
 *             when both deviations are 0
 *   SV_G_X    U_R(pi/2 + p[0]) U_P1(pi + p[1]); exact [[0,1],[1,0]] when both
 *             deviations are 0
 *   SV_G_Y    sigma_y = [[0,-i],[i,0]]
 *   SV_G_Z    U_P1(pi + p[1]); exact diag(1,-1) when p[1] == 0
 *   SV_G_RK   U_P1(2 pi / 2^iarg + p[1])  (R_k of the QFT, sec. 2.3.2)
 *   SV_G_ROT  U_R(p[0]) U_P1(p[1])
 *   SV_G_SU2  [[a+ib, c+id], [-c+id, a-ib]] with (a,b,c,d) = p[0..3] / |p[0..3]|
 *   SV_G_SWAP exchange of qubits target and target2 (no controls)
 * ctrl is a basis-index control mask as in sv_apply_ctrl.
 */
typedef struct sv_gate {
    int32_t kind;
    int32_t target;
    int32_t target2;
    int32_t iarg;
    uint64_t ctrl;
    double p[8];
} sv_gate;

enum {
    SV_G_U = 0, SV_G_H = 1, SV_G_X = 2, SV_G_Y = 3, SV_G_Z = 4,
    SV_G_RK = 5, SV_G_ROT = 6, SV_G_SU2 = 7, SV_G_SWAP = 8
};

/* Writes the 2x2 matrix of a (non-SWAP) gate record.  SV_EINVAL for SWAP,
 * an unknown kind, iarg outside [0,62] for SV_G_RK, or a zero quaternion. */
int sv_gate_matrix(const sv_gate *g, double U[8]);

/* Applies ng gate records in order.  flags = SV_RUN_PER_GATE (0) launches one
 * kernel per gate.  flags = SV_RUN_FUSED groups gates into fused passes: a
 * pass stages tiles of 2^K amplitudes in LDS and applies every gate whose
 * target bit lies in the tile (diagonal gates and controls may sit on any
 * bit), reordering gates only where they commute (no shared qubit on which
 * either acts non-diagonally); the result equals the per-gate result up to
 * rounding and is bit-exact for permutation-only circuits.  flags =
 * SV_RUN_BLOCKS clusters gates (same reordering rule) into dense blocks of
 * at most "block_qubits" qubits (sv_config_set, default 5) whose matrices
 * are composed on the host in FP64 and applied as by sv_apply_fused
 * (complex64 blocks below 4 qubits are padded with identity qubits to run on
 * MFMA); a gate touching more qubits than that runs alone.  SV_RUN_FUSED and
 * SV_RUN_BLOCKS exclude each other.  Every record is
 * validated before any work is enqueued; on SV_EINVAL *bad_index (if not
 * NULL) receives the index of the first bad record. */
enum { SV_RUN_PER_GATE = 0, SV_RUN_FUSED = 1, SV_RUN_PROFILE = 2, SV_RUN_BLOCKS = 4 };
int sv_run(sv_state *s, const sv_gate *gates, int64_t ng, int flags, int64_t *bad_index);

/* The QFT of sec. 2.3.2 on qubits q0 .. q0 + m - 1 (f2): with x the
 * sub-register index (qubit q0 its most significant bit), amplitude
 * alpha_x becomes beta_y = 2^{-m/2} sum_x e^{+2 pi i x y / 2^m} alpha_x for
 * every value of the other qubits.  flags: SV_QFT_INVERSE applies the
 * inverse (e^{-2 pi i x y / 2^m}); SV_QFT_BITREV leaves out the final bit
 * reversal, so that beta_y lands at the sub-register index with y's m bits
 * reversed (with SV_QFT_INVERSE: the input is read that way).  Runs the
 * textbook circuit (H, controlled R_k, then the bit reversal) as
 * SV_RUN_FUSED: fused passes plus one bit-permutation pass for the swaps.
 * SV_EINVAL if q0 < 0, m < 1, q0 + m > n or flags has another bit.
 * Asynchronous like sv_run. */
enum { SV_QFT_INVERSE = 1, SV_QFT_BITREV = 2 };
int sv_qft(sv_state *s, int q0, int m, int flags);

/* sv_qft on registers of n >= 12 qubits (config "qft_fft" = 1, default)
 * runs as FFT block passes instead of the circuit: blocks of at most 8
 * index bits of the range (12 for the last one when the range starts at
 * index bit 0), as few as that allows and of balanced sizes, from its
 * top, each one HBM sweep (an in-tile DFT
 * written at bit-reversed positions, then the phase of the lower qubits'
 * controlled R_k and the 2^{-t/2} of the block's H gates), leaving the
 * range bit-reversed as the circuit does before its swaps; the bit
 * reversal, where wanted, is the bit-permutation pass.  sv_qft_plan
 * describes the passes (host only): for pass p, out[SV_QFT_PLAN_WORDS p +]
 *   0..5   block low bit, block size t, stage split A (high bits), B, range
 *          low bit, tile position of the block's low bit;
 *   6..17  index bit of each of the 12 tile bits (ascending);
 *   18..21, 22..29  stage 1: tile bit of each register-index bit (4), of
 *          each thread-index bit (8);
 *   30..33, 34..41  the same for stage 2 (-1 if B = 0);
 * a 12-bit block (A = 4, B = 8) has fixed maps and -1 in words 18..41.
 * *count receives the number of passes; at most cap are written.
 * SV_EINVAL unless 12 <= n <= SV_MAX_QUBITS and the range fits. */
enum { SV_QFT_PLAN_WORDS = 42 };
int sv_qft_plan(int n, int q0, int m, int32_t *out, int64_t cap, int64_t *count);

/* With SV_RUN_PROFILE or-ed into flags, sv_run records a HIP event pair on
 * the state's stream around every kernel it launches.  sv_run_profile waits
 * for them and writes the duration in ms of step i to ms[i] and its kind to
 * kind[i] (0 fused pass, 1 swap, 2 single gate, 3 dense block) for
 * i < min(cap, *count);
 * *count is the number of steps of the last profiled run (0 if none).  A
 * later sv_run overwrites the record. */
int sv_run_profile(sv_state *s, double *ms, int32_t *kind, int64_t cap, int64_t *count);

/* The fused plan sv_run(SV_RUN_FUSED) would execute for an n-qubit register
 * of the given dtype, computed on the host only (no device call): order[i]
 * is the index of the i-th gate executed, pass_of[i] the pass it runs in
 * (-1 for a SWAP run as its own kernel), tile_mask[p] the basis-index bits
 * held in the tiles of pass p, *npasses the number of passes.  order and
 * pass_of hold ng entries, tile_mask ng entries at most; each may be NULL.
 * SV_EINVAL for a bad gate list (as sv_run) or bad n/dtype. */
int sv_plan_fused(int n, int dtype, const sv_gate *gates, int64_t ng, int64_t *order, int32_t *pass_of,
                  uint64_t *tile_mask, int64_t *npasses);

/* Source text of the specialised kernel of fused pass `pass` of a gate list
 * (host only, no device needed): *len receives its length; if buf is not
 * NULL, up to cap - 1 characters and a terminating NUL are copied.
 * SV_EINVAL for invalid arguments or pass out of range. */
int sv_jit_source(int n, int dtype, const sv_gate *gates, int64_t ng, int64_t pass, char *buf, int64_t cap,
                  int64_t *len);

/* Host model of SV_RUN_FUSED (host only, no device needed): the gate list is
 * planned and rewritten exactly as sv_run would for an n-qubit register of
 * the given dtype (tile shapes, pair fusion, rotation split and phase runs,
 * per the configuration), and the resulting ops are applied tile by tile in
 * FP64 to amps (2^n complex128 values, interleaved re, im, in place), with
 * the meaning the pass kernels give them.  For tests of the host-side
 * rewrites (evolution steps of sec. 2.2.1-2.2.2).  SV_EINVAL for n outside
 * 1..24, a bad dtype, a bad gate list or NULL amps. */
int sv_model_fused(int n, int dtype, const sv_gate *gates, int64_t ng, double *amps);

/* The dense-block plan of SV_RUN_BLOCKS with blocks of at most kmax qubits
 * (1..6), host only.  *nsteps receives the number of steps; for the first
 * min(cap, *nsteps) steps, info[8i..8i+7] = {0, k, qubits[0..5] (-1
 * padded)} for a block (qubits ascending, qubits[0] the most significant
 * bit of the block index) or {1, gate index, -1...} for a gate run alone,
 * and mats (if not NULL) holds the block's 2^k x 2^k complex matrix,
 * row-major (re, im), at offset i * 2 * 4^kmax doubles.  The planner's
 * padding of small complex64 blocks is not shown. */
int sv_plan_blocks(int n, const sv_gate *gates, int64_t ng, int kmax, int64_t *nsteps, int32_t *info, double *mats,
                   int64_t cap);

/* ---------------------------------------------------------------- a5 ----
 * Dense k-qubit block: the definition of sec. 2.2.1 with a 2^k x 2^k
 * complex matrix M in place of the 2x2 U.  For every basis index whose bits
 * of qubits[0..k-1] are 0, the 2^k amplitudes of that group are multiplied
 * by M; block row/column index i has qubits[0] as its most significant bit.
 * M is FP64 on the host, row-major, (re, im) interleaved, read during the
 * call and rounded once to FP32 for a complex64 register.  k in [1, 6],
 * distinct qubits.  complex64 blocks with k = 4 or 5 (n >= 12) run on FP32
 * MFMA through the real embedding [[Re M, -Im M], [Im M, Re M]]; other
 * cases run on the vector units.  Not checked for unitarity.  SV_EINVAL
 * for bad k, qubits or non-finite entries. */
int sv_apply_fused(sv_state *s, int k, const int qubits[], const double *M);

/* Derivative of a gate's matrix with respect to one of its angle
 * deviations: which = 0 for p[0] (the rotation angle of SV_G_H, SV_G_X,
 * SV_G_ROT), which = 1 for p[1] (the phase angle of SV_G_H, SV_G_X,
 * SV_G_ROT, SV_G_Z, SV_G_RK).  d/dtheta U_R(theta) = [[-sin, -cos], [cos,
 * -sin]], d/dphi U_P1(phi) = diag(0, i e^{i phi}) (sec. 3.2 angles).
 * SV_EINVAL if the kind has no such parameter. */
int sv_gate_dmatrix(const sv_gate *g, int which, double D[8]);

/* ---------------------------------------------------------------- a8 ----
 * Adjoint gradient of loss = 1 - |<phi|psi_L>|^2 with respect to one angle
 * deviation per gate, psi_L = U_L ... U_1 psi_0 (the gate list applied in
 * order, as sv_run).  On entry psi holds psi_L and lambda holds phi (same n
 * and dtype, distinct states).  The sweep uncomputes: for g = L..1,
 * psi <- U_g^dagger psi, partial_g = <lambda| dU_g |psi>, lambda <-
 * U_g^dagger lambda; so no intermediate state is stored and on return psi
 * holds psi_0 (up to rounding) and lambda holds U^dagger phi.
 *   dparam[g]: -1 no parameter, 0 the p[0] deviation, 1 the p[1] deviation
 *              (see sv_gate_dmatrix); host array of ng int32.
 *   grad[g]:   host array of ng doubles, -2 Re(conj(A) partial_g) (0 where
 *              dparam[g] < 0).  Partials accumulate in FP64 for both dtypes.
 *   a_out:     A = <phi|psi_L> if not NULL.
 * Controls are exact: dU_g vanishes on rows with a control bit 0.  Runs on
 * psi's stream (lambda's pending work is ordered before it) and waits.
 * SV_EINVAL for a bad gate list, dparam naming a parameter the kind lacks,
 * or a SWAP with a parameter. */
int sv_adjoint(sv_state *psi, sv_state *lambda, const sv_gate *gates, int64_t ng, const int32_t *dparam,
               double *grad, double a_out[2]);

/* ---------------------------------------------------------------- a7 ----
 * Batched noisy trajectories (sec. 3 error model; the robustness studies of
 * sec. 4.3.1 and 5.3.1 average many runs with different random draws).
 *
 * svb_create: B registers of n qubits and one dtype, stored back to back in
 *   device memory owned by the batch (B * 2^n * dtype bytes).  hip_stream is
 *   the caller's stream: a run waits for its pending work and later work on
 *   it waits for the run.  The batch also owns a private stream on which
 *   its HIP graph is captured and replayed.
 * svb_run_noisy: every register r starts at |0...0> (or, after
 *   svb_set_start(b, SVB_START_KEEP), from its current contents) and runs
 *   trajectory t = traj_offset + r of the gate list init, then iters
 *   repetitions of iter, with
 *     - operational error: Gaussian N(0, sigma^2) deviations on the angles
 *       of every gate (H, X, SV_G_ROT: rotation and phase angle; Z, R_k:
 *       phase angle; explicit matrices: none);
 *     - depolarizing error: after each gate, each qubit it touches (target
 *       and controls) independently gets sigma_x, sigma_y or sigma_z with
 *       probability p/3 each.
 *   Draws: Philox4x32-10, key = seed, counter = (t, g, slot, 0) with g the
 *   gate's position in the whole sequence; slot 0 gives the angles by
 *   Box-Muller on (r0, r1); the i-th touched qubit (ascending qubit order)
 *   reads words 2(i%2) (event iff r < floor(p 2^32)) and 2(i%2)+1 (type
 *   (3 r) >> 32) of slot 1 + i/2.
 *   Every multi-qubit gate must be diagonal (controlled phases); runs of
 *   one-qubit gates and Paulis are folded into one matrix per qubit and
 *   trajectory, composed in FP64 and rounded once to the register dtype.
 *   prob[r] = |alpha_target|^2 and norm2[r] = sum |alpha|^2 of register r
 *   after the run (host arrays of B doubles, either may be NULL).  Waits.
 *   SV_ENOTSUP for a non-diagonal multi-qubit gate or a SWAP; SV_EINVAL for
 *   bad gates, sigma < 0, p outside [0, 1], a target with bits >= n, or
 *   trajectory ids / gate positions beyond 32 bits.
 * svb_set_group: registers per pass launch (0 = all B; must divide B).
 *   Smaller groups keep a group's registers resident in the device's last
 *   level cache across the passes of a run.  Tuning only; results do not
 *   change.
 * svb_state: device pointer of register reg.
 * svb_last_run_ms: device time of the last svb_run_noisy (HIP events around
 *   the graph launch). */
typedef struct svb_batch svb_batch;
int svb_create(int n, int batch, int dtype, void *hip_stream, svb_batch **out);
int svb_destroy(svb_batch *b);
int svb_set_group(svb_batch *b, int regs_per_launch);
int svb_state(svb_batch *b, int reg, void **dev_ptr);
/* Qubits, registers and dtype of a batch (any output may be NULL), and its
 * current registers per launch. */
int svb_info(const svb_batch *b, int *n, int *batch, int *dtype);
int svb_get_group(const svb_batch *b, int *regs_per_launch);
int svb_run_noisy(svb_batch *b, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter, int iters,
                  double sigma, double p, uint64_t seed, uint64_t traj_offset, uint64_t target_index, double *prob,
                  double *norm2);
int svb_last_run_ms(const svb_batch *b, double *ms);

/* svb_set_start: where the registers of later svb_run_noisy calls start.
 *   SVB_START_ZERO (default): every register is reset to |0...0>.
 *   SVB_START_KEEP: every register starts from its current contents, as
 *   the caller wrote them through svb_state (the QFT experiment of
 *   sec. 5.1.1 starts from the register Shor's step 3(c) leaves).  A run
 *   overwrites the registers, so the caller writes them again before the
 *   next run.
 *   SV_EINVAL for another mode. */
enum { SVB_START_ZERO = 0, SVB_START_KEEP = 1 };
int svb_set_start(svb_batch *b, int mode);

/* svb_set_noise_kinds: depolarizing draws follow only the gates whose kind
 *   k (SV_G_*) has bit k set in depolarize_kinds (default: all kinds).
 *   Sec. 5.1.1 depolarizes the whole register each time an R_d is applied:
 *   a gate list says so with an explicit identity (SV_G_U) on every qubit
 *   after each R_d and depolarize_kinds = 1 << SV_G_U.  Draw counters do
 *   not move: a gate keeps its position g.  SV_EINVAL for a NULL batch. */
int svb_set_noise_kinds(svb_batch *b, uint32_t depolarize_kinds);

/* Per-register reductions over a whole batch, one launch each (the
 * robustness experiments of sec. 4.3.1, 5.1.1 and 5.3.1 evaluate every
 * trajectory).  They run on the batch's caller stream and wait.
 * svb_fidelity: for every register r, fid[r] = |<a_r|b_r>|^2 / (<a_r|a_r>
 *   <b_r|b_r>) (the fidelity of sec. 5.2, squared and normalised; 0 for a
 *   zero register) and overlap[2r], overlap[2r+1] = <a_r|b_r> (either
 *   output may be NULL, not both), accumulated in FP64 with a fixed tree.
 *   a and b have the same n and B; their dtypes may differ.  b's pending
 *   work is ordered before the launch.  SV_EINVAL otherwise or for a == b.
 * svb_measure: for every register r, index[r] = the measurement of
 *   sec. 2.2.3 with draw r_draw[r] (host arrays of B entries): the smallest
 *   i with sum_{j<=i} |alpha_j|^2 > r_draw[r], the running sum in FP64 over
 *   256 contiguous chunk sums and then element by element; if r_draw[r]
 *   reaches the total, the last index of nonzero weight; 0 for an all-zero
 *   register.  Registers are not modified.  SV_EINVAL for a negative or
 *   non-finite draw. */
int svb_fidelity(svb_batch *a, svb_batch *b, double *fid, double *overlap);
int svb_measure(svb_batch *b, const double *r_draw, uint64_t *index);

/* svb_fidelity_noalloc: svb_fidelity for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): it calls no hipMalloc, hipFree or
 * allocating library routine.  a and b are device pointers to nregs
 * registers of 2^n amplitudes each, stored back to back (dtypes dtype_a,
 * dtype_b; they may differ).  Outputs are device pointers: fid[r] and
 * overlap[2r], overlap[2r+1] as in svb_fidelity (either may be NULL, not
 * both; the same FP64 tree).  The call is asynchronous on hip_stream.
 * Partial sums go to a library-owned device array of SVB_NOALLOC_MAX_REGS
 * * 4 doubles (512 KiB), one per GPU, kept until the process ends and
 * shared by every call on that GPU: calls that overlap in time on one GPU
 * race on it (serialise them, e.g. on one stream).  Every partial is
 * written before it is read, so nothing needs clearing between calls.
 * SV_EINVAL for n outside 1..SV_MAX_QUBITS, nregs outside
 * 1..SVB_NOALLOC_MAX_REGS, a bad dtype or NULL a, b; SV_EDEVICE for a
 * device error. */
enum { SVB_NOALLOC_MAX_REGS = 16384 };
int svb_fidelity_noalloc(int n, int nregs, int dtype_a, const void *a, int dtype_b, const void *b, double *fid,
                         double *overlap, void *hip_stream);

/* svb_trajectory_gates: trajectory traj of svb_run_noisy's error model
 *   (same gate sequence init, then iters x iter; same draws from seed) as an
 *   explicit gate list for the plain per-gate path (sv_run): each gate keeps
 *   its kind with the drawn deviations added to p[0] / p[1] as svb_run_noisy
 *   adds them, and is followed by the Pauli gates (SV_G_X, SV_G_Y, SV_G_Z,
 *   exact) that its touched qubits drew, in ascending qubit order, when its
 *   kind's bit is set in depolarize_kinds.  Multi-qubit gates need not be
 *   diagonal here.  Host only, no device call.  Writes min(cap, *count)
 *   records to out (may be NULL when cap = 0); *count receives the length
 *   of the whole list.  SV_EINVAL for bad gates, n, sigma, p, traj >= 2^32 or
 *   more than 2^32 gates; SV_ENOTSUP for a SWAP. */
/* svb_plan: the program svb_run_noisy builds for these gates, computed on
 *   the host only (no device call): *npasses fused passes (each one launch
 *   over the registers) and *nslots per-register matrix slots (folded runs
 *   of one-qubit gates and Paulis, sec. 3).  SV_EINVAL as svb_run_noisy. */
int svb_plan(int n, int dtype, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter, int iters,
             int64_t *npasses, int64_t *nslots);
/* svb_jit_source: source text of the specialised kernel of pass `pass` of
 *   that program (host only), as sv_jit_source. */
int svb_jit_source(int n, int dtype, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter,
                   int iters, int64_t pass, char *buf, int64_t cap, int64_t *len);

int svb_trajectory_gates(int n, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter, int iters,
                         double sigma, double p, uint64_t seed, uint64_t traj, uint32_t depolarize_kinds,
                         sv_gate *out, int64_t cap, int64_t *count);

/* ---------------------------------------------------------------- f4 ----
 * Shor's factoring algorithm as sec. 5.1 runs it for 14-15-bit N: the
 * modular exponentiation of step 3(c) is computed classically, the register
 * holds only the 2l-qubit second register (l = bit length of N), the QFT
 * and the measurement of step 3(d) run on it, and steps 4-5 run on the
 * host.
 *
 * sv_shor_prepare: writes the register s (m = s's qubit count) left by step
 *   3(c) and a measurement of the first register: with v = x^a_star mod N,
 *   the equal superposition of every a in [0, 2^m) with x^a mod N = v, each
 *   amplitude 1/sqrt(count) (computed in FP64, rounded once to the
 *   register dtype).  Drawing a_star uniformly gives v the law of the
 *   first-register measurement.  *count (may be NULL) receives the number
 *   of such a.  Waits for the device.  SV_EINVAL unless 2 <= N < 2^32 and
 *   a_star < 2^m.
 *
 * sv_shor_classical: steps 4-5 for one measured y of an m-qubit register.
 *   Step 4 takes the coprime k/r, 0 < k < r < N, with
 *   |y/2^m - k/r| <= 1/2^(m+1) (tested exactly in integers) from the
 *   continued-fraction convergents of y/2^m; the iteration fails if there
 *   is none, if x^r != 1 (mod N), if r is odd or if x^(r/2) = +-1; else
 *   step 5 gives gcd(N, x^(r/2) - 1), or gcd(N, x^(r/2) + 1) when the first
 *   is trivial.  flags = SV_SHOR_IMPROVED adds the four checks of sec. 5.1,
 *   tried in this order, the first factor found ending the iteration:
 *     1 neighbour y: y has no k/r: the first of y+1, y-1, y+2, y-2 that has
 *       one gives r;
 *     then, only while x^r != 1 (mod N):
 *     2 GCD: for even r, gcd(N, x^(r/2) -+ 1) whatever x^r is;
 *     3 small factor: the multiples c r, c = 2, 3, ... while c r < N; the
 *       first with x^(c r) = 1 goes through the failure tests and step 5;
 *     4 LCM: lcm(r_prev, r) through the same tests, r_prev (0: none) being
 *       the candidate of the previous run of the same experiment.
 *   out: factor (0 on failure), stage (SV_SHOR_* that gave it, or
 *   SV_SHOR_FAIL), r (step 4's candidate, 0 if none), checks[i] =
 *   {successes, failures} of check i+1 in this call.  Host code only.
 *   SV_EINVAL unless 2 <= N < 2^32, 1 <= m <= 62, y < 2^m and flags is 0
 *   or SV_SHOR_IMPROVED.
 *
 * sv_shor_factor: repeats steps 1-5 until a factor is found, at most
 *   max_iters times, with the caller's random choices for run i: x[i] in
 *   [1, N-1] (step 1), a_star[i] < 2^m (the first-register outcome, as in
 *   sv_shor_prepare) and u[i] in [0, 1) (sv_measure's draw for y).  Step 2
 *   ends the run with gcd(x, N) when it exceeds 1; otherwise the run is
 *   sv_shor_prepare, sv_qft over the whole register with SV_QFT_BITREV,
 *   sv_measure, whose index read with its m bits reversed is y (the law of
 *   measuring after the swaps, without the bit-permutation pass), and
 *   sv_shor_classical (r_prev carried between runs).  The register must
 *   have exactly 2l qubits.  y_out (NULL or max_iters entries) receives
 *   each run's y (all ones for a run ended by step 2).  res: iterations
 *   (runs used, 0 if no factor within max_iters), factor, stage, checks
 *   summed over the runs.  SV_EINVAL for a bad argument or draw. */
enum {
    SV_SHOR_FAIL = -1,
    SV_SHOR_PLAIN = 0,
    SV_SHOR_NEIGHBOR = 1,
    SV_SHOR_GCD = 2,
    SV_SHOR_SMALL = 3,
    SV_SHOR_LCM = 4,
    SV_SHOR_GCDX = 5
};
enum { SV_SHOR_IMPROVED = 1 };
typedef struct {
    uint64_t factor;
    uint64_t r;
    int32_t stage;
    int32_t checks[4][2];
} sv_shor_outcome;
typedef struct {
    int64_t iterations;
    uint64_t factor;
    int32_t stage;
    int32_t checks[4][2];
} sv_shor_result;
int sv_shor_prepare(sv_state *s, uint64_t N, uint64_t x, uint64_t a_star, uint64_t *count);
int sv_shor_classical(uint64_t N, uint64_t x, uint64_t y, int m, int flags, uint64_t r_prev, sv_shor_outcome *out);
int sv_shor_factor(sv_state *s, uint64_t N, const uint64_t *x, const uint64_t *a_star, const double *u,
                   int64_t max_iters, int flags, uint64_t *y_out, sv_shor_result *res);

/* ------------------------------------------------------------------------
 * Engine tuning, process-wide, read by later calls (the autotuner below
 * searches them):
 *   "fused_tile_bits_c128"  log2 amplitudes per LDS tile of a fused pass,
 *                           complex128 (1..12, default 12 = 64 KiB)
 *   "fused_tile_bits_c64"   the same for complex64 (1..13, default 12)
 *   "fused_low_bits"        lowest index bits always in a tile, giving
 *                           contiguous HBM runs (1..12, default 4)
 *   "fused_max_ops"         gates per fused pass (1..4096, default 512)
 *   "block_qubits"          largest dense block of SV_RUN_BLOCKS (1..6, default 5)
 *   "fused_jit"             1 (default): each fused pass runs as a kernel
 *                           specialised to its op list, compiled with hipRTC
 *                           for gfx950 on first use and cached for the life of
 *                           the process (by kernel source, per device); 0:
 *                           the generic pass kernel.  Compilation failures
 *                           return SV_EDEVICE with the compiler log in
 *                           sv_last_error().
 *   "fused_pairs"           1 (default; with fused_jit): inside a pass, runs
 *                           of ops on at most two register slots (no
 *                           out-of-tile controls) are multiplied into one
 *                           2x2 or 4x4 matrix in FP64 when that needs fewer
 *                           multiply-adds; permutation-only runs are never
 *                           composed, so they stay bit-exact.  0: off.
 *   "swap_runs"             1 (default): in SV_RUN_FUSED, two or more
 *                           consecutive SWAP steps whose product is an
 *                           involution on the index bits (the bit reversal
 *                           that ends the QFT) run as one bit-permutation
 *                           pass; 0: one kernel per swap.  Both move
 *                           amplitudes only (bit-exact).
 *   "perm_low_bits"         lowest index bits per tile of that pass on a
 *                           complex128 register (1..6, default 6):
 *                           contiguous runs of 2^b amplitudes; a tile holds
 *                           them and their images.  Tiles of up to 2^10
 *                           amplitudes exchange through two LDS tiles,
 *                           larger ones (up to 2^12, 64 KiB) through one LDS
 *                           tile and registers.
 *   "perm_low_bits_c64"     the same for complex64 registers (1..6,
 *                           default 5)
 *   "gate_pairs_min_bit"    per-gate kernels (sv_apply_1q, sv_apply_ctrl,
 *                           SV_RUN_PER_GATE): target bits at or above it go
 *                           to the pair kernel, whose two loads per pair are
 *                           whole runs of lines; lower ones to the
 *                           wavefront-shuffle kernel (0..6, default 0: the
 *                           pair kernel for every bit, measured faster)
 *   "gate_cached_low"       1 (default): a target bit inside a 128-byte
 *                           line (both halves of a pair share lines) is
 *                           applied with cached loads and stores, so the
 *                           second access finds the line the first brought
 *                           in; 0: nontemporal like the other bits
 *   "gate_spread_bits"      per-gate kernels whose fixed index bits (the
 *                           controls; for a diagonal gate also a target
 *                           with one entry 1) include byte address bit
 *                           10, 11, 12, 20 or 21: the low k bits of the
 *                           workgroup index become its high bits, so
 *                           workgroups that run together spread over the
 *                           register (0..8, default 4; 0 keeps the plain
 *                           order, whose concurrent accesses then reach
 *                           fewer memory channels: controlled phases and
 *                           CNOTs there ran at 0.55-0.63 of the HBM peak,
 *                           0.70-0.80 with the spread)
 *   "perm_workgroups"       workgroups of that pass, each walking tile
 *                           pairs (1..2^20, default 16384)
 *   "fused_plan_search"     1 (default): the planner also tries every
 *                           window of contiguous qubits as a pass's tile
 *                           and keeps the schedule with the most gate
 *                           work; 0: first-come tile bits only
 *   "fused_reg_bits"        register bits (amplitudes 2^b per thread) of
 *                           specialised passes (2..4, default 4; the
 *                           generic kernel always uses 4)
 *   "fused_jit_max_ops"     longest op list of a pass that is compiled
 *                           into a specialised kernel (1..4096, default
 *                           384); with 4 register bits, longer passes run
 *                           on the generic kernel, whose compile cost is
 *                           nil (compile time grows faster than the list)
 *   "qft_fft"               sv_qft on n >= 12 qubits: 1 (default) FFT
 *                           block passes, 0 the circuit as fused passes
 *   "mfma_workgroups"       complex64 blocks on MFMA: workgroups of the
 *                           grid, which walk the column blocks of 32
 *                           groups (every block bit >= 5) or, twice as
 *                           many, the LDS tiles
 *                           (1..2^20, default 256, one per compute unit of
 *                           an MI355X: measured faster than other counts)
 *   "fused_mfma"            specialised complex64 passes of single
 *                           registers: 1 runs dense one-qubit ops and
 *                           composed 4x4 ops on the matrix cores
 *                           (v_mfma_f32_4x4x1_16b, FP32, every product
 *                           useful), 0 (default) on the vector units
 *   "batch_mfma"            the same for the passes of trajectory batches
 *                           (svb_run_noisy), whose per-trajectory matrices
 *                           stay dense: 1 (default), 0 vector units
 *   "batch_const_bits"      specialised passes of trajectory batches: 1
 *                           (default) compiles each pass's tile bits into
 *                           its kernel (one kernel per tile shape, index
 *                           offsets as constants); 0 reads them at run time
 *                           so that tile shapes share kernels
 *   "batch_waves"           specialised passes of trajectory batches:
 *                           registers budgeted for at least this many
 *                           waves per SIMD (0..8; default 4, measured
 *                           faster than the compiler's choice, 0)
 *   "fused_rotations"       specialised passes whose matrices are all
 *                           known on the host: 1 (default) applies each
 *                           unitary one-qubit matrix as phase, real
 *                           rotation with one unit coefficient per row (4
 *                           multiply-adds per amplitude pair instead of 16),
 *                           phase, and merges the phases of a pass into the
 *                           fewest runs (one complex multiply per amplitude
 *                           and run); 4x4 composition is then off.  0: off.
 * SV_EINVAL for an unknown key, a value out of range, or NULL. */
int sv_config_set(const char *key, int value);
int sv_config_get(const char *key, int *value);

/* ------------------------------------------------------------------------
 * Autotuner of the tile and fusion widths above (not in the paper, whose
 * SMP code has no such knobs).  It times the caller's own workload
 * on the device under candidate settings and leaves the fastest one set:
 * coordinate descent from the current values, one knob at a time over its
 * candidates, a change kept only when at least 1% faster; each candidate is
 * timed as the median of reps runs (kernel time from HIP events on the
 * launch stream) after one untimed run that compiles its pass kernels.
 * sv_tune_fused: the gate list run as SV_RUN_FUSED on s (its contents are
 *   overwritten by the timed runs).  Knobs: fused_tile_bits_c128 (10..12)
 *   or fused_tile_bits_c64 (11..13), fused_low_bits (3..5),
 *   fused_reg_bits (3..4) and, for complex64, fused_mfma (0, 1).
 * svb_tune_group: svb_run_noisy of the given program (sigma = 1e-2,
 *   p = 1e-4, seed 1; use a few iterations) on b, over registers per launch
 *   = 0 (all) and B/2, B/4, ... down to 32 (divisors of B only; reported as
 *   "svb_group" and set with svb_set_group), then over "batch_waves" (0, 3,
 *   4) at the chosen group (set with sv_config_set).
 * res: the knobs searched, their starting and chosen values, the median ms
 *   at the start and at the choice, and how many settings were timed.
 *   SV_EINVAL for bad arguments; errors of the timed runs are returned (the
 *   starting values are restored on SV_EDEVICE).  Process-wide settings:
 *   every later call uses them. */
enum { SV_TUNE_MAX_KEYS = 8 };
typedef struct sv_tune_result {
    int32_t nkeys;
    int32_t tried;
    char key[SV_TUNE_MAX_KEYS][24];
    int32_t start[SV_TUNE_MAX_KEYS];
    int32_t best[SV_TUNE_MAX_KEYS];
    double start_ms;
    double best_ms;
} sv_tune_result;
int sv_tune_fused(sv_state *s, const sv_gate *gates, int64_t ng, int reps, sv_tune_result *res);
int svb_tune_group(svb_batch *b, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter, int iters,
                   int reps, sv_tune_result *res);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */

// Internal declarations of the gfx950 state-vector engine (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sv.h"

struct sv_state {
    int n;
    int dtype;          // SV_C64 or SV_C128
    void *d;            // 2^n amplitudes
    bool owned;         // d allocated by sv_create
    hipStream_t stream;
    int device;
    double *d_red;      // reduction partials (device), SVI_RED_SLOTS doubles
    double *h_red;      // pinned host landing buffer, 4 doubles
    struct FusedBuffers *fused;  // pass descriptors of the fused engine (lazy)
    struct RunProfile *prof;     // per-step event pairs of the last profiled sv_run (lazy)
    struct AdjointBuffers *adj;  // per-gate partials of the adjoint sweep (lazy)
    void *work;                  // device scratch of sv_shor_prepare (lazy, grown on demand)
    size_t work_cap;
};

// Per-step timing of a profiled sv_run: one event pair per launched step.
enum StepKind { STEP_FUSED_PASS = 0, STEP_SWAP = 1, STEP_GATE = 2, STEP_BLOCK = 3 };
struct RunProfile {
    std::vector<hipEvent_t> ev;  // 2 per step, reused across runs
    std::vector<int> kind;
    size_t used = 0;
};
// Records the start event of a new step (when profiling) and returns its slot,
// or -1 when not profiling or on error.
int svi_prof_begin(sv_state *s, bool on, int kind);
void svi_prof_end(sv_state *s, int slot);
void svi_prof_release(sv_state *s);
void svi_release_adjoint(sv_state *s);

// Fixed reduction geometry: stage 1 uses at most this many blocks, so the
// summation tree depends only on the element count.
constexpr int SVI_RED_BLOCKS = 1024;
constexpr int SVI_RED_THREADS = 256;
constexpr int SVI_RED_SLOTS = 2 * SVI_RED_BLOCKS + 8;

// Matrix in the element type of the state.
template <typename R>
struct Mat2 {
    R m[8];
};

// Up to 64 ascending bit positions at which zero bits are inserted into an
// enumeration counter to form a basis index (controls + target).
struct BitSpec {
    uint8_t pos[64];
    int count;
};

// Gate classes, decided on the host from the exact matrix entries.
enum GateClass { GC_DENSE = 0, GC_DIAG = 1, GC_PERM = 2 };

GateClass svi_classify(const double U[8]);
bool svi_finite(const double U[8]);
int svi_gate_matrix(const sv_gate *g, double U[8]);
int svi_gate_dmatrix(const sv_gate *g, int which, double D[8]);

// Launchers (return hipSuccess or the launch error).
hipError_t svi_launch_reset(sv_state *s, uint64_t idx);
// Sets N amplitudes at d to the basis state |idx> (also used for every
// register of a batch with N = B * 2^n and idx covering register 0 only).
hipError_t svi_launch_reset_ptr(void *d, int dtype, uint64_t N, uint64_t idx, hipStream_t st);
hipError_t svi_launch_gate(sv_state *s, uint64_t ctrl, int q, const double U[8]);
hipError_t svi_launch_swap(sv_state *s, int q1, int q2);
// Two-stage FP64 reductions: stage-1 partials go to part (2*SVI_RED_BLOCKS
// doubles), the result to out (1 or 2 doubles), both device memory.
hipError_t svi_launch_prob(sv_state *s, uint64_t mask, uint64_t value, double *part, double *out);
hipError_t svi_launch_inner(const sv_state *a, const sv_state *b, hipStream_t st, double *part, double *out);
hipError_t svi_launch_chunk_sums(sv_state *s, uint64_t lo, uint64_t chunk, int nch, double *part);
hipError_t svi_launch_collapse(sv_state *s, uint64_t mask, uint64_t value, double scale);
// new[j] = old[F(j)], F applying the bit map f (an involution on the n index
// bits) to j; one pass (perm.hip).
hipError_t svi_launch_bitperm(sv_state *s, const int *f);
// The QFT over index bits [lo, lo + m) as FFT block passes, output left in
// bit-reversed order over the range (sign +1: QFT, -1: inverse); needs
// n >= 12 (svi_qft_fft_ok).
bool svi_qft_fft_ok(const sv_state *s);
int svi_qft_fft(sv_state *s, int lo, int m, int sign);

// Ascending positions of the set bits of mask.
BitSpec svi_bits_of(uint64_t mask);

// Host-side helpers shared by the API files.
int svi_status_from_hip(hipError_t e);
// Records "what: hip error name" as the calling thread's last error detail
// and returns the status for e (SV_OK when e == hipSuccess).
int svi_fail(const char *what, hipError_t e);
// Records a text detail and returns status.
int svi_fail_text(const char *what, int status);

// A validated gate of a gate list, with its matrix built.
struct PreparedGate {
    int kind;  // SV_G_SWAP or a matrix kind
    int q, q2;
    uint64_t ctrl;
    double U[8];
    GateClass cls;
    int32_t slot = -1;  // batched programs: matrix comes from this table row
};

// Tunable engine parameters (set through sv_config_set).
struct SviConfig {
    int fused_tile_bits_c128;  // log2 amplitudes per LDS tile
    int fused_tile_bits_c64;
    int fused_low_bits;        // contiguous low index bits always in a tile
    int fused_max_ops;         // gates per fused pass
    int block_qubits;          // largest dense block of SV_RUN_BLOCKS
    int fused_jit;             // 1: fused passes run as specialised kernels (hipRTC)
    int fused_pairs;           // specialised kernels: compose runs on <= 2 register slots
    int swap_runs;             // fused runs: involutive runs of swaps as one bit permutation
    int perm_low_bits;         // bit permutation of complex128 registers: lowest bits per tile (contiguous runs)
    int perm_workgroups;       // bit permutation: grid size (workgroups walk the tile pairs)
    int fused_plan_search;     // planner: also try windows of contiguous qubits per pass
    int fused_reg_bits;        // specialised passes: register bits per thread
    int fused_jit_max_ops;     // specialised passes: longest op list compiled
    int qft_fft;               // sv_qft: 1 = FFT block passes (fft.hip), 0 = the circuit
    int mfma_workgroups;       // LDS-free MFMA blocks: grid size (wavefronts walk column blocks)
    int fused_mfma;            // specialised complex64 passes: dense ops on v_mfma_f32_4x4x1_16b
    int fused_rotations;       // specialised passes: unitary 2x2 as phase, real rotation, phase
    int perm_low_bits_c64;     // bit permutation of complex64 registers: lowest bits per tile
    int gate_pairs_min_bit;    // per-gate kernels: lowest target bit taken by the pair kernel (below: shuffles)
    int gate_cached_low;       // per-gate kernels: cached accesses for target bits inside a line
    int batch_mfma;            // specialised complex64 passes of trajectory batches: dense ops on MFMA
    int batch_waves;           // their register budget: at least this many waves per SIMD (0: compiler's choice)
    int batch_const_bits;      // their tile bits compiled in (a kernel per tile shape) instead of read at run time
    int gate_spread_bits;      // per-gate kernels with fixed index bits at byte address bits 10..12: block-order spread
};
SviConfig &svi_config();

// Validates a gate list against n and builds every matrix; on failure *bad
// (if not NULL) is the first bad index.
int svi_prepare(int n, const sv_gate *gates, int64_t ng, std::vector<PreparedGate> &out, int64_t *bad);

// Fused execution of a validated gate list (SV_RUN_FUSED).
int svi_run_fused(sv_state *s, const PreparedGate *gates, int64_t ng, bool prof);
void svi_release_fused(sv_state *s);

// Dense 2^k x 2^k block on qubits qs (qs[0] the most significant bit).
int svi_apply_dense(sv_state *s, int k, const int *qs, const double *M);
// Execution of a validated gate list as dense blocks (SV_RUN_BLOCKS).
int svi_run_blocks(sv_state *s, const PreparedGate *gates, int64_t ng, bool prof);

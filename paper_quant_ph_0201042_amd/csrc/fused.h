// Pass and op descriptors of the fused engine, shared by the single-register
// path (fused.hip) and the batched trajectory engine (batched.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sv_internal.h"

enum OpKind : int32_t {
    OP_DENSE = 0,
    OP_PERM = 1,
    OP_DIAG = 2,
    OP_REMAP = 3,
    OP_DENSE2 = 4,
    OP_CONT = 5,
    OP_GIVENS = 6,
    OP_FACTOR = 7
};
// OP_DENSE2 (specialised kernels only): a 4x4 complex matrix on register
// slots lo = lbit & 0xff and hi = lbit >> 8 (block index = (bit hi) << 1 |
// (bit lo)); row 0 in m[], rows 1..3 in the m[] of the three OP_CONT records
// that follow; lctrl bit 4r + c is set where entry (r, c) is exactly zero.
// OP_GIVENS (specialised kernels only): the real matrix [[1, -t], [t, 1]]
// (form 0) or [[t, -1], [1, t]] (form 1) on register slot lbit & 0xff, form
// = lbit >> 8, t = m[0]; controls as for OP_DENSE.
// OP_FACTOR (specialised kernels only): one term of a phase run (a maximal
// sequence of OP_FACTOR ops).  Registers whose slots in the mask lbit & 0xf
// are all 1 are multiplied by m[0..1], or by m[2..3] where the selector is
// 1; selector lbit >> 8: 0 none, 1 + b thread-local bit b, 255 the global
// bit gtbit.  The term applies where the thread bits lctrl and the global
// bits gctrl are all 1.  Selector 254: a run of such ops holds one factor
// per register (m[0..7]: registers 4c .. 4c+3, c = lbit & 0xff).

struct FOp {
    int32_t kind;
    int32_t lbit;    // DENSE/PERM: register slot of the target; DIAG: local target bit, -1 if outside the tile
    uint32_t lctrl;  // controls inside the tile as local bits; REMAP: new register bits, 4 bits per slot
    int32_t slot;    // >= 0: the matrix is row `slot` of the per-trajectory table; -1: m[] below
    uint64_t gctrl;  // controls outside the tile, as global bits
    uint64_t gtbit;  // global target bit of a diagonal op outside the tile, else 0
    double m[8];
};
static_assert(sizeof(FOp) == 96, "FOp layout");

constexpr int kMaxTileBits = 16;
struct FPass {
    int32_t k;      // tile bits
    int32_t nlow;   // bits[0..nlow-1] == 0..nlow-1
    int32_t first;  // first op index
    int32_t nops;
    int8_t bits[kMaxTileBits];  // ascending global bit positions of the tile
};


// A gate list compiled into fused passes (host side).
struct FusedProgram {
    struct Item {
        bool swap;
        int q1, q2;  // swap qubits
        int pass;    // index into passes
    };
    std::vector<FPass> passes;
    std::vector<FOp> ops;
    int m = 4;  // register bits per thread (a pass of k < m tile bits uses k)
    // per pass: 1 = runs on the generic kernel although specialised kernels
    // are on (more ops than "fused_jit_max_ops": compile time grows faster
    // than the op count)
    std::vector<uint8_t> generic;
    std::vector<Item> items;
    std::vector<int64_t> order;    // execution order of the source gates
    std::vector<int32_t> pass_of;  // pass of each executed gate (-1: swap)
    bool batched = false;          // a trajectory batch's program (per-register matrix tables)
};
// Whether the specialised complex64 kernels of prog put dense ops on the
// matrix cores: fused_mfma for single registers, batch_mfma for batches.
inline bool svi_prog_mfma(const FusedProgram &prog) {
    return prog.batched ? svi_config().batch_mfma != 0 : svi_config().fused_mfma != 0;
}

// Waves per SIMD the specialised kernels of prog are compiled for (0: the
// compiler's choice); batches only.
inline int svi_prog_waves(const FusedProgram &prog) { return prog.batched ? svi_config().batch_waves : 0; }

// Plans and packs a validated gate list for an n-qubit register of dtype.
int svi_fused_compile(int n, int dtype, const PreparedGate *g, int64_t ng, FusedProgram &out);

// Launch of one compiled pass over nregs registers stored back to back at
// state; table (may be NULL) holds nslots matrices per register in the real
// type of dtype.
struct FusedLaunch {
    void *state;
    int n;
    int dtype;
    hipStream_t stream;
    const void *table;
    uint32_t nslots;
    uint64_t nregs;
};
hipError_t svi_fused_launch_pass(const FusedLaunch &L, int k, const FPass *dpass, const FOp *dops);

// Specialised pass kernels (jit.hip): one straight-line kernel per pass,
// compiled with hipRTC on first use and cached by source.  Launches take
// the same FusedLaunch as the generic kernel (batches of registers with
// per-register matrix tables included).
int svi_jit_prepare(int device, int dtype, const FusedProgram &prog, std::vector<hipFunction_t> &fns);
// Composes runs of ops on one or two register slots into one 2x2 or 4x4
// matrix (FP64) where that saves arithmetic; rewrites prog's ops and passes.
// one_slot: compose runs on a single slot only; only (if not NULL): the
// passes to rewrite (others are left as they are).
void svi_jit_fuse_pairs(FusedProgram &prog, bool one_slot = false, const std::vector<char> *only = nullptr);
// Splits unitary dense ops into phase, OP_GIVENS, phase and merges the
// phases of each pass into OP_FACTOR runs (rotations.cpp), in the passes
// marked in only (NULL: every pass).
void svi_jit_split_rotations(FusedProgram &prog, const std::vector<char> *only = nullptr);
// The rewrites above that the configuration turns on, in order.
void svi_jit_transform(FusedProgram &prog);
// Source text of the specialised kernel of one pass.
std::string svi_jit_pass_source(int dtype, const FusedProgram &prog, size_t pass);
hipError_t svi_jit_launch(hipFunction_t f, const FusedLaunch &L, int K, int M, const FPass *dpass, const FOp *dops);

// Mechanism-compiled source-term kernels: generation, compilation (hiprtc)
// and launch.  Host-side only.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ak_device.h"

namespace ak {

// Pressure dependence of one reaction (Sec. 2.4), host side.  A
// third-body reaction's RxnRec::log2A already counts the extra order; for
// a falloff reaction RxnRec holds the high-pressure limit.
struct PdepRec {
    int type = 0;             // AK_RXN_* of annkin.h
    int profile = -1;         // efficiency profile (third-body concentration)
    double log2A0 = 0.0;      // low-pressure limit: log2 A (SI, order + 1)
    double beta0 = 0.0;
    double negE0oR2 = 0.0;    // -(E0/R) log2(e), K
    double alpha = 0.0, T3 = 0.0, T1 = 0.0, T2 = 0.0;   // Troe
};

// What the generator needs of a prepared mechanism (host copies, sorted
// reaction order).
struct JitMech {
    int ns = 0, nr = 0;
    const SpeciesRec *sp = nullptr;   // [ns]
    const ThermoRec *th = nullptr;    // [ns] NASA-7 coefficients
    const RxnRec *rx = nullptr;       // [nr]
    const RxnAux *aux = nullptr;      // [nr]
    const PdepRec *pd = nullptr;      // [nr], or null when all are elementary
    // distinct efficiency vectors [ns] of the pressure-dependent reactions
    const std::vector<std::vector<double>> *profiles = nullptr;
};

// Generated kernels of one mechanism for one precision.
//   ak_src(T, P, Y, ldY, n, om, ldO, SP, RX, err): one lane per cell.
//   ak_src_batch(desc, nreq): the same for several requests of this
//     mechanism in one launch (workgroup -> request by binary search).
struct JitKernels {
    const double *sp = nullptr;   // device copies of JitProgram::sp and ::rx
    const double *rx = nullptr;
    double T_lo = 0.0, T_hi = 0.0;
    hipModule_t mod = nullptr;
    hipFunction_t src = nullptr;
    hipFunction_t batch = nullptr;
    int block = 64;          // cells per workgroup of both kernels
    int threads = 64;        // threads per workgroup
};

// One request of a fused launch of generated kernels (device table).
struct JitBatchDesc {
    const void *T, *P, *Y;
    void *om;
    int64_t ldY, ldO, n;
    int64_t block_begin;     // first workgroup of this request
};

// Waves per 64-cell tile of the tiled form, and the largest mechanism for
// which the whole per-cell state (a, v and the omega accumulators) is kept in
// the registers of one lane instead.
constexpr int kTileWaves = 4;
constexpr int kLaneFormMaxSpecies = 16;
// largest mechanisms with compiled kernels (two tiles per CU of 160 KB LDS)
constexpr int kJitMaxSpeciesFP32 = 102;
constexpr int kJitMaxSpeciesFP64 = 76;

// Whether a mechanism of this size gets compiled kernels: two tiles of the
// tiled form must fit a CU's LDS.
bool jit_suitable(int ns, bool f64);
size_t tile_lds_bytes(int ns, bool f64, int waves);

// Generated kernels of one mechanism and precision: the HIP source text of
// both kernels and the constant tables they read (per species the Gibbs
// layer, per reaction 3 doubles in the order of the mechanism's sorted
// reactions).  In the FP32
// path the kernels evaluate cells with T_lo <= T <= T_hi and report others
// as bad (T_lo = T_hi = 0: no restriction).
struct JitProgram {
    std::string src;
    int threads = 64;         // threads per workgroup (one workgroup: 64 cells)
    std::vector<double> sp;   // 16 doubles per species (SpeciesRec layout)
    std::vector<double> rx;
    double T_lo = 0.0, T_hi = 0.0;
};
JitProgram jit_program(const JitMech &m, bool f64);

// The same kernels for larger mechanisms, one 64-cell tile per workgroup of
// `waves` waves: the per-species factors of the tile in LDS, each wave
// sweeping a fixed subset of the reactions with its own rate accumulators,
// which the waves then add up in a fixed order.
JitProgram jit_program_tile(const JitMech &m, bool f64, int waves);

// The state Jacobian (rows omega_1..omega_NS, omega_T; columns Y_1..Y_NS,
// T) compiled for the mechanism: kernel ak_jac(T, P, Y, ldY, n, J, ldJ, SP,
// RX, err), one 64-cell tile per workgroup of JitProgram::threads threads.
// `f64out`: double states and J, else float (the arithmetic is double in
// both).  `interleaved`: J[(row (NS+1) + col) ldJ + cell], else
// J[cell ldJ + row (NS+1) + col].  Elementary reactions only.
JitProgram jit_program_jac(const JitMech &m, bool f64out, bool interleaved = false);
// The vector-jacobian product of omega compiled for the mechanism: kernel
// ak_vjp(T, P, Y, ldY, n, G, ldG, GY, ldGY, GT, SP, RX, err) (layouts of
// ak_eval_vjp), the same tiles, tables and limits as the Jacobian.
JitProgram jit_program_vjp(const JitMech &m, bool f64out);
hipError_t jit_vjp_launch(const JitKernels &k, const void *T, const void *P, const void *Y,
                          int64_t ldY, int64_t n, const void *G, int64_t ldG, void *GY,
                          int64_t ldGY, void *GT, unsigned long long *err, hipStream_t st);
// Compiler options of that kernel beyond the common ones (the machine
// scheduler that interleaves independent reactions: with two waves per SIMD
// the kernel needs the instruction-level parallelism).
std::vector<std::string> jac_compile_options();
// LDS of a tile of the compiled Jacobian; the kernel needs it below the
// device's 160 KB.
size_t jac_lds_bytes(int ns, int nr);
bool jac_suitable(const JitMech &m);

// The form that suits the mechanism (lane-per-cell for small ones, tiled
// otherwise).
JitProgram jit_generate(const JitMech &m, bool f64);

// Compile the text for gfx950 with hiprtc; returns 0 or an AK_E* code (the
// compiler log goes to `log`).  Results are cached in the process by text.
int jit_compile(const std::string &src, std::vector<char> &code, std::string &log,
                const std::vector<std::string> &extra = {});

// Load a code object on the current device; `fn` and `batch` (may be null)
// are the kernels' names.
int jit_load(const std::vector<char> &code, JitKernels &out, const char *fn = "ak_src",
             const char *batch = "ak_src_batch");
void jit_unload(JitKernels &k);

hipError_t jit_launch(const JitKernels &k, const void *T, const void *P, const void *Y,
                      int64_t ldY, int64_t n, void *om, int64_t ldO, unsigned long long *err,
                      hipStream_t st);
hipError_t jit_batch_launch(const JitKernels &k, const JitBatchDesc *d_desc, int nreq,
                            int64_t blocks, unsigned long long *err, hipStream_t st);

}  // namespace ak

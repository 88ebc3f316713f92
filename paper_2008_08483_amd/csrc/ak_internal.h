// Host-side internals shared by the annkin translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "ak_device.h"
#include "ak_jit.h"

struct ak_mechanism {
    int device = 0;
    int ns = 0, nr = 0;
    ak::MechView view{};
    unsigned char *dev = nullptr;        // single device allocation for all tables
    int lds_max = 0;                     // LDS bytes per workgroup on the device
    int vjp_tile = 0;                    // cells per VJP workgroup tile
    std::vector<ak::SpeciesRec> host_species;
    std::vector<ak::RxnRec> host_rxn;   // shape-sorted order
    std::vector<int> rxn_order;         // file index of each sorted reaction
    ak::JitKernels jit[2];              // mechanism-compiled kernels per precision (FP64, FP32)
    bool pdep = false;                  // third-body or falloff reactions (compiled kernels only)
    // what the compiled Jacobian is generated from (host copies, sorted order)
    std::vector<ak::RxnAux> host_aux;
    std::vector<ak::ThermoRec> host_th;
    // the compiled Jacobian per precision and layout (cell-major,
    // interleaved), built at the first call that uses it: state 0 not
    // tried, 1 loaded
    mutable std::mutex jac_mu;
    mutable ak::JitKernels jac[2][2];
    mutable int jac_state[2][2] = {{0, 0}, {0, 0}};
    // the compiled vector-Jacobian product per precision (same tables)
    mutable ak::JitKernels vjp[2];
    mutable int vjp_state[2] = {0, 0};
    mutable unsigned char *jac_dev = nullptr;   // their constant tables
    // the ln K_c tables (descriptor-order reactions, sorted-to-descriptor
    // index), uploaded at the first call that needs them
    mutable unsigned char *kc_dev = nullptr;
    mutable bool kc_wide = false;   // a reaction has more than 4 distinct species
    mutable int kc_pieces = 0;      // intervals of the composed ln K_c layers (0: not built)
    mutable size_t kc_fold_off = 0; // their records' offset in kc_dev
    // nu in the matrix-core operand order of the split-bfloat16
    // contraction, uploaded at its first call
    mutable unsigned char *prod_dev = nullptr;
};

namespace ak {

int set_error(int code, const char *fmt, ...);
// Let a kernel use the device's whole LDS as dynamic shared memory (set once
// per kernel and device, on the current device).
hipError_t allow_dynamic_lds(const void *fn);
int hip_error(hipError_t e, const char *what);

// Makes `dev` current for the lifetime of the guard, restoring the caller's
// device afterwards.
struct DeviceGuard {
    int prev;
    bool ok;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

size_t source_lds_bytes(int ns, int tile);
hipError_t source_launch(const MechView &m, bool f64, const void *T, const void *P,
                         const void *Y, int64_t ldY, int64_t n, void *om, int64_t ldO,
                         hipStream_t st);

// max_ns: the largest species count among the batch's mechanisms
hipError_t source_batch_launch(bool f64, const BatchDesc *d_desc, int nreq, int64_t blocks,
                               size_t lds, int max_ns, hipStream_t st);
hipError_t euler_update_launch(const MechView &m, bool f64, void *T, const void *P, void *Y,
                               int64_t ldY, int64_t n, const void *om, int64_t ldO, double dt,
                               hipStream_t st);
size_t implicit_lds_bytes(int ns);
hipError_t implicit_update_launch(const MechView &m, bool f64, void *T, const void *P, void *Y,
                                  int64_t ldY, int64_t n, const void *om, int64_t ldO,
                                  const void *J, int64_t ldJ, double dt, hipStream_t st);
// Argument checks of the integrators (fn names the entry point in messages)
// and their body: n_steps of (source term into `omega` [NS][n], update).
int integrate_check(const char *fn, const ak_mechanism *m, int prec, const void *T,
                    const void *P, const void *Y, int64_t ldY, int64_t n, double dt,
                    int n_steps);
int integrate_run(const ak_mechanism *m, int prec, void *T, const void *P, void *Y,
                  int64_t ldY, int64_t n, double dt, int n_steps, void *omega, void *stream);
size_t jacobian_lds_bytes(int ns);
hipError_t jacobian_launch(const MechView &m, int lds_max, bool f64, const void *T, const void *P,
                           const void *Y, int64_t ldY, int64_t n, void *J, int64_t ldJ,
                           hipStream_t st);
int vjp_tile(int ns, int lds_max);
hipError_t vjp_launch(const MechView &m, int tile, bool f64, const void *T, const void *P,
                      const void *Y, int64_t ldY, int64_t n, const void *G, int64_t ldG,
                      void *GY, int64_t ldGY, void *GT, hipStream_t st);

}  // namespace ak

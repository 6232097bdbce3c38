// Context object behind the opaque swe_ctx of include/swe.h (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "swe_internal.h"
#include "swe_kernels.h"

struct swe_ctx {
    swe_config cfg{};
    int dev = 0;
    hipStream_t stream = nullptr;
    bool own_stream = true;  // false: borrowed from the caller (swe_config.stream)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::string err;
    bool has_mesh = false, has_state = false, ran = false;
    int n_owned = 0, n_total = 0, n_scen = 1, n_send = 0, n_ghost = 0;
    int send_prefix = 0;  // the send cells are local cells [0, send_prefix)
    size_t tsize = 4;
    // device buffers
    void *nbr = nullptr, *cell = nullptr, *man2 = nullptr, *he_geo = nullptr, *he_dist = nullptr;
    void *he_co = nullptr, *he_lam = nullptr, *he_gam = nullptr;  // tiled kernel's half-edge set
    void *he_dfw = nullptr;     // tiled WAF kernel: centroid distance per half-edge (WAF contexts)
    void *he_nrm = nullptr;     // tiled WAF kernel: unit normal per half-edge (WAF contexts)
    void *U[2] = {nullptr, nullptr}, *U1 = nullptr, *tmp3 = nullptr, *bed = nullptr;
    float *phi = nullptr;       // learned-limiter output, one per half-edge
    void *mlp = nullptr;        // learned-limiter weights (MlpDev, BF16)
    bool has_mlp = false;
    bool phi_stale = false;  // learned limiter: the next step evaluates phi whatever its index
    unsigned long long *clock = nullptr;  // 3 slots x (1 + ncopy) lines per scenario
    int ncopy = 64;
    swe::ScenParams *scen = nullptr;
    double *ser_t = nullptr, *ser_q = nullptr, *t0 = nullptr;
    int *health = nullptr, *flag = nullptr, *send_idx = nullptr;
    int *pk_off = nullptr, *pk_ent = nullptr;  // send entries per send cell (CSR)
    // host mirrors
    std::vector<swe::ScenParams> h_scen;
    std::vector<std::pair<std::vector<double>, std::vector<double>>> series;  // per scenario
    std::vector<double> h_ser_t, h_ser_q, h_t0;
    std::vector<int> scen_off;  // first cell of each scenario, n_scen + 1 entries
    // launch shape: threads per block and blocks of a persistent launch (0:
    // one tile per block); picked by swe_autotune when tuned
    int grid_persist = 0;
    int waves = 0;  // tiled FP32 kernel, 256-cell tiles: 0 automatic, 6 or 7
    int ncu = 0;    // compute units of the device
    bool tuned = false;
    double computed_inflow_len = 0.0, given_inflow_len = 0.0;
    long long step_count = 0;  // steps since set_state (selects clock slots and buffers)
    int block = 256;
    // graphs: chunk of kGraphSteps steps starting at a step index multiple of it
    hipGraphExec_t graph = nullptr;
    double graph_dt = -1.0;
    bool use_graphs = true;
};


namespace swe {
// Learned limiter (swe_mlp.hip): phi of every half-edge of state U into
// out[3 * n_total], on the context stream.
int launch_limiter_phi(swe_ctx *c, const void *U, float *out);
// Clock slots of a freshly set state U[0] (time t, CFL minima); syncs.
int init_clock(swe_ctx *c, double t);
}  // namespace swe

// Device memory of a context: the configured allocator, else hipMalloc.
// Freed only once the context's stream has finished with it.
inline hipError_t dalloc(swe_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    if (!c->cfg.alloc) return hipMalloc(p, bytes);
    *p = c->cfg.alloc(bytes, c->cfg.alloc_user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline void dfree(swe_ctx *c, void *&p)
{
    if (p) {
        if (c->cfg.free) c->cfg.free(p, c->cfg.alloc_user);
        else (void)hipFree(p);
    }
    p = nullptr;
}

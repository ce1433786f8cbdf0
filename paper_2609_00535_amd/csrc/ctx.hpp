// Host-side context of one solve (the opaque slbm_ctx of the C ABI).
#pragma once

#include <string>
#include <vector>

#include "../../include/semlbm.h"
#include "internal.hpp"

#include <new>

namespace slbm {
// Every slbm_status entry point runs its body through this: no exception leaves the C ABI
// (host allocation failures come back as SLBM_ENOMEM, anything else as SLBM_EINVAL).
template <class F>
inline slbm_status slbm_guard(F &&f) noexcept {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return SLBM_ENOMEM;
    } catch (...) {
        return SLBM_EINVAL;
    }
}
// enqueue n full time steps for one (lattice key, N) group of solves: element plan ep, and
// sp for the node kernels of the unfused step (nodes past each member's interior range)
int enqueue_steps(int d, int N, const LaunchPlan &ep, const LaunchPlan &sp, int64_t n, void *stream,
                  bool fused);
// capture 'steps' calls of fn(stream) into an instantiated graph (hipGraphExec_t)
int capture_graph(void *stream, void **exec, int (*fn)(void *, void *), void *arg);
int launch_graph(void *exec, void *stream);
void destroy_graph(void *exec);
}  // namespace slbm

// meshes (and batch groups) over this many local nodes step with the unfused kernels, which
// gather each shared node once and finish element-interior nodes in the element kernels;
// below it the fused kernels' fewer launches win.  Measured crossovers: between 0.53 M and
// 1.05 M local nodes in 2-D (N = 4, 6, 8), between 0.12 M and 0.24 M in 3-D (N = 3-6,
// both lattices), where the fused kernels gather up to eight copies per copy
constexpr int64_t kUnfusedAboveLocalNodes2D = (int64_t)1 << 20;
constexpr int64_t kUnfusedAboveLocalNodes3D = (int64_t)1 << 17;
inline int64_t unfused_above(int dim) { return dim == 3 ? kUnfusedAboveLocalNodes3D : kUnfusedAboveLocalNodes2D; }

struct slbm_ctx {
    slbm_params prm{};
    double tau = 0.0;  // relaxation time in use (prm.tau, or from prm.nu at set_mesh)
    int dim = 0, Q = 0, N = 0, Np = 0, nloc = 0;
    int dq = 0;  // lattice key of the kernel launchers: 2 (D2Q9), 3 (D3Q19), 13 (D3Q13)
    double beta = 0, kappa = 0, omega = 0, dt = 0, hmin = 0;
    double ev[slbm::kMaxQ][3] = {};
    double tw[slbm::kMaxQ] = {}, tc[slbm::kMaxQ] = {};
    int opp[slbm::kMaxQ] = {};
    std::vector<double> xi, wq, Dm, wn;
    // mesh (host copies)
    bool has_mesh = false;
    int64_t E = 0, Nl = 0, Ng = 0, nw = 0;
    std::vector<double> xyz;
    std::vector<int32_t> lgid, ig2ug, csr_ptr, csr_idx, gcopy, lwall, lcp;
    int vmax = 0;
    bool fused = true;  // fused element-kernel path (needs vmax <= the fused copy slots)
    int64_t Nint = 0;   // element-interior nodes numbered first (unfused path; see SolveDesc)
    int64_t lstride = 0, Nld = 0;  // device element stride and size of the per-local-node arrays
    std::vector<double> Ja, Gm, MA, Minv, w_dat;
    // device
    struct Offsets {
        size_t desc, eplan, nplan, lgid, gcopy, csr_idx, lcp, lwall, w_dat, Ja, G, Minv, Dm, wn, f, g0, g1,
            g2, rho, mu, rl, gl, rs, aux, diag, red;
    } off{};
    size_t ws_bytes = 0;
    int n_eblocks = 0, n_nblocks = 0, n_sblocks = 0, epb = 1;
    bool bound = false, has_state = false;
    // the Laplacian partials no longer belong to the state: a fused-path context stepped by
    // the unfused kernels in a batch (their last stage leaves the partials of its input)
    bool rl_stale = false;
    void *dev = nullptr;
    void *stream = nullptr;
    slbm::SolveDesc desc{};
    // element blocks, node blocks over every node, node blocks over nodes Nint .. Ng-1
    slbm::LaunchPlan eplan{}, nplan{}, splan{};
    int64_t step = 0;
    std::string err;
    // HIP graphs of 1 and kGraphSteps time steps (captured lazily on a non-null stream)
    static constexpr int kGraphSteps = 10;
    void *graph[2] = {nullptr, nullptr};  // hipGraphExec_t
    bool use_graph = true;

    ~slbm_ctx();
    slbm_status enqueue(int64_t n);

    slbm_status fail(slbm_status s, const char *fmt, ...);
    slbm_status hip_check(int e, const char *what);
    int stride(int a) const;
    int along(int n, int a) const;
    double dline(const double *h, int n, int a) const;
    void layout();
    slbm_status require_bound(bool need_state);
    slbm_status upload_f_and_density(const std::vector<double> &f_int);
    // recompute the Laplacian partials of the state if they are stale (fused path only)
    int refresh_lap();
    slbm_status read_diag(double *ke, double *mass);
    slbm_status put(double *dst, const double *src_user, int fields);
    slbm_status get(const double *src, double *dst_user, int fields);
    slbm_status restore_density();
};

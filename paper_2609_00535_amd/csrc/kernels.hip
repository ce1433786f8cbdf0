// Dispatch of the kernel launchers (internal.hpp) to the per-order translation units, and
// the batch-wide reduction kernel.
#include "kernels.hpp"

namespace slbm {

#define SLBM_DECLARE_SET(SFX)                                                                \
    int launch_lap_##SFX(int, int, const LaunchPlan &, void *);                              \
    int launch_mu_##SFX(int, int, const LaunchPlan &, void *);                               \
    int launch_grad_##SFX(int, int, const LaunchPlan &, int, void *);                        \
    int launch_gavg_##SFX(int, int, const LaunchPlan &, void *);                             \
    int launch_collide_##SFX(int, int, const LaunchPlan &, int, void *);                     \
    int launch_stream_##SFX(int, int, const LaunchPlan &, int, void *);                      \
    int launch_rk_##SFX(int, int, const LaunchPlan &, int, void *);                          \
    int launch_density_##SFX(int, int, const LaunchPlan &, int, void *);                     \
    int launch_diag_##SFX(int, int, const LaunchPlan &, void *);                             \
    int launch_fA_##SFX(int, int, const LaunchPlan &, void *);                               \
    int launch_fB_##SFX(int, int, const LaunchPlan &, void *);                               \
    int launch_fC_##SFX(int, int, const LaunchPlan &, int, void *);                          \
    int launch_fD_##SFX(int, int, const LaunchPlan &, int, void *);
SLBM_DECLARE_SET(2a)
SLBM_DECLARE_SET(2b)
SLBM_DECLARE_SET(3d)
SLBM_DECLARE_SET(3q)

bool supported_order(int d, int N) {
#define X(DD, NN) if (d == DD && N == NN) return true;
    SLBM_ORDERS_2A(X)
    SLBM_ORDERS_2B(X)
    SLBM_ORDERS_3D(X)
    SLBM_ORDERS_3Q(X)
#undef X
    return false;
}

// (lattice key, N) -> instance set
#define SLBM_PICK(NAME, ...)                                                                 \
    (d == 13 ? launch_##NAME##_3q(d, N, __VA_ARGS__) :                                       \
     d == 3 ? launch_##NAME##_3d(d, N, __VA_ARGS__)                                          \
            : (N <= 7 ? launch_##NAME##_2a(d, N, __VA_ARGS__) : launch_##NAME##_2b(d, N, __VA_ARGS__)))

int launch_lap(int d, int N, const LaunchPlan &p, void *stream) { return SLBM_PICK(lap, p, stream); }
int launch_mu(int d, int N, const LaunchPlan &p, void *stream) { return SLBM_PICK(mu, p, stream); }
int launch_grad(int d, int N, const LaunchPlan &p, int collide, void *stream) {
    return SLBM_PICK(grad, p, collide, stream);
}
int launch_gavg(int d, int N, const LaunchPlan &p, void *stream) { return SLBM_PICK(gavg, p, stream); }
int launch_collide(int d, int N, const LaunchPlan &p, int use_aux, void *stream) {
    return SLBM_PICK(collide, p, use_aux, stream);
}
int launch_stream(int d, int N, const LaunchPlan &p, int stage, void *stream) {
    return SLBM_PICK(stream, p, stage, stream);
}
int launch_rk(int d, int N, const LaunchPlan &p, int stage, void *stream) { return SLBM_PICK(rk, p, stage, stream); }
int launch_density(int d, int N, const LaunchPlan &p, int which, void *stream) {
    return SLBM_PICK(density, p, which, stream);
}
int launch_diag(int d, int N, const LaunchPlan &p, void *stream) { return SLBM_PICK(diag, p, stream); }
int launch_fA(int d, int N, const LaunchPlan &p, void *stream) { return SLBM_PICK(fA, p, stream); }
int launch_fB(int d, int N, const LaunchPlan &p, void *stream) { return SLBM_PICK(fB, p, stream); }
int launch_fC(int d, int N, const LaunchPlan &p, int stage, void *stream) { return SLBM_PICK(fC, p, stage, stream); }
int launch_fD(int d, int N, const LaunchPlan &p, int stage, void *stream) { return SLBM_PICK(fD, p, stage, stream); }

// second pass of the KE / mass reduction: one block per member; also into out[2 * member]
// when out is given (a batch reads all members with one copy)
__global__ __launch_bounds__(kNodeThreads) void k_diag_final(const SolveDesc *desc, double *out) {
    __shared__ double smax[kNodeThreads], ssum[kNodeThreads];
    const SolveDesc &sd = desc[blockIdx.x];
    const int nb = (sd.Ng + kNodeThreads - 1) / kNodeThreads;
    const int tid = threadIdx.x;
    double km = 0.0, ms = 0.0;
    for (int b = tid; b < nb; b += kNodeThreads) {
        const double a = sd.red[2 * b];
        km = (km >= a || km != km) ? km : a;
        ms += sd.red[2 * b + 1];
    }
    smax[tid] = km;
    ssum[tid] = ms;
    __syncthreads();
    for (int s = kNodeThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double a = smax[tid], b = smax[tid + s];
            smax[tid] = (a >= b || a != a) ? a : b;
            ssum[tid] += ssum[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        sd.diag[0] = smax[0];
        sd.diag[1] = ssum[0];
        if (out) {
            out[2 * blockIdx.x] = smax[0];
            out[2 * blockIdx.x + 1] = ssum[0];
        }
    }
}

int launch_diag_final(const SolveDesc *desc, int nsolves, void *stream, double *out) {
    if (nsolves <= 0) return 0;
    k_diag_final<<<nsolves, kNodeThreads, 0, (hipStream_t)stream>>>(desc, out);
    return (int)hipGetLastError();
}

}  // namespace slbm

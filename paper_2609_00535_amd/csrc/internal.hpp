// Internal interface between the host runtime (semlbm.cpp, serve.cpp) and the HIP
// kernels (kernels.hpp and the kernels*.hip units).  Not part of the public C ABI.
#pragma once

#include <cstddef>
#include <cstdint>

// Pointers into device memory are qualified as global-address-space when compiled for the
// GPU (the host sees plain pointers; both are 64-bit, so the layouts agree).  Pointers read
// from a descriptor would otherwise be generic and compile to FLAT instructions, which share
// the LDS wait counter and serialise memory with LDS traffic.
#if defined(__HIP_DEVICE_COMPILE__)
#define SLBM_GLOBAL __attribute__((address_space(1)))
#else
#define SLBM_GLOBAL
#endif
// helpers shared by host and device code (plain inline functions in host-only builds)
#if defined(__HIPCC__)
#define SLBM_HD __host__ __device__
#else
#define SLBM_HD
#endif

namespace slbm {

constexpr int kMaxQ = 19;

// First DSS copies of a global node: csr position k0 of its local copies, their count nc
// and the first two local indices (i1 repeats i0 for a single copy), read with one 16-byte
// load; copies beyond the second are read through csr_idx.
struct alignas(16) NodeCopies {
    int k0, nc, i0, i1;
};

// Everything one solve's kernels need, resident in device memory (one entry per batch
// member).  Index arrays are int32: a solve holds < 2^31 local nodes.
struct SolveDesc {
    int E, Nl, Ng, vmax;
    // element-interior split (unfused path): global nodes 0 .. Nint-1 are the nodes strictly
    // inside an element, numbered first (element by element).  The element kernels finish
    // them (mu in k_lap, the collision in k_grad, the Runge-Kutta stage in k_stream) and the
    // node kernels mu, collide and rk run over nodes Nint .. Ng-1 only.  0: no split.
    int Nint;
    // element stride of the per-local-node arrays (lgid, lwall, Ja, G and the per-copy
    // partials): (N+1)^d, or on the 3-D split path that count rounded up to 16 doubles, so
    // every element's block of each array starts on a 128-byte line (at N = 5 the runs of
    // each face's 16 nodes then fill whole lines); Nl is E times this stride
    int lstride;
    // mesh tables (device)
    const int SLBM_GLOBAL *lgid;      // [Nl] local node -> internal global node
    const double SLBM_GLOBAL *Ja;     // [d*d][Nl] J * d xi_a / d x_c, index (a*d + c)
    const double SLBM_GLOBAL *G;      // [d(d+1)/2][Nl] w (Ja_a . Ja_b) / J, upper triangle row-major
    const double SLBM_GLOBAL *Minv;   // [Ng] inverse assembled lumped mass
    const NodeCopies SLBM_GLOBAL *gcopy;  // [Ng] first copies of each global node
    const int SLBM_GLOBAL *csr_idx;   // [Nl]   local copies of the global nodes, ascending per node
    const int SLBM_GLOBAL *lcp;       // [vmax][Nl] local copies of the global node of each local node,
                                      // ascending, -1 padded (fused path)
    const int SLBM_GLOBAL *lwall;     // [Nl] (first wall entry << 2) | number of entries of the node
    const double SLBM_GLOBAL *w_dat;  // [nw][2d+1] per wall entry: s n (d), u_b (d),
                                      // s cos(theta) sqrt(2 beta / kappa); a node's entries adjacent
    const double SLBM_GLOBAL *Dm;     // [(N+1)^2] GLL differentiation matrix, Dm[i*(N+1)+m]
    const double SLBM_GLOBAL *wn;     // [(N+1)^d] tensor GLL weights
    // state and work buffers (device)
    double SLBM_GLOBAL *f;    // [Q][Ng] f-bar (state)
    double SLBM_GLOBAL *g0;   // [Q][Ng] post-collision f*
    double SLBM_GLOBAL *g1;   // [Q][Ng] Runge-Kutta stage 1 (the unfused path keeps every stage here)
    double SLBM_GLOBAL *g2;   // [Q][Ng] Runge-Kutta stage 2 (fused path)
    double SLBM_GLOBAL *rho;  // [Ng]
    double SLBM_GLOBAL *mu;   // [Ng]
    double SLBM_GLOBAL *rl;   // [Nl] Laplacian residual of each local copy
    double SLBM_GLOBAL *gl;   // [2d][Nl] lumped-mass weighted element gradients of rho and mu
    double SLBM_GLOBAL *rs;   // [Q-1][Nl] streaming residual of each local copy
    double SLBM_GLOBAL *aux;  // [2d][Ng] averaged gradients (operator entry points)
    double SLBM_GLOBAL *diag; // [4] KE_max, mass, -, -
    double SLBM_GLOBAL *red;  // [2 * max blocks] reduction partials
    // physics
    double rho_l, rho_v, beta, kappa, omega, dt;
    // lattice weights t and t / cs^2 by class: |e|^2 = 0 (rest), 1 (axis), 2 (diagonal) for
    // D2Q9 and D3Q19; 0 (rest), 1 (moving) for D3Q13
    double tw[3], twc[3];
    // D3Q13 component magnitudes a = sqrt((5 - sqrt 5)/6), b = sqrt((5 + sqrt 5)/6) (else 0)
    double lat_a, lat_b;
};

// Launch-shape bookkeeping shared by host and device.
struct LaunchPlan {
    const SolveDesc SLBM_GLOBAL *desc;   // device array of descriptors
    const int SLBM_GLOBAL *blk_solve;    // device: block -> batch member index
    const int SLBM_GLOBAL *blk_local;    // device: block -> block index within its member
    int nblocks;             // logical blocks (single member) or table length
    int single;              // one member: no table lookup, XCD-aware block mapping
    int epb;                 // elements per block of element kernels (wide or 1)
    int grid;                // launched blocks (nblocks for a single member, else a multiple of kXcds)
    // single member: its descriptor by value in the kernel arguments, so a block reads it
    // with one scalar load from the argument segment instead of two dependent ones
    SolveDesc one;
};

// MI355X dispatches consecutive workgroups round-robin over its 8 accelerator dies (XCDs),
// each with its own L2.  Block tables (batches): logical block j is run by hardware block b
// with j = (b % 8) * ceil(n / 8) + b / 8 over a grid padded to a multiple of 8 (padding
// entries are -1), so each die works on one contiguous range of elements or nodes and
// neighbours share that die's L2.  A single solve launches exactly n blocks and uses the
// bijection xcd_single below (no padding block, so no block exits before its loads).
constexpr int kXcds = 8;
inline int xcd_grid(int n) { return ((n + kXcds - 1) / kXcds) * kXcds; }
inline int xcd_logical(int b, int n) { const int per = (n + kXcds - 1) / kXcds; return (b % kXcds) * per + b / kXcds; }
// hardware block b -> logical block for a grid of exactly n blocks: the first 8*(n/8)
// blocks as above with n/8 per die, the remaining n % 8 blocks keep their index
SLBM_HD inline int xcd_single(int b, int n) {
    const int per = n / kXcds;
    return b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
}

// Element-kernel shape for order N in d dimensions (must match Shape in kernels.hpp): "wide" blocks
// hold as many elements as fit in 256 threads; small meshes use one element per block so
// that every compute unit gets work.
inline int nloc_of(int d, int N) { int p = N + 1; return d == 2 ? p * p : p * p * p; }  // d: 2, 3 or 13
inline int epb_wide(int d, int N) { int n = nloc_of(d, N); return n <= 256 ? 256 / n : 1; }
inline int epb_for(int d, int N, int64_t E) {
    const int w = epb_wide(d, N);
    return (E + w - 1) / w < 256 ? 1 : w;
}
constexpr int kNodeThreads = 256;

// Kernel launchers (kernels.hip dispatches them to the per-order units).  'd' is the lattice
// key: 2 (D2Q9), 3 (D3Q19) or 13 (D3Q13).  'stage' is 1..3
// for the RK stages.  All launch on 'stream' and return the hipError_t of the launch as int.
int launch_lap(int d, int N, const LaunchPlan &p, void *stream);
int launch_mu(int d, int N, const LaunchPlan &p, void *stream);
// collide != 0 (in-step): element-interior nodes are collided here (see SolveDesc::Nint)
int launch_grad(int d, int N, const LaunchPlan &p, int collide, void *stream);
int launch_gavg(int d, int N, const LaunchPlan &p, void *stream);
// use_aux: operator entry point (averaged gradients from aux, every node); else in-step
int launch_collide(int d, int N, const LaunchPlan &p, int use_aux, void *stream);

// stage 1..3: streams g0 (1) or g1 (2, 3) and finishes element-interior nodes with that
// Runge-Kutta stage; stage 0 (operator entry point): streams g1, interior nodes get L
int launch_stream(int d, int N, const LaunchPlan &p, int stage, void *stream);
int launch_rk(int d, int N, const LaunchPlan &p, int stage, void *stream);
int launch_density(int d, int N, const LaunchPlan &p, int which, void *stream);
int launch_diag(int d, int N, const LaunchPlan &p, void *stream);
int launch_diag_final(const SolveDesc *desc, int nsolves, void *stream, double *out = nullptr);
// fused path: four element kernels per stage sequence (A: mu + gradients, B: collision +
// stage-1 residual, C: DSS + Runge-Kutta combine + Laplacian residual, D: mu + residual)
constexpr int kCopySlots[2] = {4, 8};  // register copy slots of the fused kernels (2-D, 3-D)
int launch_fA(int d, int N, const LaunchPlan &p, void *stream);
int launch_fB(int d, int N, const LaunchPlan &p, void *stream);
int launch_fC(int d, int N, const LaunchPlan &p, int stage, void *stream);
int launch_fD(int d, int N, const LaunchPlan &p, int stage, void *stream);
bool supported_order(int d, int N);

// Allocation-free batched stepping: the launch tables live in a file-scope device array of
// this many bytes per GPU (static_scratch.hip); static_scratch returns its device address on
// the current device (looked up once per device), or a hipError_t.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
int static_scratch(void **ptr);

}  // namespace slbm

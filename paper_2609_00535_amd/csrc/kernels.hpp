// HIP kernels (gfx950) of the two-phase spectral-element LBM time step: device code and
// kernel templates.  Each kernels_*.hip translation unit instantiates them for a set of
// (dimension, order) pairs (compiled in parallel); kernels.hip dispatches (d, N) to them.
//
// Two kernel families alternate inside a step:
//   * element kernels: one thread per element node, several elements per 256-thread block,
//     element fields staged in LDS; tensor-product GLL derivatives are contractions of an
//     LDS line with a row (or column) of the differentiation matrix;
//   * node kernels: one thread per global node; they finish the direct stiffness summation
//     (DSS) by gathering the node's local copies in ascending order (deterministic, no
//     atomics) and apply the pointwise physics.
// Every kernel serves a whole batch: block b works on member blk_solve[b], block
// blk_local[b] of it, with the member's tables and state in its SolveDesc.  A single solve
// is a batch of one.
//
// Memory-level parallelism: each kernel issues all of its global loads (index tables
// first, then the data they address) before its first global store, and reads the
// descriptor into registers at entry.  A store through a state pointer may alias any
// later load as far as the compiler knows, so loads placed after a store are issued only
// after it and their latencies add up; this ordering keeps every wave to two dependent
// memory round trips (index, data) plus its barriers.
//
// Floating point: the build disables contraction; the GLL contractions use fma explicitly
// and every other expression is written with the operand order of the CPU oracle, so the
// two implementations round identically.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

#ifndef SLBM_WPE_STREAM_3D
#define SLBM_WPE_STREAM_3D 2
#endif

namespace slbm {

// ------------------------------------------------------------------------------------------
// lattice tables
// ------------------------------------------------------------------------------------------
template <int Q> struct Lat;
template <> struct Lat<9> {
    static constexpr int D = 2;
    static constexpr int e[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};
template <> struct Lat<19> {
    static constexpr int D = 3;
    static constexpr int e[19][3] = {
        {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
        {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};
// D3Q13: the rest velocity and the twelve vertices of an icosahedron with |e|^2 = 5/3.  The
// table holds the pattern of each velocity: 0, +-1 for a component of magnitude a and +-2
// for magnitude b (a = sqrt((5 - sqrt 5)/6), b = sqrt((5 + sqrt 5)/6), in the descriptor).
template <> struct Lat<13> {
    static constexpr int D = 3;
    static constexpr int e[13][3] = {{0, 0, 0},  {0, 1, 2},   {0, -1, -2}, {0, 1, -2}, {0, -1, 2},
                                     {1, 2, 0},  {-1, -2, 0}, {1, -2, 0},  {-1, 2, 0}, {2, 0, 1},
                                     {-2, 0, -1}, {2, 0, -1}, {-2, 0, 1}};
    static constexpr int opp[13] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11};
};
template <int D> struct QOf;
template <> struct QOf<2> { static constexpr int Q = 9; };
template <> struct QOf<3> { static constexpr int Q = 19; };
// Kernel templates take a lattice key DQ: 2 (D2Q9), 3 (D3Q19) or 13 (D3Q13).
template <int DQ> struct DimOf { static constexpr int v = DQ == 2 ? 2 : 3; };
template <int DQ> struct QOfDQ { static constexpr int v = DQ == 2 ? 9 : (DQ == 3 ? 19 : 13); };

// weight class of population q: t_q = tw[class], t_q / cs^2 = twc[class]; |e_q|^2 (0 rest,
// 1 axis, 2 diagonal) for D2Q9 and D3Q19, rest (0) or moving (1) for D3Q13
template <int Q>
__device__ __forceinline__ constexpr int wcls(int q) {
    if constexpr (Q == 13) return q == 0 ? 0 : 1;
    else return Lat<Q>::e[q][0] * Lat<Q>::e[q][0] + Lat<Q>::e[q][1] * Lat<Q>::e[q][1] +
                Lat<Q>::e[q][2] * Lat<Q>::e[q][2];
}

// s + x (e_q)_c with the rounding of the plain product-and-sum: components 1 and -1 add or
// subtract x exactly, zero components add nothing (s + (+-0) == s for the sums here, which
// start from +0.0), and the D3Q13 magnitudes multiply
template <int Q>
__device__ __forceinline__ double acc_e(double s, double x, int q, int c, const SolveDesc &sd) {
    const int ec = Lat<Q>::e[q][c];
    if constexpr (Q == 13) {
        if (ec == 0) return s;
        const double m = (ec == 1 || ec == -1) ? sd.lat_a : sd.lat_b;
        return s + x * (ec > 0 ? m : -m);
    } else {
        if (ec == 1) return s + x;
        if (ec == -1) return s - x;
        return s;
    }
}

// v . e_q summed in ascending component order from 0 (equals the plain dot product bit for bit)
template <int Q, int D>
__device__ __forceinline__ double dot_e(const double *v, int q, const SolveDesc &sd) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) s = acc_e<Q>(s, v[c], q, c, sd);
    return s;
}

// Streaming accesses (NT): the unfused streaming kernel runs on meshes far beyond the caches
// and reads its metric terms and writes its residual partials and finished populations
// once per launch; those accesses carry the non-temporal hint so that they do not displace
// lines that neighbouring blocks still reuse (the populations, densities and chemical
// potentials of shared nodes): c4 3.18 -> 3.15 ms per step.  The same hint on the other
// unfused kernels' accesses measured slower (on the node kernels' partial gathers, whose
// lines neighbouring lanes reuse, much slower), and the fused kernels, which run on
// cache-resident meshes, use plain accesses.
template <bool NT>
__device__ __forceinline__ double ld_s(const double SLBM_GLOBAL *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st_s(double SLBM_GLOBAL *p, double v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// ------------------------------------------------------------------------------------------
// element shapes
// ------------------------------------------------------------------------------------------
template <int D, int N, bool WIDE = true> struct Shape {
    static constexpr int NP = N + 1;
    static constexpr int NLOC = D == 2 ? NP * NP : NP * NP * NP;
    static constexpr int EPB = WIDE && NLOC <= 256 ? 256 / NLOC : 1;
    static constexpr int NB = EPB * NLOC;  // nodes of one block
    static constexpr int NT = ((NB + 63) / 64) * 64;
    static constexpr int NG = D * (D + 1) / 2;
    static constexpr int NINT = D == 2 ? (NP - 2) * (NP - 2) : (NP - 2) * (NP - 2) * (NP - 2);  // interior nodes
    // minimum waves per SIMD asked of the 3-D streaming kernels (a register cap; at 2 the
    // kernels need no spill slots, at 3 they spill and run slower on c4)
    static constexpr int WPE_STREAM = D == 3 ? SLBM_WPE_STREAM_3D : 1;
    static_assert(NT >= NP * NP, "one differentiation-matrix entry per thread");
};

template <int NP, int A> struct Stride { static constexpr int v = A == 0 ? 1 : (A == 1 ? NP : NP * NP); };

// d/dxi_A at element node n of an LDS field s (element base): sum_m D[i][m] s[.. m ..]
template <int NP, int A>
__device__ __forceinline__ double dref(const double *__restrict__ sD, const double *__restrict__ s, int n) {
    constexpr int st = Stride<NP, A>::v;
    const int i = (n / st) % NP;
    const double *row = sD + i * NP;
    const double *line = s + (n - i * st);
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) acc = fma(row[m], line[m * st], acc);
    return acc;
}

// transpose: sum_m D[m][i] v[.. m ..]
template <int NP, int A>
__device__ __forceinline__ double drefT(const double *__restrict__ sD, const double *__restrict__ v, int n) {
    constexpr int st = Stride<NP, A>::v;
    const int i = (n / st) % NP;
    const double *line = v + (n - i * st);
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) acc = fma(sD[m * NP + i], line[m * st], acc);
    return acc;
}

template <int D, int NP>
__device__ __forceinline__ void grad_ref(const double *sD, const double *s, int n, double *out) {
    out[0] = dref<NP, 0>(sD, s, n);
    out[1] = dref<NP, 1>(sD, s, n);
    if constexpr (D == 3) out[2] = dref<NP, 2>(sD, s, n);
}

template <int D, int NP>
__device__ __forceinline__ double div_refT(const double *sD, const double *v, int stride_field, int n) {
    double s = 0.0;
    s += drefT<NP, 0>(sD, v, n);
    s += drefT<NP, 1>(sD, v + stride_field, n);
    if constexpr (D == 3) s += drefT<NP, 2>(sD, v + 2 * stride_field, n);
    return s;
}

// The differentiation matrix is fetched into a register with the block's first loads and
// written to LDS just before the first barrier, so its latency overlaps theirs.
template <int NP>
__device__ __forceinline__ double dm_fetch(const SolveDesc &sd, int tid) {
    return sd.Dm[tid < NP * NP ? tid : 0];
}
template <int NP>
__device__ __forceinline__ void dm_store(double *sD, int tid, double v) {
    if (tid < NP * NP) sD[tid] = v;
}

// block -> (member descriptor, first element of the block)
struct BlockSlot {
    const SolveDesc SLBM_GLOBAL *sd;
    int local;
    bool valid;  // padding blocks of the XCD-aware grid do nothing
};
// SINGLE (a compile-time copy of p.single): a single solve's blocks find everything in
// the kernel arguments, so its kernels start with one scalar round trip
template <bool SINGLE>
__device__ __forceinline__ BlockSlot block_slot(const LaunchPlan &p) {
    BlockSlot b;
    if (SINGLE) {
        b.sd = p.desc;
        b.local = xcd_single((int)blockIdx.x, p.nblocks);
        b.valid = true;  // the grid is exactly nblocks
    } else {
        const int j = blockIdx.x < (unsigned)p.nblocks ? (int)blockIdx.x : 0;
        b.local = p.blk_local[j];
        b.valid = blockIdx.x < (unsigned)p.nblocks && b.local >= 0;
        b.sd = p.desc + (b.valid ? p.blk_solve[j] : 0);
    }
    return b;
}

// The member's descriptor in registers, read before the kernel's first global store (a
// store through a state pointer could otherwise alias the descriptor in memory and force
// reloads).  A single solve passes it in the kernel arguments.
template <bool SINGLE>
__device__ __forceinline__ SolveDesc desc_of(const LaunchPlan &p, const BlockSlot &b) {
    if (SINGLE) return p.one;
    return *b.sd;
}

// ------------------------------------------------------------------------------------------
// wall entries of a local node (at most d faces of its element): the first entry and the
// count come from lwall; entries beyond the count repeat the last one so every slot can be
// loaded without a branch (only nodes with walls load anything)
// ------------------------------------------------------------------------------------------
template <int D> struct WallLap {
    int cnt;
    double lap[D];  // s cos(theta) sqrt(2 beta / kappa) of each face through the node
};
template <int D>
__device__ __forceinline__ void load_wall_lap(const SolveDesc &sd, int l, WallLap<D> &w) {
    const int v = sd.lwall[l];
    const int k0 = v >> 2;
    w.cnt = v & 3;
#pragma unroll
    for (int j = 0; j < D; ++j) w.lap[j] = 0.0;
    if (w.cnt > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int k = k0 + (j < w.cnt ? j : w.cnt - 1);
            w.lap[j] = sd.w_dat[(size_t)k * (2 * D + 1) + 2 * D];
        }
    }
}
template <int D> struct WallFlux {
    int cnt;
    double sn[D][D];  // s n of each face through the node
    double ub[D][D];  // wall velocity of that face
};
template <int D>
__device__ __forceinline__ void load_wall_flux(const SolveDesc &sd, int l, WallFlux<D> &w) {
    const int v = sd.lwall[l];
    const int k0 = v >> 2;
    w.cnt = v & 3;
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
        for (int c = 0; c < D; ++c) w.sn[j][c] = w.ub[j][c] = 0.0;
    if (w.cnt > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int k = k0 + (j < w.cnt ? j : w.cnt - 1);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                w.sn[j][c] = sd.w_dat[(size_t)k * (2 * D + 1) + c];
                w.ub[j][c] = sd.w_dat[(size_t)k * (2 * D + 1) + D + c];
            }
        }
    }
}

// wetting term of Eq. (8) at a wall node: s n.grad(rho) = s cos(theta) sqrt(2 beta/kappa)
// |(rho-rl)(rho-rv)| for every face through the node, in the caller's face order
template <int D>
__device__ __forceinline__ double wall_lap_term(const SolveDesc &sd, const WallLap<D> &w, double rh, double r) {
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (j < w.cnt) r += w.lap[j] * fabs((rh - sd.rho_l) * (rh - sd.rho_v));
    return r;
}

// ------------------------------------------------------------------------------------------
// DSS through the CSR copy lists: the first two copies come from the node's NodeCopies
// entry (one load); further copies, on nodes shared by more than two elements, through
// csr_idx.  Ascending local order, from +0.0, as the oracle sums.
// ------------------------------------------------------------------------------------------
// Copies beyond the second are fetched kCsrAhead at a time: all their indices, then all
// their values, then the sums in order (one dependent round trip per group of copies, not
// two per copy).
constexpr int kCsrAhead = 6;

template <class P>
__device__ __forceinline__ double dss_sum(P v, const NodeCopies &c, const int SLBM_GLOBAL *csr_idx) {
    const double x0 = v[c.i0], x1 = v[c.i1];
    double s = 0.0;
    s += x0;
    s += c.nc > 1 ? x1 : 0.0;
    for (int k = 2; k < c.nc; k += kCsrAhead) {
        int li[kCsrAhead];
        double x[kCsrAhead];
#pragma unroll
        for (int j = 0; j < kCsrAhead; ++j) li[j] = k + j < c.nc ? csr_idx[c.k0 + k + j] : -1;
#pragma unroll
        for (int j = 0; j < kCsrAhead; ++j) x[j] = li[j] >= 0 ? v[li[j]] : 0.0;
#pragma unroll
        for (int j = 0; j < kCsrAhead; ++j)
            if (k + j < c.nc) s += x[j];
    }
    return s;
}

// ------------------------------------------------------------------------------------------
// Eq. (8): element part of the weak Laplacian, r = -sum_a D_a^T (G^{ab} D_b rho), plus the
// wetting boundary integral s n.grad(rho) = s cos(theta) sqrt(2 beta/kappa) |(rho-rl)(rho-rv)|
// ------------------------------------------------------------------------------------------
// Eq. (2): mu = mu0(rho) - kappa lap, lap = DSS(r) / M (reading: mu0 = 2 beta (rho-rl)(rho-rv)(2rho-rl-rv))
__device__ __forceinline__ double mu_of(const SolveDesc &sd, double pr, double lap) {
    const double rl = sd.rho_l, rv = sd.rho_v;
    const double mu0 = 2.0 * sd.beta * (pr - rl) * (pr - rv) * (2.0 * pr - rl - rv);
    return mu0 - sd.kappa * lap;
}

// element node n (i fastest) on the element's boundary?  Nodes inside an element belong to
// it alone (the fused path is selected only for meshes where that holds).
// (bitwise, not short-circuit: a chain of || becomes a chain of divergent branches, and
// hipcc has been seen to reuse a live register inside such a chain at N = 3 in 2-D)
template <int D, int NP>
__device__ __forceinline__ bool on_elem_boundary(int n) {
    const int i = n % NP, j = (n / NP) % NP;
    int b = (int)(i == 0) | (int)(i == NP - 1) | (int)(j == 0) | (int)(j == NP - 1);
    if constexpr (D == 3) {
        const int k = n / (NP * NP);
        b |= (int)(k == 0) | (int)(k == NP - 1);
    }
    return b != 0;
}

// Element-interior split: the local nodes of an element are stored interior-first: the
// (N-1)^d interior nodes in natural order, then the boundary nodes grouped by class (the
// nodes inside face 0, 1, .., 2d-1 (xi-, xi+, eta-, ...) face by face, then the nodes
// inside edges, then the corners; natural order within each group).  Lanes of an element
// thus take interior and boundary nodes in separate runs (3-D N = 5: the first wave is
// exactly the 64 interior nodes), and the copies of a shared face sit in one run of slots in
// each of its two elements, which the shared-node numbering follows.  split_node maps the
// storage position m within the element to the element node n = i + (N+1) j (+ (N+1)^2 k).
template <int D, int NP>
struct BoundaryOrder {
    static constexpr int NLOC = D == 2 ? NP * NP : NP * NP * NP;
    static constexpr int NINT = D == 2 ? (NP - 2) * (NP - 2) : (NP - 2) * (NP - 2) * (NP - 2);
    static constexpr int NBD = NLOC - NINT;
    int node[NBD];
    // number of coordinates on the element boundary, and the face (2a + side) when it is one
    static constexpr int cls(int n, int *face) {
        int b = 0;
        for (int a = 0, st = 1; a < D; ++a, st *= NP) {
            const int i = (n / st) % NP;
            if (i == 0 || i == NP - 1) {
                ++b;
                *face = 2 * a + (i == NP - 1 ? 1 : 0);
            }
        }
        return b;
    }
    constexpr BoundaryOrder() : node{} {
        int k = 0;
        for (int f = 0; f < 2 * D; ++f)
            for (int n = 0; n < NLOC; ++n) {
                int fc = -1;
                if (cls(n, &fc) == 1 && fc == f) node[k++] = n;
            }
        for (int c = 2; c <= D; ++c)
            for (int n = 0; n < NLOC; ++n) {
                int fc = -1;
                if (cls(n, &fc) == c) node[k++] = n;
            }
    }
};
template <int D, int NP>
__device__ __forceinline__ int split_node(int m) {
    constexpr int NI = NP - 2;
    constexpr int NINT = D == 2 ? NI * NI : NI * NI * NI;
    if (m < NINT) {
        const int i = 1 + m % NI, j = 1 + (m / NI) % NI;
        return D == 2 ? i + NP * j : i + NP * j + NP * NP * (1 + m / (NI * NI));
    }
    static constexpr BoundaryOrder<D, NP> order{};
    return order.node[m - NINT];
}

// Lane of an unfused element kernel -> (element slot es within the block, storage position
// m within that element).  Split mesh: the interior nodes of all the block's elements take
// the first lanes and the boundary nodes the rest, so at most one wave of a block holds
// both kinds; otherwise lanes follow the natural node order element by element.
template <int D, int N, bool WIDE>
__device__ __forceinline__ void lane_slot(int tid, bool split, int &es, int &m) {
    using S = Shape<D, N, WIDE>;
    constexpr int NI = S::NINT, NBD = S::NLOC - S::NINT;
    if (!split) {
        es = tid / S::NLOC;
        m = tid - es * S::NLOC;
    } else if (tid < S::EPB * NI) {
        es = tid / NI;
        m = tid - es * NI;
    } else {
        const int t = tid - S::EPB * NI;
        es = t / NBD;
        m = NI + (t - es * NBD);
    }
}

template <int D, int NB, int NG>
__device__ __forceinline__ void metric_times_grad(const double *g, const double *d, double *sv, int tid) {
    // v_a = sum_b G_ab d_b (ascending b from 0)
    if constexpr (D == 2) {
        double v0 = 0.0, v1 = 0.0;
        v0 += g[0] * d[0]; v0 += g[1] * d[1];
        v1 += g[1] * d[0]; v1 += g[2] * d[1];
        sv[tid] = v0; sv[NB + tid] = v1;
    } else {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        v0 += g[0] * d[0]; v0 += g[1] * d[1]; v0 += g[2] * d[2];
        v1 += g[1] * d[0]; v1 += g[3] * d[1]; v1 += g[4] * d[2];
        v2 += g[2] * d[0]; v2 += g[4] * d[1]; v2 += g[5] * d[2];
        sv[tid] = v0; sv[NB + tid] = v1; sv[2 * NB + tid] = v2;
    }
}

template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT)) void k_lap(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    __shared__ double sD[NP * NP];
    __shared__ double srho[NB];
    __shared__ double sv[D * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    double dmv = 0.0;
    // element slot es and storage position m of the lane's node, its element node n, and
    // its LDS slot ln (natural order within the element)
    int es, m;
    lane_slot<D, N, WIDE>(tid, sd.Nint > 0, es, m);
    const int n = sd.Nint > 0 ? split_node<D, NP>(m) : m;
    const int ln = es * NLOC + n;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * sd.lstride + m;
    // element-interior node of a split mesh: its Laplacian has this copy alone, so mu is
    // finished here (as k_mu would: the sum of one copy, times 1/M)
    const bool own = sd.Nint > 0 && m < S::NINT;
    double rh = 0.0, mi = 0.0;
    int G = 0;
    double g[S::NG];
    WallLap<D> wl;
    // every lane below (N+1)^2 fetches its entry of D (with the split lane map such a lane
    // can belong to an element slot past the end of the mesh)
    dmv = dm_fetch<NP>(sd, tid);
    if (act) {
        G = sd.lgid[l];
#pragma unroll
        for (int k = 0; k < S::NG; ++k) g[k] = sd.G[(size_t)k * sd.Nl + l];
        load_wall_lap<D>(sd, l, wl);
        rh = sd.rho[G];
        if (own) mi = sd.Minv[G];
        srho[ln] = rh;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (act) {
        double d[D];
        grad_ref<D, NP>(sD, srho + es * NLOC, n, d);
        metric_times_grad<D, NB, S::NG>(g, d, sv, ln);
    }
    __syncthreads();
    if (!act) return;
    const double r = -div_refT<D, NP>(sD, sv + es * NLOC, NB, n);
    if (own) {
        sd.mu[G] = mu_of(sd, rh, (0.0 + r) * mi);  // no wall faces pass through an interior node
        return;
    }
    sd.rl[l] = wall_lap_term<D>(sd, wl, rh, r);
}

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kNodeThreads) void k_mu(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int G = sd.Nint + bs.local * kNodeThreads + threadIdx.x;  // interior nodes: k_lap
    if (G >= sd.Ng) return;
    const NodeCopies c = sd.gcopy[G];
    const double mi = sd.Minv[G], pr = sd.rho[G];
    const double lap = dss_sum(sd.rl, c, sd.csr_idx) * mi;
    sd.mu[G] = mu_of(sd, pr, lap);
}

// Eq. (4) with (A.2), (A.6)-(A.7) and F** of Sec. 2.1 at one node:
// f* = f - omega (f - (feq - dt/2 F**)) + dt F**, F = cs^2 grad(rho) - rho grad(mu)
// moments and force shared by the populations of a node: u = sum f e / rho, F, u.F, u.u
template <int Q, int D> struct CollidePrep {
    double u[D], F[D], uF, uu;
};
template <int Q, int D>
__device__ __forceinline__ void collide_prep(const SolveDesc &sd, const double *f, double pr, const double *gr,
                                             const double *gm, CollidePrep<Q, D> &c) {
    const double cs2 = 1.0 / 3.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double m = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) m = acc_e<Q>(m, f[q], q, k, sd);
        c.u[k] = m / pr;
        c.F[k] = cs2 * gr[k] - pr * gm[k];
    }
    c.uF = 0.0;
    c.uu = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        c.uF += c.u[k] * c.F[k];
        c.uu += c.u[k] * c.u[k];
    }
}
// f*_q of one population
template <int Q, int D>
__device__ __forceinline__ double collide_q(const SolveDesc &sd, int q, double fq, double pr,
                                            const CollidePrep<Q, D> &c) {
    const double dt = sd.dt, om = sd.omega;
    const double eu = dot_e<Q, D>(c.u, q, sd), eF = dot_e<Q, D>(c.F, q, sd);
    const double tq = sd.tw[wcls<Q>(q)], tc = sd.twc[wcls<Q>(q)];
    const double Fss = tc * (eu * eF * 3.0 - c.uF);
    const double feq = pr * tq * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * c.uu);
    const double fbeq = feq - 0.5 * dt * Fss;
    return fq - om * (fq - fbeq) + dt * Fss;
}
template <int Q, int D>
__device__ __forceinline__ void collide_node(const SolveDesc &sd, const double *f, double pr,
                                             const double *gr, const double *gm, double *fs) {
    CollidePrep<Q, D> c;
    collide_prep<Q, D>(sd, f, pr, gr, gm, c);
#pragma unroll
    for (int q = 0; q < Q; ++q) fs[q] = collide_q<Q, D>(sd, q, f[q], pr, c);
}

// lumped-mass weighted element gradients w Ja^T grad_ref of rho and mu (for the collision);
// with collide != 0 the element-interior nodes of a split mesh (one copy each, so their
// averaged gradient is this copy's times 1/M) are collided here as k_collide would
template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT)) void k_grad(LaunchPlan p, int collide) {
    constexpr int D = DimOf<DQ>::v;
    constexpr int Q = QOfDQ<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    __shared__ double sD[NP * NP];
    __shared__ double sf[2 * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    double dmv = 0.0;
    // element slot es and storage position m of the lane's node, its element node n, and
    // its LDS slot ln (natural order within the element)
    int es, m;
    lane_slot<D, N, WIDE>(tid, sd.Nint > 0, es, m);
    const int n = sd.Nint > 0 ? split_node<D, NP>(m) : m;
    const int ln = es * NLOC + n;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * sd.lstride + m;
    const bool own = collide && sd.Nint > 0 && m < S::NINT;
    const size_t Ng = sd.Ng;
    double J[D][D];
    double w = 0.0, pr = 0.0, mi = 0.0;
    double f[Q];
    int G = 0;
    // every lane below (N+1)^2 fetches its entry of D (with the split lane map such a lane
    // can belong to an element slot past the end of the mesh)
    dmv = dm_fetch<NP>(sd, tid);
    if (act) {
        G = sd.lgid[l];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int c = 0; c < D; ++c) J[a][c] = sd.Ja[(size_t)(a * D + c) * sd.Nl + l];
        w = sd.wn[n];
        pr = sd.rho[G];
        sf[ln] = pr;
        sf[NB + ln] = sd.mu[G];
        if (own) {
            mi = sd.Minv[G];
#pragma unroll
            for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
        }
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
    double gs[2][D];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double d[D];
        grad_ref<D, NP>(sD, sf + k * NB + es * NLOC, n, d);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) s += J[a][c] * d[a];
            gs[k][c] = w * s;
            if (!own) sd.gl[(size_t)(k * D + c) * sd.Nl + l] = gs[k][c];
        }
    }
    if (!own) return;
    double gr[D], gm[D], fs[Q];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        gr[c] = (0.0 + gs[0][c]) * mi;
        gm[c] = (0.0 + gs[1][c]) * mi;
    }
    collide_node<Q, D>(sd, f, pr, gr, gm, fs);
#pragma unroll
    for (int q = 0; q < Q; ++q) sd.g0[q * Ng + G] = fs[q];
}

// averaged gradients DSS(gl) / M into aux [2d][Ng] (operator entry point)
template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kNodeThreads) void k_gavg(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int G = bs.local * kNodeThreads + threadIdx.x;
    if (G >= sd.Ng) return;
    const NodeCopies cp = sd.gcopy[G];
    const double mi = sd.Minv[G];
    double s[2 * D];
#pragma unroll
    for (int c = 0; c < 2 * D; ++c) s[c] = dss_sum(sd.gl + (size_t)c * sd.Nl, cp, sd.csr_idx);
#pragma unroll
    for (int c = 0; c < 2 * D; ++c) sd.aux[(size_t)c * sd.Ng + G] = s[c] * mi;
}

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kNodeThreads) void k_collide(LaunchPlan p, int use_aux) {
    constexpr int D = DimOf<DQ>::v;
    constexpr int Q = QOfDQ<DQ>::v;
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    // in-step: element-interior nodes were collided by k_grad; the operator covers every node
    const int G = (use_aux ? 0 : sd.Nint) + bs.local * kNodeThreads + threadIdx.x;
    if (G >= sd.Ng) return;
    const size_t Ng = sd.Ng;
    double gr[D], gm[D];
    double f[Q];
    if (use_aux) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = sd.aux[c * Ng + G];
            gm[c] = sd.aux[(D + c) * Ng + G];
        }
    } else {
        const NodeCopies cp = sd.gcopy[G];
        const double mi = sd.Minv[G];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = dss_sum(sd.gl + (size_t)c * sd.Nl, cp, sd.csr_idx) * mi;
            gm[c] = dss_sum(sd.gl + (size_t)(D + c) * sd.Nl, cp, sd.csr_idx) * mi;
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
    const double pr = sd.rho[G];
    double fs[Q];
    collide_node<Q, D>(sd, f, pr, gr, gm, fs);
#pragma unroll
    for (int q = 0; q < Q; ++q) sd.g0[q * Ng + G] = fs[q];
}

// ------------------------------------------------------------------------------------------
// Eqs. (5)-(6), (12), (9): element residual of the force-split weak streaming,
//   r_a = -w [ (Ja e_a) . D(g_a - t_a rho) + (t_a/cs^2) rho (Ja e_a) . D mu ]
// plus, on wall faces with (s n).e_a < 0, (s n . e_a) [g_a - g_opp - 2 (t_a/cs^2) rho e_a.u_b]
// ------------------------------------------------------------------------------------------
// per-node metric and wall data of the streaming, loaded with the block's first loads
template <int D> struct NodeGeo {
    double J[D][D];
    double w;
    WallFlux<D> wf;
};
template <int D, bool NT = false>
__device__ __forceinline__ void load_metric(const SolveDesc &sd, int n, int l, NodeGeo<D> &g) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) g.J[a][c] = ld_s<NT>(sd.Ja + (size_t)(a * D + c) * sd.Nl + l);
    g.w = sd.wn[n];
}
template <int D>
__device__ __forceinline__ void load_geo(const SolveDesc &sd, int n, int l, NodeGeo<D> &g) {
    load_metric<D>(sd, n, l, g);
    load_wall_flux<D>(sd, l, g.wf);
}

// residual at node n from LDS h_q = g_q - t_q rho (fields of stride NB, element base es),
// LDS mu, register g (for the flux); the loop reads only LDS and registers, so its stores
// delay no load
// residual of population q at node n (h_q of the element in LDS at sh_q, stride 1 within
// the element; dmu = reference gradient of mu; gq, gopp: g_q and g_opp(q) for the flux)
template <int Q, int D, int NP>
__device__ __forceinline__ double residual_q(const SolveDesc &sd, int q, const double *sD, const double *sh_q,
                                             int n, const double *dmu, double pr, double gq, double gopp,
                                             const NodeGeo<D> &geo) {
    double dh[D];
    grad_ref<D, NP>(sD, sh_q, n, dh);
    double adv = 0.0, frc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double ca = dot_e<Q, D>(geo.J[a], q, sd);
        adv += ca * dh[a];
        frc += ca * dmu[a];
    }
    const double tc = sd.twc[wcls<Q>(q)];
    double r = -(geo.w * (adv + tc * pr * frc));
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j < geo.wf.cnt) {
            const double cn = dot_e<Q, D>(geo.wf.sn[j], q, sd);
            if (cn < 0.0) {
                const double eub = dot_e<Q, D>(geo.wf.ub[j], q, sd);
                const double bc = gq - gopp - 2.0 * tc * pr * eub;
                r += cn * bc;
            }
        }
    }
    return r;
}

template <int Q, int D, int N, bool WIDE, bool NT = false>
__device__ __forceinline__ void stream_residual(const SolveDesc &sd, const double *sD, const double *sh,
                                                const double *smu_e, int es, int n, int l,
                                                double pr, const double *gq, const NodeGeo<D> &geo) {
    using S = Shape<D, N, WIDE>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    double dmu[D];
    grad_ref<D, NP>(sD, smu_e, n, dmu);
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const double r = residual_q<Q, D, NP>(sd, q, sD, sh + (q - 1) * NB + es * NLOC, n, dmu, pr, gq[q],
                                              gq[Lat<Q>::opp[q]], geo);
        st_s<NT>(sd.rs + (size_t)(q - 1) * sd.Nl + l, r);
    }
}

// SSP-RK3 stage combination after DSS(r)/M, and the new stage's density (Eq. (10))
//   stage 0 (operator entry point only): g1 = L(g1)
//   stage 1: g1 = g0 + dt L(g0); stage 2: g1 = 3/4 g0 + 1/4 (g1 + dt L(g1));
//   stage 3: f = (g0 + 2 (g1 + dt L(g1))) / 3
template <int Q>
__device__ __forceinline__ double rk_combine(int stage, double L, double gin, double g0, double dt) {
    const double x = gin + dt * L;
    if (stage == 0) return L;  // operator entry point: the assembled right-hand side
    if (stage == 1) return x;
    if (stage == 2) return 0.75 * g0 + 0.25 * x;
    return (g0 + 2.0 * x) / 3.0;
}

// Element-interior node of a split mesh (one copy, no wall face): its residual needs no
// summation, so the stage is finished here as k_rk would (L = (0 + r) / M, the stage
// combination and the new density in ascending q); stage 0 stores L (operator entry point)
template <int Q, int D, int N, bool WIDE>
__device__ __forceinline__ void stream_finish(const SolveDesc &sd, const double *sD, const double *sh,
                                              const double *smu_e, int es, int n, int G, double pr,
                                              const NodeGeo<D> &geo, int stage) {
    using S = Shape<D, N, WIDE>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    const size_t Ng = sd.Ng;
    const double SLBM_GLOBAL *gin = stage == 1 ? sd.g0 : sd.g1;
    double SLBM_GLOBAL *gout = stage == 3 ? sd.f : sd.g1;
    // the loads go out before the first store; the stage input is read again here (the
    // block read it before the barrier, so these are cache hits) rather than kept in
    // registers across the barrier
    const double mi = sd.Minv[G], dt = sd.dt;
    double gq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) gq[q] = gin[q * Ng + G];
    double g0v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g0v[q] = 0.0;
    if (stage >= 2) {
#pragma unroll
        for (int q = 0; q < Q; ++q) g0v[q] = sd.g0[q * Ng + G];
    }
    double dmu[D];
    grad_ref<D, NP>(sD, smu_e, n, dmu);
    double rho = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double L = 0.0;
        if (q > 0) {
            const double r = residual_q<Q, D, NP>(sd, q, sD, sh + (q - 1) * NB + es * NLOC, n, dmu, pr, gq[q],
                                                  gq[Lat<Q>::opp[q]], geo);
            L = (0.0 + r) * mi;
        }
        const double out = rk_combine<Q>(stage, L, gq[q], g0v[q], dt);
        st_s<true>(gout + q * Ng + G, out);
        rho += out;
    }
    st_s<true>(sd.rho + G, rho);
}

// After the barrier of the streaming kernel, one pass for both kinds of lanes: the
// residual of every population, then either the interior node's Runge-Kutta stage (as
// stream_finish, with the stage input the lane already holds) or the shared copy's partial
// (as stream_residual).  A wave that holds both kinds runs the residual work once instead
// of once per kind.  Used in 3-D where a block's interior nodes do not fill whole waves
// (N = 4: 54 interior lanes, 5% faster steps on a 3 M-node mesh); where they do (N = 5: 64)
// the two separate paths are faster (the joint pass holds 224 VGPRs against 187, 6% slower
// steps on c4).
template <int Q, int D, int N, bool WIDE>
__device__ __forceinline__ void stream_own_or_partial(const SolveDesc &sd, const double *sD, const double *sh,
                                                      const double *smu_e, int es, int n, int l, int G,
                                                      double pr, double *gq, NodeGeo<D> &geo, bool own,
                                                      int stage) {
    using S = Shape<D, N, WIDE>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    const size_t Ng = sd.Ng;
    const double SLBM_GLOBAL *gin = stage == 1 ? sd.g0 : sd.g1;
    double SLBM_GLOBAL *gout = stage == 3 ? sd.f : sd.g1;
    double g0v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g0v[q] = 0.0;
    double mi = 0.0;
    if (own) {
        mi = sd.Minv[G];
        gq[0] = gin[G];
        if (stage >= 2) {
#pragma unroll
            for (int q = 0; q < Q; ++q) g0v[q] = sd.g0[q * Ng + G];
        }
    } else {
        load_wall_flux<D>(sd, l, geo.wf);
    }
    double dmu[D];
    grad_ref<D, NP>(sD, smu_e, n, dmu);
    double rho = 0.0;
    if (own) {
        const double out = rk_combine<Q>(stage, 0.0, gq[0], g0v[0], sd.dt);
        st_s<true>(gout + G, out);
        rho += out;
    }
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const double r = residual_q<Q, D, NP>(sd, q, sD, sh + (q - 1) * NB + es * NLOC, n, dmu, pr, gq[q],
                                              gq[Lat<Q>::opp[q]], geo);
        if (own) {
            const double out = rk_combine<Q>(stage, (0.0 + r) * mi, gq[q], g0v[q], sd.dt);
            st_s<true>(gout + q * Ng + G, out);
            rho += out;
        } else {
            st_s<true>(sd.rs + (size_t)(q - 1) * sd.Nl + l, r);
        }
    }
    if (own) st_s<true>(sd.rho + G, rho);
}

// stage 1 streams g0, stages 2-3 stream g1 (stage 0, the operator entry point, streams g1)
template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT), (Shape<DimOf<DQ>::v, N, WIDE>::WPE_STREAM)) void k_stream(LaunchPlan p, int stage) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    __shared__ double sD[NP * NP];
    __shared__ double smu[NB];
    __shared__ double sh[(Q - 1) * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const double SLBM_GLOBAL *g = stage == 1 ? sd.g0 : sd.g1;
    const int tid = threadIdx.x;
    double dmv = 0.0;
    // element slot es and storage position m of the lane's node, its element node n, and
    // its LDS slot ln (natural order within the element)
    int es, m;
    lane_slot<D, N, WIDE>(tid, sd.Nint > 0, es, m);
    const int n = sd.Nint > 0 ? split_node<D, NP>(m) : m;
    const int ln = es * NLOC + n;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * sd.lstride + m;
    const size_t Ng = sd.Ng;
    const bool own = sd.Nint > 0 && m < S::NINT;
    double pr = 0.0;
    NodeGeo<D> geo;
    int G = 0;
    // the wall data of boundary nodes are loaded after the barrier (an interior node has
    // none): they are not live across it, and not at all on the interior path
    geo.wf.cnt = 0;
    // every lane below (N+1)^2 fetches its entry of D (with the split lane map such a lane
    // can belong to an element slot past the end of the mesh)
    dmv = dm_fetch<NP>(sd, tid);
    double gq[Q];  // kept across the barrier for the flux bounce-back of wall nodes
    if (act) {
        G = sd.lgid[l];
        load_metric<D, true>(sd, n, l, geo);
        pr = sd.rho[G];
        smu[ln] = sd.mu[G];
#pragma unroll
        for (int q = 1; q < Q; ++q) gq[q] = g[q * Ng + G];
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + ln] = gq[q] - sd.tw[wcls<Q>(q)] * pr;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
    // 3-D blocks whose interior nodes leave a wave holding both kinds of node take the joint
    // pass (in 2-D it measured slower: the 256-solve batch, whose members have no interior
    // split, 3.19 -> 3.27 ms per step)
    constexpr bool kMixedWave = D == 3 && (S::EPB * S::NINT) % 64 != 0;
    if constexpr (kMixedWave) {
        stream_own_or_partial<Q, D, N, WIDE>(sd, sD, sh, smu + es * NLOC, es, n, l, G, pr, gq, geo, own, stage);
    } else {
        if (own) {
            stream_finish<Q, D, N, WIDE>(sd, sD, sh, smu + es * NLOC, es, n, G, pr, geo, stage);
            return;
        }
        load_wall_flux<D>(sd, l, geo.wf);
        stream_residual<Q, D, N, WIDE, true>(sd, sD, sh, smu + es * NLOC, es, n, l, pr, gq, geo);
    }
}

// Elements of more than 256 nodes in blocks of four waves (256 lanes), with two nodes on
// some lanes, on meshes of at least kTailMinBlocks blocks (below that, with few blocks per
// compute unit, one lane per node is the shorter path).
constexpr int kTailThreads = 256;
constexpr int kTailMinBlocks = 512;

// k_stream for 3-D elements of more than 256 nodes (N = 6: 343) in blocks of four waves.
// One lane per node would need six waves, and such blocks keep far fewer waves resident
// per compute unit than blocks of four.  Lane t handles storage position t of its element
// (one element per block, so that is the lane map of k_stream), and lanes 128 + j, j <
// NLOC - 256, also position 256 + j, a shared node (the interior ones come first), whose
// loads go out before the lane's own and whose g and rho cross the barrier in LDS.  The
// second nodes sit on the lanes of shared first nodes, so the lanes that finish interior
// nodes take no second one.  Per node the arithmetic is that of k_stream: same bits.
template <int DD, int NN> constexpr bool kTail3 =
    DimOf<DD>::v == 3 && Shape<3, NN, true>::NLOC > kTailThreads && Shape<3, NN, true>::NLOC <= 2 * kTailThreads;
constexpr int kTailSecondLane = 128;

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kTailThreads, SLBM_WPE_STREAM_3D) void k_streamt(LaunchPlan p, int stage) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, true>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    constexpr int NX = NLOC - kTailThreads;  // second nodes, on lanes kTailSecondLane + j
    static_assert(S::EPB == 1 && NX > 0 && kTailSecondLane + NX <= kTailThreads && NP * NP <= kTailThreads &&
                  S::NINT <= kTailSecondLane,
                  "one element per block; second nodes on lanes whose first node is shared");
    __shared__ double sD[NP * NP];
    __shared__ double smu[NB];
    __shared__ double sh[(Q - 1) * NB];
    __shared__ double sx[Q * NX];  // second nodes: rho, then g_q for q >= 1
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const double SLBM_GLOBAL *g = stage == 1 ? sd.g0 : sd.g1;
    const int tid = threadIdx.x;
    const bool split = sd.Nint > 0;
    const int e = bs.local;
    const bool act = e < sd.E;
    const int m = tid;
    const int n = split ? split_node<D, NP>(m) : m;
    const int l = e * sd.lstride + m;
    const size_t Ng = sd.Ng;
    const bool own = split && m < S::NINT;
    const int j = tid - kTailSecondLane;
    const bool two = act && j >= 0 && j < NX;
    const int m2 = kTailThreads + (two ? j : 0);
    const int n2 = split ? split_node<D, NP>(m2) : m2;
    const int l2 = e * sd.lstride + m2;
    double pr = 0.0;
    NodeGeo<D> geo;
    int G = 0;
    geo.wf.cnt = 0;
    const double dmv = dm_fetch<NP>(sd, tid);
    if (two) {
        const int G2 = sd.lgid[l2];
        const double p2 = sd.rho[G2];
        smu[n2] = sd.mu[G2];
        sx[j] = p2;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const double x = g[q * Ng + G2];
            sx[q * NX + j] = x;
            sh[(q - 1) * NB + n2] = x - sd.tw[wcls<Q>(q)] * p2;
        }
    }
    double gq[Q];
    if (act) {
        G = sd.lgid[l];
        load_metric<D, true>(sd, n, l, geo);
        pr = sd.rho[G];
        smu[n] = sd.mu[G];
#pragma unroll
        for (int q = 1; q < Q; ++q) gq[q] = g[q * Ng + G];
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + n] = gq[q] - sd.tw[wcls<Q>(q)] * pr;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
    if (own) {
        stream_finish<Q, D, N, true>(sd, sD, sh, smu, 0, n, G, pr, geo, stage);
        return;  // interior lanes carry no second node
    }
    load_wall_flux<D>(sd, l, geo.wf);
    stream_residual<Q, D, N, true, true>(sd, sD, sh, smu, 0, n, l, pr, gq, geo);
    if (two) {
        NodeGeo<D> g2;
        load_metric<D, true>(sd, n2, l2, g2);
        load_wall_flux<D>(sd, l2, g2.wf);
        double x[Q];
        x[0] = 0.0;
#pragma unroll
        for (int q = 1; q < Q; ++q) x[q] = sx[q * NX + j];
        stream_residual<Q, D, N, true, true>(sd, sD, sh, smu, 0, n2, l2, sx[j], x, g2);
    }
}

// k_lap and k_grad for 3-D elements of more than 256 nodes in blocks of four waves, with the
// lane map of k_streamt: lane t takes storage position t, lanes kTailSecondLane + j also the
// shared node at position 256 + j.  Per node the arithmetic is that of k_lap / k_grad.
template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kTailThreads) void k_lapt(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, true>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    constexpr int NX = NLOC - kTailThreads;
    static_assert(S::EPB == 1 && NX > 0 && kTailSecondLane + NX <= kTailThreads && NP * NP <= kTailThreads &&
                  S::NINT <= kTailSecondLane,
                  "one element per block; second nodes on lanes whose first node is shared");
    __shared__ double sD[NP * NP];
    __shared__ double srho[NB];
    __shared__ double sv[D * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    const bool split = sd.Nint > 0;
    const int e = bs.local;
    const bool act = e < sd.E;
    const int m = tid;
    const int n = split ? split_node<D, NP>(m) : m;
    const int l = e * sd.lstride + m;
    const bool own = split && m < S::NINT;
    const int j = tid - kTailSecondLane;
    const bool two = act && j >= 0 && j < NX;
    const int m2 = kTailThreads + (two ? j : 0);
    const int n2 = split ? split_node<D, NP>(m2) : m2;
    const int l2 = e * sd.lstride + m2;
    double rh = 0.0, mi = 0.0, rh2 = 0.0;
    int G = 0;
    double g[S::NG];
    WallLap<D> wl;
    const double dmv = dm_fetch<NP>(sd, tid);
    if (two) {
        rh2 = sd.rho[sd.lgid[l2]];
        srho[n2] = rh2;
    }
    if (act) {
        G = sd.lgid[l];
#pragma unroll
        for (int k = 0; k < S::NG; ++k) g[k] = sd.G[(size_t)k * sd.Nl + l];
        load_wall_lap<D>(sd, l, wl);
        rh = sd.rho[G];
        if (own) mi = sd.Minv[G];
        srho[n] = rh;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (act) {
        double d[D];
        grad_ref<D, NP>(sD, srho, n, d);
        metric_times_grad<D, NB, S::NG>(g, d, sv, n);
    }
    if (two) {
        double g2[S::NG], d[D];
#pragma unroll
        for (int k = 0; k < S::NG; ++k) g2[k] = sd.G[(size_t)k * sd.Nl + l2];
        grad_ref<D, NP>(sD, srho, n2, d);
        metric_times_grad<D, NB, S::NG>(g2, d, sv, n2);
    }
    __syncthreads();
    if (!act) return;
    const double r = -div_refT<D, NP>(sD, sv, NB, n);
    if (own) sd.mu[G] = mu_of(sd, rh, (0.0 + r) * mi);  // no wall faces pass through an interior node
    else sd.rl[l] = wall_lap_term<D>(sd, wl, rh, r);
    if (two) {
        WallLap<D> wl2;
        load_wall_lap<D>(sd, l2, wl2);
        const double r2 = -div_refT<D, NP>(sD, sv, NB, n2);
        sd.rl[l2] = wall_lap_term<D>(sd, wl2, rh2, r2);
    }
}

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kTailThreads) void k_gradt(LaunchPlan p, int collide) {
    constexpr int D = DimOf<DQ>::v;
    constexpr int Q = QOfDQ<DQ>::v;
    using S = Shape<D, N, true>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    constexpr int NX = NLOC - kTailThreads;
    static_assert(S::EPB == 1 && NX > 0 && kTailSecondLane + NX <= kTailThreads && NP * NP <= kTailThreads &&
                  S::NINT <= kTailSecondLane,
                  "one element per block; second nodes on lanes whose first node is shared");
    __shared__ double sD[NP * NP];
    __shared__ double sf[2 * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    const bool split = sd.Nint > 0;
    const int e = bs.local;
    const bool act = e < sd.E;
    const int m = tid;
    const int n = split ? split_node<D, NP>(m) : m;
    const int l = e * sd.lstride + m;
    const bool own = collide && split && m < S::NINT;
    const int j = tid - kTailSecondLane;
    const bool two = act && j >= 0 && j < NX;
    const int m2 = kTailThreads + (two ? j : 0);
    const int n2 = split ? split_node<D, NP>(m2) : m2;
    const int l2 = e * sd.lstride + m2;
    const size_t Ng = sd.Ng;
    double J[D][D];
    double w = 0.0, pr = 0.0, mi = 0.0;
    double f[Q];
    int G = 0;
    const double dmv = dm_fetch<NP>(sd, tid);
    if (two) {
        const int G2 = sd.lgid[l2];
        sf[n2] = sd.rho[G2];
        sf[NB + n2] = sd.mu[G2];
    }
    if (act) {
        G = sd.lgid[l];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int c = 0; c < D; ++c) J[a][c] = sd.Ja[(size_t)(a * D + c) * sd.Nl + l];
        w = sd.wn[n];
        pr = sd.rho[G];
        sf[n] = pr;
        sf[NB + n] = sd.mu[G];
        if (own) {
            mi = sd.Minv[G];
#pragma unroll
            for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
        }
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
    double gs[2][D];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double d[D];
        grad_ref<D, NP>(sD, sf + k * NB, n, d);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) s += J[a][c] * d[a];
            gs[k][c] = w * s;
            if (!own) sd.gl[(size_t)(k * D + c) * sd.Nl + l] = gs[k][c];
        }
    }
    if (own) {
        double gr[D], gm[D], fs[Q];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = (0.0 + gs[0][c]) * mi;
            gm[c] = (0.0 + gs[1][c]) * mi;
        }
        collide_node<Q, D>(sd, f, pr, gr, gm, fs);
#pragma unroll
        for (int q = 0; q < Q; ++q) sd.g0[q * Ng + G] = fs[q];
    }
    if (two) {
        double J2[D][D];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int c = 0; c < D; ++c) J2[a][c] = sd.Ja[(size_t)(a * D + c) * sd.Nl + l2];
        const double w2 = sd.wn[n2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            double d[D];
            grad_ref<D, NP>(sD, sf + k * NB, n2, d);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) s += J2[a][c] * d[a];
                sd.gl[(size_t)(k * D + c) * sd.Nl + l2] = w2 * s;
            }
        }
    }
}

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kNodeThreads) void k_rk(LaunchPlan p, int stage) {
    constexpr int D = DimOf<DQ>::v;
    constexpr int Q = QOfDQ<DQ>::v;
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int G = sd.Nint + bs.local * kNodeThreads + threadIdx.x;  // interior nodes: k_stream
    if (G >= sd.Ng) return;
    const size_t Ng = sd.Ng, Nl = sd.Nl;
    const double SLBM_GLOBAL *gin = stage == 1 ? sd.g0 : sd.g1;
    double SLBM_GLOBAL *gout = stage == 3 ? sd.f : sd.g1;
    const NodeCopies cp = sd.gcopy[G];
    const double mi = sd.Minv[G], dt = sd.dt;
    // every load is issued before the first store: residuals of the first two copies,
    // the stage input and g0
    double x0[Q], x1[Q], gi[Q], g0v[Q];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        x0[q] = sd.rs[(size_t)(q - 1) * Nl + cp.i0];
        x1[q] = sd.rs[(size_t)(q - 1) * Nl + cp.i1];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) gi[q] = gin[q * Ng + G];
#pragma unroll
    for (int q = 0; q < Q; ++q) g0v[q] = 0.0;
    if (stage >= 2) {
#pragma unroll
        for (int q = 0; q < Q; ++q) g0v[q] = sd.g0[q * Ng + G];
    }
    double R[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) R[q] = 0.0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        R[q] += x0[q];
        R[q] += cp.nc > 1 ? x1[q] : 0.0;
    }
    // copies beyond the second (edges and corners): the indices of up to kCsrAhead of them
    // in one round trip, then their residuals two copies at a time, summed in copy order
    for (int k = 2; k < cp.nc; k += kCsrAhead) {
        int li[kCsrAhead];
#pragma unroll
        for (int j = 0; j < kCsrAhead; ++j) li[j] = k + j < cp.nc ? sd.csr_idx[cp.k0 + k + j] : -1;
#pragma unroll
        for (int j = 0; j < kCsrAhead; j += 2) {
            if (li[j] >= 0) {
                double xa[Q], xb[Q];
#pragma unroll
                for (int q = 1; q < Q; ++q) {
                    xa[q] = sd.rs[(size_t)(q - 1) * Nl + li[j]];
                    xb[q] = li[j + 1] >= 0 ? sd.rs[(size_t)(q - 1) * Nl + li[j + 1]] : 0.0;
                }
#pragma unroll
                for (int q = 1; q < Q; ++q) R[q] += xa[q];
                if (li[j + 1] >= 0) {
#pragma unroll
                    for (int q = 1; q < Q; ++q) R[q] += xb[q];
                }
            }
        }
    }
    double rho = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double L = q > 0 ? R[q] * mi : 0.0;
        const double out = rk_combine<Q>(stage, L, gi[q], g0v[q], dt);
        gout[q * Ng + G] = out;
        rho += out;
    }
    sd.rho[G] = rho;
}

// rho = sum_a f_a (Eq. (10)) of the state (which = 0) or of g1 (which = 1)
template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kNodeThreads) void k_density(LaunchPlan p, int which) {
    constexpr int D = DimOf<DQ>::v;
    constexpr int Q = QOfDQ<DQ>::v;
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int G = bs.local * kNodeThreads + threadIdx.x;
    if (G >= sd.Ng) return;
    const double SLBM_GLOBAL *src = which == 0 ? sd.f : sd.g1;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += src[(size_t)q * sd.Ng + G];
    sd.rho[G] = s;
}

// KE_max = max 1/2 rho |u|^2 and mass = sum M rho; per-block partials in red[]
template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kNodeThreads) void k_diag(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    constexpr int Q = QOfDQ<DQ>::v;
    __shared__ double smax[kNodeThreads], ssum[kNodeThreads];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    const int G = bs.local * kNodeThreads + tid;
    double ke = 0.0, ms = 0.0;
    if (G < sd.Ng) {
        const size_t Ng = sd.Ng;
        double f[Q];
        double pr = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            f[q] = sd.f[q * Ng + G];
            pr += f[q];
        }
        double uu = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double m = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) m = acc_e<Q>(m, f[q], q, c, sd);
            const double u = m / pr;
            uu += u * u;
        }
        ke = 0.5 * pr * uu;
        ms = (1.0 / sd.Minv[G]) * pr;
    }
    smax[tid] = ke;
    ssum[tid] = ms;
    __syncthreads();
    for (int s = kNodeThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double a = smax[tid], b = smax[tid + s];
            smax[tid] = (a >= b || a != a) ? a : b;  // NaN propagates
            ssum[tid] += ssum[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        sd.red[2 * bs.local] = smax[0];
        sd.red[2 * bs.local + 1] = ssum[0];
    }
}

// ------------------------------------------------------------------------------------------
// Fused path.  Each element kernel finishes the previous pass's direct stiffness summation
// itself: every thread gathers the per-copy partial sums of all local copies of its node
// (ascending local order, the same sum as the node kernels) and applies the pointwise
// update; the lowest local copy ("owner") stores the node's global value.  Shared nodes
// are thus updated redundantly and identically by each element that holds them, which
// halves the number of grid-wide dependencies of a step (7 kernels instead of 14).
// ------------------------------------------------------------------------------------------

// Copy list of local node l in registers (K slots: 4 in 2-D, 8 in 3-D), ascending; slots
// beyond the node's copies repeat the first copy.  Two gather forms, both with all loads of
// a gather in flight together and both summing in ascending order:
//   * PRED (wide blocks, bandwidth bound): element-interior nodes skip their copy list and
//     slot k is loaded only in lanes with more than k copies (predicated loads);
//   * branch-free (one element per block, latency bound): every slot is loaded and the
//     unused ones are masked out of the sum, adding +0.0 after the real terms (the sum
//     starts from +0.0 and never becomes -0.0, so the result is the same).
template <int D> struct CopyList {
    static constexpr int K = kCopySlots[D - 2];
    int cp[K];
    int nc;
};
template <int D, int NP, bool PRED>
__device__ __forceinline__ void load_copies(const SolveDesc &sd, int n, int l, CopyList<D> &c) {
    c.cp[0] = l;
    c.nc = 1;
#pragma unroll
    for (int k = 1; k < CopyList<D>::K; ++k) c.cp[k] = l;
    if (!PRED || on_elem_boundary<D, NP>(n)) {
        // all K rows of the table exist (-1 padded): the slot loads go out together
        int v[CopyList<D>::K];
#pragma unroll
        for (int k = 0; k < CopyList<D>::K; ++k) v[k] = sd.lcp[(size_t)k * sd.Nl + l];
        c.nc = 1;
#pragma unroll
        for (int k = 1; k < CopyList<D>::K; ++k) c.nc += v[k] >= 0 ? 1 : 0;
        c.cp[0] = v[0];
#pragma unroll
        for (int k = 1; k < CopyList<D>::K; ++k) c.cp[k] = v[k] >= 0 ? v[k] : v[0];
    }
}

template <int D, bool PRED, class P>
__device__ __forceinline__ double gather1(P v, const CopyList<D> &c) {
    double x[CopyList<D>::K];
    double s = 0.0;
    if constexpr (PRED) {
        x[0] = v[c.cp[0]];
#pragma unroll
        for (int k = 1; k < CopyList<D>::K; ++k) {
            x[k] = 0.0;
            if (k < c.nc) x[k] = v[c.cp[k]];
        }
        s += x[0];
#pragma unroll
        for (int k = 1; k < CopyList<D>::K; ++k)
            if (k < c.nc) s += x[k];
    } else {
#pragma unroll
        for (int k = 0; k < CopyList<D>::K; ++k) x[k] = v[c.cp[k]];
        s += x[0];  // every node has its first copy
#pragma unroll
        for (int k = 1; k < CopyList<D>::K; ++k) s += k < c.nc ? x[k] : 0.0;
    }
    return s;
}

// A: mu of the state's density (DSS of the Laplacian partials) and the lumped-mass
// weighted element gradients of rho and mu for the collision
template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT)) void k_fA(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    __shared__ double sD[NP * NP];
    __shared__ double sf[2 * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    double dmv = 0.0;  // fetched by the active lanes (every lane below (N+1)^2 is active)
    const int es = tid / NLOC, n = tid - es * NLOC;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * NLOC + n;
    double J[D][D];
    double w = 0.0;
    if (act) {
        dmv = dm_fetch<NP>(sd, tid);
        CopyList<D> cl;
        load_copies<D, NP, WIDE>(sd, n, l, cl);
        const int G = sd.lgid[l];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int c = 0; c < D; ++c) J[a][c] = sd.Ja[(size_t)(a * D + c) * sd.Nl + l];
        w = sd.wn[n];
        const double pr = sd.rho[G];
        const double mu = mu_of(sd, pr, gather1<D, WIDE>(sd.rl, cl) * sd.Minv[G]);
        if (cl.cp[0] == l) sd.mu[G] = mu;
        sf[tid] = pr;
        sf[NB + tid] = mu;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        double d[D];
        grad_ref<D, NP>(sD, sf + f * NB + es * NLOC, n, d);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) s += J[a][c] * d[a];
            sd.gl[(size_t)(f * D + c) * sd.Nl + l] = w * s;
        }
    }
}

// B: averaged gradients (DSS), collision (Eq. (4)) at every element node, owners store f*
// in g0, then the stage-1 streaming residual of f*
template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT)) void k_fB(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    __shared__ double sD[NP * NP];
    __shared__ double smu[NB];
    __shared__ double sh[(Q - 1) * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    double dmv = 0.0;  // fetched by the active lanes (every lane below (N+1)^2 is active)
    const int es = tid / NLOC, n = tid - es * NLOC;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * NLOC + n;
    const size_t Ng = sd.Ng;
    double fs[Q];
    double pr = 0.0;
    NodeGeo<D> geo;
    if (act) {
        dmv = dm_fetch<NP>(sd, tid);
        CopyList<D> cl;
        load_copies<D, NP, WIDE>(sd, n, l, cl);
        const int G = sd.lgid[l];
        load_geo<D>(sd, n, l, geo);
        const double mi = sd.Minv[G];
        double gr[D], gm[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = gather1<D, WIDE>(sd.gl + (size_t)c * sd.Nl, cl) * mi;
            gm[c] = gather1<D, WIDE>(sd.gl + (size_t)(D + c) * sd.Nl, cl) * mi;
        }
        double f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
        pr = sd.rho[G];
        const double mu = sd.mu[G];
        collide_node<Q, D>(sd, f, pr, gr, gm, fs);
        if (cl.cp[0] == l) {
#pragma unroll
            for (int q = 0; q < Q; ++q) sd.g0[q * Ng + G] = fs[q];
        }
        smu[tid] = mu;
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + tid] = fs[q] - sd.tw[wcls<Q>(q)] * pr;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
    stream_residual<Q, D, N, WIDE>(sd, sD, sh, smu + es * NLOC, es, n, l, pr, fs, geo);
}

// C: DSS of the streaming residual, SSP-RK3 combination and the stage density at every
// element node (owners store them), then the Laplacian partials of the new density
//   stage 1: g1 = g0 + dt L;  stage 2: g2 = 3/4 g0 + 1/4 (g1 + dt L);
//   stage 3: f = (g0 + 2 (g2 + dt L)) / 3
template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT)) void k_fC(LaunchPlan p, int stage) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    constexpr int K = CopyList<D>::K;
    __shared__ double sD[NP * NP];
    __shared__ double srho[NB];
    __shared__ double sv[D * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    double dmv = 0.0;  // fetched by the active lanes (every lane below (N+1)^2 is active)
    const int es = tid / NLOC, n = tid - es * NLOC;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * NLOC + n;
    const size_t Ng = sd.Ng, Nl = sd.Nl;
    const double SLBM_GLOBAL *gin = stage == 1 ? sd.g0 : (stage == 2 ? sd.g1 : sd.g2);
    double SLBM_GLOBAL *gout = stage == 1 ? sd.g1 : (stage == 2 ? sd.g2 : sd.f);
    double rho = 0.0;
    double gm[S::NG];
    WallLap<D> wl;
    if (act) {
        dmv = dm_fetch<NP>(sd, tid);
        CopyList<D> cl;
        load_copies<D, NP, WIDE>(sd, n, l, cl);
        const int G = sd.lgid[l];
#pragma unroll
        for (int k = 0; k < S::NG; ++k) gm[k] = sd.G[(size_t)k * Nl + l];
        load_wall_lap<D>(sd, l, wl);
        // every load before the first store: residual partials of all copies, the stage
        // input and g0
        // (3-D: the first two slots; copies of edge and corner nodes beyond them in a loop,
        // which keeps the register footprint of 8 slots x 18 populations away)
        constexpr int KU = D == 2 ? K : 2;
        double R[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = 0.0;
        double x[KU][Q];
#pragma unroll
        for (int k = 0; k < KU; ++k) {
#pragma unroll
            for (int q = 1; q < Q; ++q) x[k][q] = 0.0;
            if (!WIDE || k == 0 || k < cl.nc) {
#pragma unroll
                for (int q = 1; q < Q; ++q) x[k][q] = sd.rs[(size_t)(q - 1) * Nl + cl.cp[k]];
            }
        }
#pragma unroll
        for (int k = 0; k < KU; ++k) {
            const bool valid = k < cl.nc;
            if (WIDE || k == 0) {
                if (k == 0 || valid) {
#pragma unroll
                    for (int q = 1; q < Q; ++q) R[q] += x[k][q];
                }
            } else {
#pragma unroll
                for (int q = 1; q < Q; ++q) R[q] += valid ? x[k][q] : 0.0;
            }
        }
        if constexpr (KU < K) {
            for (int k = KU; k < cl.nc; ++k) {
                double x[Q];
                const int c = k == 2 ? cl.cp[2] : (k == 3 ? cl.cp[3] : (k == 4 ? cl.cp[4] :
                              (k == 5 ? cl.cp[5] : (k == 6 ? cl.cp[6] : cl.cp[7]))));
#pragma unroll
                for (int q = 1; q < Q; ++q) x[q] = sd.rs[(size_t)(q - 1) * Nl + c];
#pragma unroll
                for (int q = 1; q < Q; ++q) R[q] += x[q];
            }
        }
        double gi[Q], g0v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) gi[q] = gin[q * Ng + G];
#pragma unroll
        for (int q = 0; q < Q; ++q) g0v[q] = 0.0;
        if (stage != 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) g0v[q] = sd.g0[q * Ng + G];
        }
        const double mi = sd.Minv[G], dt = sd.dt;
        const bool owner = cl.cp[0] == l;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double L = q > 0 ? R[q] * mi : 0.0;
            const double out = rk_combine<Q>(stage, L, gi[q], g0v[q], dt);
            rho += out;
            if (owner) gout[q * Ng + G] = out;
        }
        if (owner) sd.rho[G] = rho;
        srho[tid] = rho;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (act) {
        double d[D];
        grad_ref<D, NP>(sD, srho + es * NLOC, n, d);
        metric_times_grad<D, NB, S::NG>(gm, d, sv, tid);
    }
    __syncthreads();
    if (!act) return;
    const double r = -div_refT<D, NP>(sD, sv + es * NLOC, NB, n);
    sd.rl[l] = wall_lap_term<D>(sd, wl, rho, r);
}

// D: mu of the stage density (DSS of the Laplacian partials) and the streaming residual of
// stage 2 (g1) or 3 (g2)
template <int DQ, int N, bool WIDE, bool SINGLE>
__global__ __launch_bounds__((Shape<DimOf<DQ>::v, N, WIDE>::NT)) void k_fD(LaunchPlan p, int stage) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, WIDE>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    __shared__ double sD[NP * NP];
    __shared__ double smu[NB];
    __shared__ double sh[(Q - 1) * NB];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    double dmv = 0.0;  // fetched by the active lanes (every lane below (N+1)^2 is active)
    const int es = tid / NLOC, n = tid - es * NLOC;
    const int e = bs.local * S::EPB + es;
    const bool act = tid < NB && e < sd.E;
    const int l = e * NLOC + n;
    const size_t Ng = sd.Ng;
    const double SLBM_GLOBAL *g = stage == 2 ? sd.g1 : sd.g2;
    double gq[Q];
    double pr = 0.0;
    NodeGeo<D> geo;
    if (act) {
        dmv = dm_fetch<NP>(sd, tid);
        CopyList<D> cl;
        load_copies<D, NP, WIDE>(sd, n, l, cl);
        const int G = sd.lgid[l];
        load_geo<D>(sd, n, l, geo);
        pr = sd.rho[G];
        smu[tid] = mu_of(sd, pr, gather1<D, WIDE>(sd.rl, cl) * sd.Minv[G]);
#pragma unroll
        for (int q = 0; q < Q; ++q) gq[q] = g[q * Ng + G];
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + tid] = gq[q] - sd.tw[wcls<Q>(q)] * pr;
    }
    dm_store<NP>(sD, tid, dmv);
    __syncthreads();
    if (!act) return;
    stream_residual<Q, D, N, WIDE>(sd, sD, sh, smu + es * NLOC, es, n, l, pr, gq, geo);
}

// ------------------------------------------------------------------------------------------
// B and D for elements of more than 256 nodes (2-D N = 16: 289) in blocks of four waves:
// lane t handles node t, and lanes t < NLOC - 256 also node 256 + t.  With one lane per
// node such an element needs a fifth wave, and blocks of five waves keep about half as
// many waves resident per compute unit as blocks of four.  The second node's LDS inputs
// are written first; what its residuals need across the barrier (f* or g, and rho) goes
// through LDS, its metrics are read again after the barrier.  Every node's and every
// population's arithmetic is that of k_fB / k_fD (wide instances), so the results are the
// same bits.  Launched for meshes of many blocks (kTailMinBlocks); the fifth wave is faster
// where few blocks share a compute unit.
// ------------------------------------------------------------------------------------------
template <int DD, int NN> constexpr bool kTail =
    DimOf<DD>::v == 2 && Shape<2, NN, true>::NLOC > kTailThreads && Shape<2, NN, true>::NLOC <= 2 * kTailThreads;

// After the barrier the residuals of the second nodes are spread over the four waves: lane
// j < NLOC - 256 of wave w computes populations 1 + w (Q-1)/4 .. (w+1) (Q-1)/4 of node
// 256 + j, so every wave adds a quarter of a node's residuals instead of the first wave
// adding a whole node's (g or f* and rho of the second nodes come from LDS sx)
template <int Q, int D, int N, int QA, int QN>
__device__ __forceinline__ void tail_residuals(const SolveDesc &sd, const double *sD, const double *sh,
                                               const double *smu, const double *sx, int e, int j) {
    using S = Shape<D, N, true>;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB, NX = NLOC - kTailThreads;
    const int n2 = kTailThreads + j, l2 = e * NLOC + n2;
    NodeGeo<D> geo;
    load_geo<D>(sd, n2, l2, geo);
    const double p2 = sx[Q * NX + j];
    double dmu[D];
    grad_ref<D, NP>(sD, smu, n2, dmu);
#pragma unroll
    for (int k = 0; k < QN; ++k) {
        const int q = QA + k;
        const double r = residual_q<Q, D, NP>(sd, q, sD, sh + (q - 1) * NB, n2, dmu, p2, sx[q * NX + j],
                                              sx[Lat<Q>::opp[q] * NX + j], geo);
        sd.rs[(size_t)(q - 1) * sd.Nl + l2] = r;
    }
}
template <int Q, int D, int N>
__device__ __forceinline__ void tail_residuals_spread(const SolveDesc &sd, const double *sD, const double *sh,
                                                      const double *smu, const double *sx, int e, int tid) {
    constexpr int NX = Shape<D, N, true>::NLOC - kTailThreads;
    constexpr int QN = (Q - 1) / 4;
    static_assert((Q - 1) % 4 == 0 && kTailThreads == 4 * 64, "four waves, equal shares of populations");
    const int j = tid & 63, w = tid >> 6;
    if (j >= NX) return;
    if (w == 0) tail_residuals<Q, D, N, 1, QN>(sd, sD, sh, smu, sx, e, j);
    else if (w == 1) tail_residuals<Q, D, N, 1 + QN, QN>(sd, sD, sh, smu, sx, e, j);
    else if (w == 2) tail_residuals<Q, D, N, 1 + 2 * QN, QN>(sd, sD, sh, smu, sx, e, j);
    else tail_residuals<Q, D, N, 1 + 3 * QN, QN>(sd, sD, sh, smu, sx, e, j);
}

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kTailThreads) void k_fBt(LaunchPlan p) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, true>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    constexpr int NX = NLOC - kTailThreads;  // nodes of the second pass
    static_assert(S::EPB == 1 && NX > 0 && NX <= kTailThreads && NP * NP <= 2 * kTailThreads,
                  "one element per block, at most two nodes and two matrix entries per lane");
    __shared__ double sD[NP * NP];
    __shared__ double smu[NB];
    __shared__ double sh[(Q - 1) * NB];
    __shared__ double sx[(Q + 1) * NX];  // second nodes: f*_q, then rho
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    const int e = bs.local;
    const bool act = e < sd.E;
    const bool two = act && tid < NX;
    const int n = tid, n2 = kTailThreads + tid;
    const int l = e * NLOC + n, l2 = e * NLOC + (two ? n2 : n);
    const size_t Ng = sd.Ng;
    double dmv = 0.0, dmv2 = 0.0;
    double fs[Q];
    double pr = 0.0;
    NodeGeo<D> geo;
    if (act) {
        dmv = sd.Dm[tid];
        dmv2 = sd.Dm[n2 < NP * NP ? n2 : 0];
    }
    if (two) {
        CopyList<D> cl;
        load_copies<D, NP, true>(sd, n2, l2, cl);
        const int G = sd.lgid[l2];
        const double mi = sd.Minv[G];
        double gr[D], gm[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = gather1<D, true>(sd.gl + (size_t)c * sd.Nl, cl) * mi;
            gm[c] = gather1<D, true>(sd.gl + (size_t)(D + c) * sd.Nl, cl) * mi;
        }
        double f[Q], f2[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
        const double p2 = sd.rho[G];
        const double mu = sd.mu[G];
        collide_node<Q, D>(sd, f, p2, gr, gm, f2);
        if (cl.cp[0] == l2) {
#pragma unroll
            for (int q = 0; q < Q; ++q) sd.g0[q * Ng + G] = f2[q];
        }
        smu[n2] = mu;
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + n2] = f2[q] - sd.tw[wcls<Q>(q)] * p2;
#pragma unroll
        for (int q = 0; q < Q; ++q) sx[q * NX + tid] = f2[q];
        sx[Q * NX + tid] = p2;
    }
    if (act) {
        CopyList<D> cl;
        load_copies<D, NP, true>(sd, n, l, cl);
        const int G = sd.lgid[l];
        load_geo<D>(sd, n, l, geo);
        const double mi = sd.Minv[G];
        double gr[D], gm[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = gather1<D, true>(sd.gl + (size_t)c * sd.Nl, cl) * mi;
            gm[c] = gather1<D, true>(sd.gl + (size_t)(D + c) * sd.Nl, cl) * mi;
        }
        double f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
        pr = sd.rho[G];
        const double mu = sd.mu[G];
        collide_node<Q, D>(sd, f, pr, gr, gm, fs);
        if (cl.cp[0] == l) {
#pragma unroll
            for (int q = 0; q < Q; ++q) sd.g0[q * Ng + G] = fs[q];
        }
        smu[n] = mu;
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + n] = fs[q] - sd.tw[wcls<Q>(q)] * pr;
    }
    sD[tid] = dmv;
    if (n2 < NP * NP) sD[n2] = dmv2;
    __syncthreads();
    if (!act) return;
    stream_residual<Q, D, N, true>(sd, sD, sh, smu, 0, n, l, pr, fs, geo);
    tail_residuals_spread<Q, D, N>(sd, sD, sh, smu, sx, e, tid);
}

template <int DQ, int N, bool SINGLE>
__global__ __launch_bounds__(kTailThreads) void k_fDt(LaunchPlan p, int stage) {
    constexpr int D = DimOf<DQ>::v;
    using S = Shape<D, N, true>;
    constexpr int Q = QOfDQ<DQ>::v;
    constexpr int NP = S::NP, NLOC = S::NLOC, NB = S::NB;
    constexpr int NX = NLOC - kTailThreads;
    static_assert(S::EPB == 1 && NX > 0 && NX <= kTailThreads && NP * NP <= 2 * kTailThreads,
                  "one element per block, at most two nodes and two matrix entries per lane");
    __shared__ double sD[NP * NP];
    __shared__ double smu[NB];
    __shared__ double sh[(Q - 1) * NB];
    __shared__ double sx[(Q + 1) * NX];  // second nodes: g_q, then rho
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x;
    const int e = bs.local;
    const bool act = e < sd.E;
    const bool two = act && tid < NX;
    const int n = tid, n2 = kTailThreads + tid;
    const int l = e * NLOC + n, l2 = e * NLOC + (two ? n2 : n);
    const size_t Ng = sd.Ng;
    const double SLBM_GLOBAL *g = stage == 2 ? sd.g1 : sd.g2;
    double dmv = 0.0, dmv2 = 0.0;
    double gq[Q];
    double pr = 0.0;
    NodeGeo<D> geo;
    if (act) {
        dmv = sd.Dm[tid];
        dmv2 = sd.Dm[n2 < NP * NP ? n2 : 0];
    }
    if (two) {
        CopyList<D> cl;
        load_copies<D, NP, true>(sd, n2, l2, cl);
        const int G = sd.lgid[l2];
        const double p2 = sd.rho[G];
        smu[n2] = mu_of(sd, p2, gather1<D, true>(sd.rl, cl) * sd.Minv[G]);
        double g2[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) g2[q] = g[q * Ng + G];
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + n2] = g2[q] - sd.tw[wcls<Q>(q)] * p2;
#pragma unroll
        for (int q = 0; q < Q; ++q) sx[q * NX + tid] = g2[q];
        sx[Q * NX + tid] = p2;
    }
    if (act) {
        CopyList<D> cl;
        load_copies<D, NP, true>(sd, n, l, cl);
        const int G = sd.lgid[l];
        load_geo<D>(sd, n, l, geo);
        pr = sd.rho[G];
        smu[n] = mu_of(sd, pr, gather1<D, true>(sd.rl, cl) * sd.Minv[G]);
#pragma unroll
        for (int q = 0; q < Q; ++q) gq[q] = g[q * Ng + G];
#pragma unroll
        for (int q = 1; q < Q; ++q) sh[(q - 1) * NB + n] = gq[q] - sd.tw[wcls<Q>(q)] * pr;
    }
    sD[tid] = dmv;
    if (n2 < NP * NP) sD[n2] = dmv2;
    __syncthreads();
    if (!act) return;
    stream_residual<Q, D, N, true>(sd, sD, sh, smu, 0, n, l, pr, gq, geo);
    tail_residuals_spread<Q, D, N>(sd, sD, sh, smu, sx, e, tid);
}

// ------------------------------------------------------------------------------------------
// 2-D fused kernels B, C, D for one element per block (the latency-bound regime), with the
// populations split over four groups of lanes: group g handles the opposite pair
// (qa, opp(qa)), qa = 1, 2, 5, 6, and group 0 also q = 0.  Every group holds the whole
// element (one lane per node); per-node quantities every group needs (moments, mu) are
// computed by each group with the same arithmetic.  A wave thus runs a quarter of the
// population work, and four waves per element fill the SIMDs that one wave per element
// leaves idle.  Arithmetic and summation orders are those of k_fB, k_fC, k_fD.
// ------------------------------------------------------------------------------------------
template <int N> struct Split2 {
    static constexpr int NP = N + 1;
    static constexpr int NLOC = NP * NP;
    static constexpr int NTP = ((NLOC + 63) / 64) * 64;  // lanes of one group
    static constexpr int NT = 4 * NTP;
};
// first population of group g's pair (the second is Lat<9>::opp of it)
template <int G> struct PairOf;
template <> struct PairOf<0> { static constexpr int qa = 1; };
template <> struct PairOf<1> { static constexpr int qa = 2; };
template <> struct PairOf<2> { static constexpr int qa = 5; };
template <> struct PairOf<3> { static constexpr int qa = 6; };

// call f(GroupC<g>{}) for the calling group g (uniform within a wave)
template <int G> struct GroupC { static constexpr int value = G; };
template <class F>
__device__ __forceinline__ void for_group(int grp, F &&f) {
    switch (grp) {
    case 0: f(GroupC<0>{}); break;
    case 1: f(GroupC<1>{}); break;
    case 2: f(GroupC<2>{}); break;
    default: f(GroupC<3>{}); break;
    }
}

template <int N, bool SINGLE>
__global__ __launch_bounds__(Split2<N>::NT) void k_fB4(LaunchPlan p) {
    using S = Split2<N>;
    constexpr int D = 2, Q = 9, NP = S::NP, NLOC = S::NLOC, NTP = S::NTP;
    __shared__ double sD[NP * NP];
    __shared__ double smu[NTP];
    __shared__ double sh[(Q - 1) * NTP];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x, grp = tid / NTP, n = tid - grp * NTP;
    const int e = bs.local;
    const bool act = n < NLOC && e < sd.E;
    const int l = e * NLOC + n;
    const size_t Ng = sd.Ng;
    double dmv = 0.0;
    double pr = 0.0, fa = 0.0, fb = 0.0;
    NodeGeo<D> geo;
    if (act) {
        if (grp == 0) dmv = dm_fetch<NP>(sd, n);
        CopyList<D> cl;
        load_copies<D, NP, false>(sd, n, l, cl);
        const int G = sd.lgid[l];
        load_geo<D>(sd, n, l, geo);
        const double mi = sd.Minv[G];
        double gr[D], gm[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            gr[c] = gather1<D, false>(sd.gl + (size_t)c * sd.Nl, cl) * mi;
            gm[c] = gather1<D, false>(sd.gl + (size_t)(D + c) * sd.Nl, cl) * mi;
        }
        double f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sd.f[q * Ng + G];
        pr = sd.rho[G];
        const double mu = sd.mu[G];
        CollidePrep<Q, D> cp;
        collide_prep<Q, D>(sd, f, pr, gr, gm, cp);
        const bool owner = cl.cp[0] == l;
        for_group(grp, [&](auto gc) {
            constexpr int qa = PairOf<decltype(gc)::value>::qa, qb = Lat<Q>::opp[qa];
            fa = collide_q<Q, D>(sd, qa, f[qa], pr, cp);
            fb = collide_q<Q, D>(sd, qb, f[qb], pr, cp);
            if (owner) {
                sd.g0[qa * Ng + G] = fa;
                sd.g0[qb * Ng + G] = fb;
                if (decltype(gc)::value == 0) sd.g0[G] = collide_q<Q, D>(sd, 0, f[0], pr, cp);
            }
            sh[(qa - 1) * NTP + n] = fa - sd.tw[wcls<Q>(qa)] * pr;
            sh[(qb - 1) * NTP + n] = fb - sd.tw[wcls<Q>(qb)] * pr;
        });
        if (grp == 0) smu[n] = mu;
    }
    if (grp == 0) dm_store<NP>(sD, n, dmv);
    __syncthreads();
    if (!act) return;
    double dmu[D];
    grad_ref<D, NP>(sD, smu, n, dmu);
    for_group(grp, [&](auto gc) {
        constexpr int qa = PairOf<decltype(gc)::value>::qa, qb = Lat<Q>::opp[qa];
        const double ra = residual_q<Q, D, NP>(sd, qa, sD, sh + (qa - 1) * NTP, n, dmu, pr, fa, fb, geo);
        const double rb = residual_q<Q, D, NP>(sd, qb, sD, sh + (qb - 1) * NTP, n, dmu, pr, fb, fa, geo);
        sd.rs[(size_t)(qa - 1) * sd.Nl + l] = ra;
        sd.rs[(size_t)(qb - 1) * sd.Nl + l] = rb;
    });
}

template <int N, bool SINGLE>
__global__ __launch_bounds__(Split2<N>::NT) void k_fC4(LaunchPlan p, int stage) {
    using S = Split2<N>;
    constexpr int D = 2, Q = 9, NP = S::NP, NLOC = S::NLOC, NTP = S::NTP;
    constexpr int K = CopyList<D>::K;
    __shared__ double sD[NP * NP];
    __shared__ double sout[Q * NTP];
    __shared__ double srho[NTP];
    __shared__ double sv[D * NTP];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x, grp = tid / NTP, n = tid - grp * NTP;
    const int e = bs.local;
    const bool act = n < NLOC && e < sd.E;
    const int l = e * NLOC + n;
    const size_t Ng = sd.Ng, Nl = sd.Nl;
    const double SLBM_GLOBAL *gin = stage == 1 ? sd.g0 : (stage == 2 ? sd.g1 : sd.g2);
    double SLBM_GLOBAL *gout = stage == 1 ? sd.g1 : (stage == 2 ? sd.g2 : sd.f);
    double dmv = 0.0;
    double gm[3] = {0.0, 0.0, 0.0};
    WallLap<D> wl;
    wl.cnt = 0;
    bool owner = false;
    int G = 0;
    if (act) {
        CopyList<D> cl;
        load_copies<D, NP, false>(sd, n, l, cl);
        G = sd.lgid[l];
        owner = cl.cp[0] == l;
        if (grp == 0) {
            dmv = dm_fetch<NP>(sd, n);
#pragma unroll
            for (int k = 0; k < 3; ++k) gm[k] = sd.G[(size_t)k * Nl + l];
            load_wall_lap<D>(sd, l, wl);
        }
        const double mi = sd.Minv[G], dt = sd.dt;
        // DSS of the residual of q over the copies and the RK combination; q = 0 has L = 0
        auto one = [&](int q, double gi, double g0) {
            double L = 0.0;
            if (q > 0) {
                double x[K];
#pragma unroll
                for (int k = 0; k < K; ++k) x[k] = sd.rs[(size_t)(q - 1) * Nl + cl.cp[k]];
                double R = 0.0;
                R += x[0];
#pragma unroll
                for (int k = 1; k < K; ++k) R += k < cl.nc ? x[k] : 0.0;
                L = R * mi;
            }
            return rk_combine<Q>(stage, L, gi, g0, dt);
        };
        for_group(grp, [&](auto gc) {
            constexpr int GR = decltype(gc)::value;
            constexpr int qa = PairOf<GR>::qa, qb = Lat<Q>::opp[qa];
            const double gia = gin[qa * Ng + G], gib = gin[qb * Ng + G];
            const double gi0 = GR == 0 ? gin[G] : 0.0;
            double g0a = 0.0, g0b = 0.0, g00 = 0.0;
            if (stage != 1) {
                g0a = sd.g0[qa * Ng + G];
                g0b = sd.g0[qb * Ng + G];
                if (GR == 0) g00 = sd.g0[G];
            }
            const double oa = one(qa, gia, g0a), ob = one(qb, gib, g0b);
            sout[qa * NTP + n] = oa;
            sout[qb * NTP + n] = ob;
            if (owner) {
                gout[qa * Ng + G] = oa;
                gout[qb * Ng + G] = ob;
            }
            if (GR == 0) {
                const double o0 = one(0, gi0, g00);
                sout[n] = o0;
                if (owner) gout[G] = o0;
            }
        });
    }
    if (grp == 0) dm_store<NP>(sD, n, dmv);
    __syncthreads();
    // stage density in ascending population order, then the Laplacian partials (group 0)
    double rho = 0.0;
    if (act && grp == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) rho += sout[q * NTP + n];
        if (owner) sd.rho[G] = rho;
        srho[n] = rho;
    }
    __syncthreads();
    if (act && grp == 0) {
        double d[D];
        grad_ref<D, NP>(sD, srho, n, d);
        metric_times_grad<D, NTP, 3>(gm, d, sv, n);
    }
    __syncthreads();
    if (!act || grp != 0) return;
    const double r = -div_refT<D, NP>(sD, sv, NTP, n);
    sd.rl[l] = wall_lap_term<D>(sd, wl, rho, r);
}

template <int N, bool SINGLE>
__global__ __launch_bounds__(Split2<N>::NT) void k_fD4(LaunchPlan p, int stage) {
    using S = Split2<N>;
    constexpr int D = 2, Q = 9, NP = S::NP, NLOC = S::NLOC, NTP = S::NTP;
    __shared__ double sD[NP * NP];
    __shared__ double smu[NTP];
    __shared__ double sh[(Q - 1) * NTP];
    const BlockSlot bs = block_slot<SINGLE>(p);
    if (!bs.valid) return;
    const SolveDesc sd = desc_of<SINGLE>(p, bs);
    const int tid = threadIdx.x, grp = tid / NTP, n = tid - grp * NTP;
    const int e = bs.local;
    const bool act = n < NLOC && e < sd.E;
    const int l = e * NLOC + n;
    const size_t Ng = sd.Ng;
    const double SLBM_GLOBAL *g = stage == 2 ? sd.g1 : sd.g2;
    double dmv = 0.0;
    double pr = 0.0, ga = 0.0, gb = 0.0;
    NodeGeo<D> geo;
    if (act) {
        if (grp == 0) dmv = dm_fetch<NP>(sd, n);
        CopyList<D> cl;
        load_copies<D, NP, false>(sd, n, l, cl);
        const int G = sd.lgid[l];
        load_geo<D>(sd, n, l, geo);
        pr = sd.rho[G];
        const double mu = mu_of(sd, pr, gather1<D, false>(sd.rl, cl) * sd.Minv[G]);
        if (grp == 0) smu[n] = mu;
        for_group(grp, [&](auto gc) {
            constexpr int qa = PairOf<decltype(gc)::value>::qa, qb = Lat<Q>::opp[qa];
            ga = g[qa * Ng + G];
            gb = g[qb * Ng + G];
            sh[(qa - 1) * NTP + n] = ga - sd.tw[wcls<Q>(qa)] * pr;
            sh[(qb - 1) * NTP + n] = gb - sd.tw[wcls<Q>(qb)] * pr;
        });
    }
    if (grp == 0) dm_store<NP>(sD, n, dmv);
    __syncthreads();
    if (!act) return;
    double dmu[D];
    grad_ref<D, NP>(sD, smu, n, dmu);
    for_group(grp, [&](auto gc) {
        constexpr int qa = PairOf<decltype(gc)::value>::qa, qb = Lat<Q>::opp[qa];
        const double ra = residual_q<Q, D, NP>(sd, qa, sD, sh + (qa - 1) * NTP, n, dmu, pr, ga, gb, geo);
        const double rb = residual_q<Q, D, NP>(sd, qb, sD, sh + (qb - 1) * NTP, n, dmu, pr, gb, ga, geo);
        sd.rs[(size_t)(qa - 1) * sd.Nl + l] = ra;
        sd.rs[(size_t)(qb - 1) * sd.Nl + l] = rb;
    });
}

// narrow (one element per block) launches of B, C, D: the population-split kernels in 2-D
// where four groups of an element's lanes fit in one block of at most 1024 threads
// (N <= 14), the one-lane-per-node kernels otherwise
template <int DD, int NN> constexpr bool kSplit = DD == 2 && Split2<NN>::NT <= 1024;
template <int DD, int NN, bool S>
inline void launch_narrow_fB(const LaunchPlan &p, hipStream_t st) {
    if constexpr (kSplit<DD, NN>) k_fB4<NN, S><<<p.grid, Split2<NN>::NT, 0, st>>>(p);
    else k_fB<DD, NN, false, S><<<p.grid, Shape<DimOf<DD>::v, NN, false>::NT, 0, st>>>(p);
}
template <int DD, int NN, bool S>
inline void launch_narrow_fC(const LaunchPlan &p, hipStream_t st, int stage) {
    if constexpr (kSplit<DD, NN>) k_fC4<NN, S><<<p.grid, Split2<NN>::NT, 0, st>>>(p, stage);
    else k_fC<DD, NN, false, S><<<p.grid, Shape<DimOf<DD>::v, NN, false>::NT, 0, st>>>(p, stage);
}
template <int DD, int NN, bool S>
inline void launch_narrow_fD(const LaunchPlan &p, hipStream_t st, int stage) {
    if constexpr (kSplit<DD, NN>) k_fD4<NN, S><<<p.grid, Split2<NN>::NT, 0, st>>>(p, stage);
    else k_fD<DD, NN, false, S><<<p.grid, Shape<DimOf<DD>::v, NN, false>::NT, 0, st>>>(p, stage);
}

// wide launches of B and D: the four-wave two-node kernels for elements of more than 256
// nodes on meshes of many blocks, the one-lane-per-node kernels otherwise
template <int DD, int NN, bool S>
inline void launch_wide_fB(const LaunchPlan &p, hipStream_t st) {
    if constexpr (kTail<DD, NN>) {
        if (p.nblocks >= kTailMinBlocks) {
            k_fBt<DD, NN, S><<<p.grid, kTailThreads, 0, st>>>(p);
            return;
        }
    }
    k_fB<DD, NN, true, S><<<p.grid, Shape<DimOf<DD>::v, NN, true>::NT, 0, st>>>(p);
}
template <int DD, int NN, bool S>
inline void launch_wide_fD(const LaunchPlan &p, hipStream_t st, int stage) {
    if constexpr (kTail<DD, NN>) {
        if (p.nblocks >= kTailMinBlocks) {
            k_fDt<DD, NN, S><<<p.grid, kTailThreads, 0, st>>>(p, stage);
            return;
        }
    }
    k_fD<DD, NN, true, S><<<p.grid, Shape<DimOf<DD>::v, NN, true>::NT, 0, st>>>(p, stage);
}

template <int DD, int NN, bool S>
inline void launch_wide_lap(const LaunchPlan &p, hipStream_t st) {
    if constexpr (kTail3<DD, NN>) {
        if (p.nblocks >= kTailMinBlocks) {
            k_lapt<DD, NN, S><<<p.grid, kTailThreads, 0, st>>>(p);
            return;
        }
    }
    k_lap<DD, NN, true, S><<<p.grid, Shape<DimOf<DD>::v, NN, true>::NT, 0, st>>>(p);
}
template <int DD, int NN, bool S>
inline void launch_wide_grad(const LaunchPlan &p, hipStream_t st, int collide) {
    if constexpr (kTail3<DD, NN>) {
        if (p.nblocks >= kTailMinBlocks) {
            k_gradt<DD, NN, S><<<p.grid, kTailThreads, 0, st>>>(p, collide);
            return;
        }
    }
    k_grad<DD, NN, true, S><<<p.grid, Shape<DimOf<DD>::v, NN, true>::NT, 0, st>>>(p, collide);
}
template <int DD, int NN, bool S>
inline void launch_wide_stream(const LaunchPlan &p, hipStream_t st, int stage) {
    if constexpr (kTail3<DD, NN>) {
        if (p.nblocks >= kTailMinBlocks) {
            k_streamt<DD, NN, S><<<p.grid, kTailThreads, 0, st>>>(p, stage);
            return;
        }
    }
    k_stream<DD, NN, true, S><<<p.grid, Shape<DimOf<DD>::v, NN, true>::NT, 0, st>>>(p, stage);
}

// ------------------------------------------------------------------------------------------
// launchers of one set of (d, N) instances: SLBM_LAUNCHER_SET(sfx, ORDERS) defines
// launch_<kernel>_<sfx>(d, N, plan, ..., stream) for the orders listed by ORDERS(X)
// ------------------------------------------------------------------------------------------
#define SLBM_ELEM_LAUNCH(KERNEL, DD, NN, W, S, ...)                                          \
    KERNEL<DD, NN, W, S><<<p.grid, Shape<DimOf<DD>::v, NN, W>::NT, 0, st>>>(p, ##__VA_ARGS__)
#define SLBM_ELEM_CASE(KERNEL, DD, NN, ...)                                                  \
    if (!done && d == DD && N == NN) {                                                       \
        const bool wide = p.epb == Shape<DimOf<DD>::v, NN, true>::EPB;                                 \
        if (wide && p.single) SLBM_ELEM_LAUNCH(KERNEL, DD, NN, true, true, ##__VA_ARGS__);   \
        else if (wide) SLBM_ELEM_LAUNCH(KERNEL, DD, NN, true, false, ##__VA_ARGS__);         \
        else if (p.single) SLBM_ELEM_LAUNCH(KERNEL, DD, NN, false, true, ##__VA_ARGS__);     \
        else SLBM_ELEM_LAUNCH(KERNEL, DD, NN, false, false, ##__VA_ARGS__);                  \
        done = true;                                                                         \
    }
#define SLBM_SPLIT_CASE(KERNEL, NARROW, DD, NN, ...)                                        \
    if (!done && d == DD && N == NN) {                                                       \
        const bool wide = p.epb == Shape<DimOf<DD>::v, NN, true>::EPB;                                 \
        if (wide && p.single) SLBM_ELEM_LAUNCH(KERNEL, DD, NN, true, true, ##__VA_ARGS__);   \
        else if (wide) SLBM_ELEM_LAUNCH(KERNEL, DD, NN, true, false, ##__VA_ARGS__);         \
        else if (p.single) NARROW<DD, NN, true>(p, st, ##__VA_ARGS__);                       \
        else NARROW<DD, NN, false>(p, st, ##__VA_ARGS__);                                    \
        done = true;                                                                         \
    }
#define SLBM_SPLIT_WIDE_CASE(WIDEFN, NARROW, DD, NN, ...)                                    \
    if (!done && d == DD && N == NN) {                                                       \
        const bool wide = p.epb == Shape<DimOf<DD>::v, NN, true>::EPB;                                 \
        if (wide && p.single) WIDEFN<DD, NN, true>(p, st, ##__VA_ARGS__);                    \
        else if (wide) WIDEFN<DD, NN, false>(p, st, ##__VA_ARGS__);                          \
        else if (p.single) NARROW<DD, NN, true>(p, st, ##__VA_ARGS__);                       \
        else NARROW<DD, NN, false>(p, st, ##__VA_ARGS__);                                    \
        done = true;                                                                         \
    }
#define SLBM_NODE_CASE(KERNEL, DD, NN, ...)                                                  \
    if (!done && d == DD && N == NN) {                                                       \
        if (p.single) KERNEL<DD, NN, true><<<p.grid, kNodeThreads, 0, st>>>(p, ##__VA_ARGS__); \
        else KERNEL<DD, NN, false><<<p.grid, kNodeThreads, 0, st>>>(p, ##__VA_ARGS__);       \
        done = true;                                                                         \
    }
#define SLBM_ELEM_WIDE_CASE(KERNEL, WIDEFN, DD, NN, ...)                                     \
    if (!done && d == DD && N == NN) {                                                       \
        const bool wide = p.epb == Shape<DimOf<DD>::v, NN, true>::EPB;                                 \
        if (wide && p.single) WIDEFN<DD, NN, true>(p, st, ##__VA_ARGS__);                    \
        else if (wide) WIDEFN<DD, NN, false>(p, st, ##__VA_ARGS__);                          \
        else if (p.single) SLBM_ELEM_LAUNCH(KERNEL, DD, NN, false, true, ##__VA_ARGS__);     \
        else SLBM_ELEM_LAUNCH(KERNEL, DD, NN, false, false, ##__VA_ARGS__);                  \
        done = true;                                                                         \
    }
#define SLBM_CASE_lap(DD, NN) SLBM_ELEM_WIDE_CASE(k_lap, launch_wide_lap, DD, NN)
#define SLBM_CASE_mu(DD, NN) SLBM_NODE_CASE(k_mu, DD, NN)
#define SLBM_CASE_grad(DD, NN) SLBM_ELEM_WIDE_CASE(k_grad, launch_wide_grad, DD, NN, collide)
#define SLBM_CASE_gavg(DD, NN) SLBM_NODE_CASE(k_gavg, DD, NN)
#define SLBM_CASE_collide(DD, NN) SLBM_NODE_CASE(k_collide, DD, NN, use_aux)
#define SLBM_CASE_stream(DD, NN) SLBM_ELEM_WIDE_CASE(k_stream, launch_wide_stream, DD, NN, stage)
#define SLBM_CASE_rk(DD, NN) SLBM_NODE_CASE(k_rk, DD, NN, stage)
#define SLBM_CASE_density(DD, NN) SLBM_NODE_CASE(k_density, DD, NN, which)
#define SLBM_CASE_diag(DD, NN) SLBM_NODE_CASE(k_diag, DD, NN)
#define SLBM_CASE_fA(DD, NN) SLBM_ELEM_CASE(k_fA, DD, NN)
#define SLBM_CASE_fB(DD, NN) SLBM_SPLIT_WIDE_CASE(launch_wide_fB, launch_narrow_fB, DD, NN)
#define SLBM_CASE_fC(DD, NN) SLBM_SPLIT_CASE(k_fC, launch_narrow_fC, DD, NN, stage)
#define SLBM_CASE_fD(DD, NN) SLBM_SPLIT_WIDE_CASE(launch_wide_fD, launch_narrow_fD, DD, NN, stage)

#define SLBM_DISPATCH(ORDERS, KERNEL)                                                        \
    do {                                                                                     \
        if (p.nblocks <= 0 || p.grid <= 0) return 0;                                         \
        hipStream_t st = (hipStream_t)stream;                                                \
        bool done = false;                                                                   \
        ORDERS(SLBM_CASE_##KERNEL)                                                           \
        if (!done) return (int)hipErrorInvalidValue;                                         \
        return (int)hipGetLastError();                                                       \
    } while (0)

#define SLBM_LAUNCHER_SET(SFX, ORDERS)                                                       \
    int launch_lap_##SFX(int d, int N, const LaunchPlan &p, void *stream) { SLBM_DISPATCH(ORDERS, lap); } \
    int launch_mu_##SFX(int d, int N, const LaunchPlan &p, void *stream) { SLBM_DISPATCH(ORDERS, mu); } \
    int launch_grad_##SFX(int d, int N, const LaunchPlan &p, int collide, void *stream) {                \
        SLBM_DISPATCH(ORDERS, grad);                                                         \
    }                                                                                        \
    int launch_gavg_##SFX(int d, int N, const LaunchPlan &p, void *stream) { SLBM_DISPATCH(ORDERS, gavg); } \
    int launch_collide_##SFX(int d, int N, const LaunchPlan &p, int use_aux, void *stream) {             \
        SLBM_DISPATCH(ORDERS, collide);                                                      \
    }                                                                                        \
    int launch_stream_##SFX(int d, int N, const LaunchPlan &p, int stage, void *stream) {                \
        SLBM_DISPATCH(ORDERS, stream);                                                       \
    }                                                                                        \
    int launch_rk_##SFX(int d, int N, const LaunchPlan &p, int stage, void *stream) { SLBM_DISPATCH(ORDERS, rk); } \
    int launch_density_##SFX(int d, int N, const LaunchPlan &p, int which, void *stream) {               \
        SLBM_DISPATCH(ORDERS, density);                                                      \
    }                                                                                        \
    int launch_diag_##SFX(int d, int N, const LaunchPlan &p, void *stream) { SLBM_DISPATCH(ORDERS, diag); } \
    int launch_fA_##SFX(int d, int N, const LaunchPlan &p, void *stream) { SLBM_DISPATCH(ORDERS, fA); } \
    int launch_fB_##SFX(int d, int N, const LaunchPlan &p, void *stream) { SLBM_DISPATCH(ORDERS, fB); } \
    int launch_fC_##SFX(int d, int N, const LaunchPlan &p, int stage, void *stream) { SLBM_DISPATCH(ORDERS, fC); } \
    int launch_fD_##SFX(int d, int N, const LaunchPlan &p, int stage, void *stream) { SLBM_DISPATCH(ORDERS, fD); }

// the instance sets (one translation unit each)
#define SLBM_ORDERS_2A(X) X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(2, 7)
#define SLBM_ORDERS_2B(X) X(2, 8) X(2, 9) X(2, 10) X(2, 11) X(2, 12) X(2, 14) X(2, 16)
#define SLBM_ORDERS_3D(X) X(3, 2) X(3, 3) X(3, 4) X(3, 5) X(3, 6)
#define SLBM_ORDERS_3Q(X) X(13, 2) X(13, 3) X(13, 4) X(13, 5) X(13, 6)

}  // namespace slbm

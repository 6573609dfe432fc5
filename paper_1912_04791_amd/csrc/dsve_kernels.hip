// dsve_kernels.hip -- HIP kernels of the A-DOT hot path for gfx950 (wave64).
//
// k_step      one fused kernel per time step over the flat edge space of all channels:
//             ghost cells (boundary conditions), DOT fluctuation of every edge, exchange of
//             D^- through LDS, cell update into the other ping-pong buffer, CFL speed of the
//             new state reduced per channel (wave shuffles -> LDS -> one global atomic max).
// k_cfl       CFL maximum of a state (start of a run, and the cfl_reduce entry point).
// k_fluct     pairwise fluctuations (dot_edge_fluct entry point).
// k_update    cell update from given fluctuations (cell_update entry point).
//
// Tiling of the step kernel: a workgroup of T threads takes T consecutive edges of the flat
// edge space and updates the T-1 cells whose two faces both lie in the tile; tile k starts at
// edge k (T-1), so consecutive tiles share one edge, which both compute.  Every cell is
// updated by exactly one thread and every value computed depends only on its own edge or
// cell, so results do not depend on T or on the number of workgroups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsve_internal.hpp"
#include "dsve_math.hpp"

namespace dsve {

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = (o > v) ? o : v;
    }
    return v;
}

// Per-channel maximum of `v` (bit patterns of non-negative doubles, so unsigned order is
// value order and a NaN wins) over the active lanes of a wave.  Lanes are grouped by channel;
// a group whose channel is `home` goes to the workgroup accumulator in LDS, any other group
// straight to the global slot of its channel.
__device__ __forceinline__ void reduce_channel_max(unsigned long long v, int chan, bool active,
                                                   int home, unsigned long long *s_acc,
                                                   unsigned long long *gmax)
{
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int cl = __shfl(chan, leader, 64);
        const bool mine = active && (chan == cl);
        const unsigned long long m = wave_max_u64(mine ? v : 0ull);
        if (lane == leader) {
            if (cl == home) atomicMax(s_acc, m);
            else atomicMax(&gmax[cl], m);
        }
        pending &= ~__ballot(mine);
    }
}

__device__ __forceinline__ void raise_flag(unsigned int *flags, bool bad)
{
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 1u);
}

// Edge fluctuation and cell speed for the chosen precision.
template <int G, int PREC>
__device__ __forceinline__ void edge_fluct(double hL, double qL, double zL, double hR, double qR,
                                           double zR, double g, const Closure &K,
                                           const GaussRule &rule, double Dm[3], double Dp[3],
                                           bool &bad)
{
    if constexpr (PREC == PREC_FP64) fluct64<G>(hL, qL, zL, hR, qR, zR, g, K, rule, Dm, Dp, bad);
    else fluct_mixed<G>(hL, qL, zL, hR, qR, zR, g, K, rule, Dm, Dp, bad);
}

template <int PREC>
__device__ __forceinline__ double cell_speed(double h, double q, double g, const Closure &K,
                                             bool &bad)
{
    if constexpr (PREC == PREC_FP64) return speed64(h, q, g, K, bad);
    else return speed_mixed(h, q, g, K, bad);
}

// ---------------------------------------------------------------------------
template <int G, int PREC>
__global__ __launch_bounds__(kMaxTile, PREC == PREC_FP64 ? DSVE_MINW_FP64 : DSVE_MINW_MIXED) void k_step(StepArgs A)
{
    extern __shared__ double s_dm[];          // [3][T]
    __shared__ unsigned long long s_acc;
    const int T = blockDim.x;
    const int t = threadIdx.x;
    unsigned long long reg_acc = 0ull;        // used by thread 0 only
    int reg_chan = -1;

    for (int64_t k = blockIdx.x; k < A.n_tiles; k += gridDim.x) {
        const int home = A.tile_chan[k];
        if (t == 0) s_acc = 0ull;
        const int64_t ge = k * (int64_t)(T - 1) + t;
        const bool have_edge = ge < A.n_edges;
        int c = home;
        if (have_edge)
            while (ge >= A.eoff[c + 1]) ++c;
        const ChanInfo ci = A.ch[c];
        const Closure K = closure_of(ci);
        const int64_t e = ge - A.eoff[c];
        bool bad = false;
        double Dm[3] = {0.0, 0.0, 0.0}, Dp[3] = {0.0, 0.0, 0.0};
        double hR = 0.0, qR = 0.0, zR = 0.0;
        if (have_edge) {
            const int64_t N = ci.ncell, base = ci.cell0;
            const int64_t il = (e == 0) ? (ci.bcl == BC_PERIODIC ? base + N - 1 : base) : base + e - 1;
            const int64_t ir = (e == N) ? (ci.bcr == BC_PERIODIC ? base : base + N - 1) : base + e;
            const double hL = A.h[il];
            double qL = A.q[il];
            const double zL = A.z[il];
            hR = A.h[ir];
            qR = A.q[ir];
            zR = A.z[ir];
            if (e == 0 && ci.bcl == BC_INFLOW_Q) qL = ci.q_in;
            double qRe = qR;
            if (e == N && ci.bcr == BC_INFLOW_Q) qRe = ci.q_in;
            edge_fluct<G, PREC>(hL, qL, zL, hR, qRe, zR, A.g, K, A.rule, Dm, Dp, bad);
        }
        s_dm[t] = Dm[0];
        s_dm[T + t] = Dm[1];
        s_dm[2 * T + t] = Dm[2];
        __syncthreads();
        const bool upd = have_edge && (t < T - 1) && (e < ci.ncell);
        unsigned long long sp_bits = 0ull;
        if (upd) {
            const double amax = __longlong_as_double((long long)A.amax_cur[c]);
            const double dt = ci.cfl_dx * rcp_h(amax);
            const double r = dt * ci.inv_dx;
            const int64_t i = ci.cell0 + e;
            // W_i^{n+1} = W_i^n - dt/dx (D^-_{i+1/2} + D^+_{i-1/2})   (Sec. 3, Eq. scheme)
            const double hn = hR - r * (s_dm[t + 1] + Dp[0]);
            const double qn = qR - r * (s_dm[T + t + 1] + Dp[1]);
            const double zn = zR - r * (s_dm[2 * T + t + 1] + Dp[2]);
            A.hn[i] = hn;
            A.qn[i] = qn;
            A.zn[i] = zn;
            const double sp = fabs(cell_speed<PREC>(hn, qn, A.g, K, bad));
            sp_bits = (unsigned long long)__double_as_longlong(sp);
            if (e == 0) {
                A.t[c] += dt;
                A.amax_clear[c] = 0ull;
            }
        }
        raise_flag(A.flags, bad);
        reduce_channel_max(sp_bits, c, upd, home, &s_acc, A.amax_next);
        __syncthreads();
        if (t == 0) {
            if (home != reg_chan) {
                if (reg_chan >= 0) atomicMax(&A.amax_next[reg_chan], reg_acc);
                reg_chan = home;
                reg_acc = s_acc;
            } else {
                reg_acc = (s_acc > reg_acc) ? s_acc : reg_acc;
            }
        }
    }
    if (t == 0 && reg_chan >= 0) atomicMax(&A.amax_next[reg_chan], reg_acc);
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_channel(const int64_t *off, int C, int64_t i)
{
    int lo = 0, hi = C;   // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Grid-stride over cells; each workgroup keeps its running maximum for one channel at a
// time and flushes it with one global atomic when the channel changes (cells are visited in
// increasing order within a workgroup, so channels change monotonically).
template <int PREC>
__global__ __launch_bounds__(256) void k_cfl(CflArgs A)
{
    __shared__ unsigned long long s_acc;
    unsigned long long reg_acc = 0ull;   // thread 0 only
    int reg_chan = -1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < A.n_cells; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        const bool active = i < A.n_cells;
        const int home = find_channel(A.off, A.n_channels, i0);
        if (threadIdx.x == 0) s_acc = 0ull;
        __syncthreads();
        int c = home;
        unsigned long long bits = 0ull;
        bool bad = false;
        if (active) {
            while (i >= A.off[c + 1]) ++c;
            const double sp = fabs(cell_speed<PREC>(A.h[i], A.q[i], A.g, closure_of(A.ch[c]), bad));
            bits = (unsigned long long)__double_as_longlong(sp);
        }
        raise_flag(A.flags, bad);
        reduce_channel_max(bits, c, active, home, &s_acc, A.amax);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (home != reg_chan) {
                if (reg_chan >= 0) atomicMax(&A.amax[reg_chan], reg_acc);
                reg_chan = home;
                reg_acc = s_acc;
            } else {
                reg_acc = (s_acc > reg_acc) ? s_acc : reg_acc;
            }
        }
    }
    if (threadIdx.x == 0 && reg_chan >= 0) atomicMax(&A.amax[reg_chan], reg_acc);
}

template <int G, int PREC>
__global__ __launch_bounds__(256) void k_fluct(FluctArgs A)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (e < A.n) {
        double Dm[3], Dp[3];
        edge_fluct<G, PREC>(A.hL[e], A.qL[e], A.zL[e], A.hR[e], A.qR[e], A.zR[e], A.g, closure_of(A.ci), A.rule,
                            Dm, Dp, bad);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            A.Dm[r * A.n + e] = Dm[r];
            A.Dp[r * A.n + e] = Dp[r];
        }
    }
    raise_flag(A.flags, bad);
}

__global__ __launch_bounds__(256) void k_update(const double *Dm, const double *Dp, const double *dt,
                                                double dx, int64_t N, double *h, double *q,
                                                double *z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t E = N + 1;
    const double r = dt[0] / dx;
    h[i] = h[i] - r * (Dm[i + 1] + Dp[i]);
    q[i] = q[i] - r * (Dm[E + i + 1] + Dp[E + i]);
    z[i] = z[i] - r * (Dm[2 * E + i + 1] + Dp[2 * E + i]);
}

__global__ void k_dt(const unsigned long long *amax, const ChanInfo *ch, int32_t C, double *dt)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) dt[c] = ch[c].cfl_dx / __longlong_as_double((long long)amax[c]);
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(unsigned int *p, int64_t n, unsigned int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
static inline unsigned int blocks_for(int64_t n, int bs)
{
    return (unsigned int)((n + bs - 1) / bs);
}

// CFL kernel grid: enough workgroups to fill the chip, few enough that the per-workgroup
// global atomics (serialised on one address per channel) stay cheap.
static inline unsigned int cfl_grid(int64_t n_cells)
{
    const unsigned int full = blocks_for(n_cells, 256);
    return full < 2048u ? full : 2048u;
}

template <int PREC>
static hipError_t launch_fluct_prec(const FluctArgs &a, int G, hipStream_t stream)
{
    const dim3 grid(blocks_for(a.n, 256)), block(256);
    switch (G) {
    case 1: hipLaunchKernelGGL((k_fluct<1, PREC>), grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((k_fluct<2, PREC>), grid, block, 0, stream, a); break;
    case 3: hipLaunchKernelGGL((k_fluct<3, PREC>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((k_fluct<4, PREC>), grid, block, 0, stream, a); break;
    case 5: hipLaunchKernelGGL((k_fluct<5, PREC>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_step_prec(const StepArgs &a, int G, int tile, int grid, hipStream_t s)
{
    const size_t lds = sizeof(double) * 3 * (size_t)tile;
    switch (G) {
    case 1: hipLaunchKernelGGL((k_step<1, PREC>), dim3(grid), dim3(tile), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_step<2, PREC>), dim3(grid), dim3(tile), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_step<3, PREC>), dim3(grid), dim3(tile), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_step<4, PREC>), dim3(grid), dim3(tile), lds, s, a); break;
    case 5: hipLaunchKernelGGL((k_step<5, PREC>), dim3(grid), dim3(tile), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PREC>
static int occupancy_prec(int G, int tile)
{
    int n = 0;
    const size_t lds = sizeof(double) * 3 * (size_t)tile;
    hipError_t e = hipErrorInvalidValue;
    switch (G) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<1, PREC>, tile, lds); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<2, PREC>, tile, lds); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<3, PREC>, tile, lds); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<4, PREC>, tile, lds); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<5, PREC>, tile, lds); break;
    default: break;
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

int step_blocks_per_cu(int precision, int G, int tile)
{
    return precision == PREC_MIXED ? occupancy_prec<PREC_MIXED>(G, tile)
                                   : occupancy_prec<PREC_FP64>(G, tile);
}

hipError_t launch_step(const StepArgs &a, int precision, int G, int tile, int grid,
                       hipStream_t stream)
{
    if (tile < 64 || tile > kMaxTile || (tile & 63) || grid < 1) return hipErrorInvalidValue;
    if (precision == PREC_FP64) return launch_step_prec<PREC_FP64>(a, G, tile, grid, stream);
    if (precision == PREC_MIXED) return launch_step_prec<PREC_MIXED>(a, G, tile, grid, stream);
    return hipErrorNotSupported;
}

hipError_t launch_cfl(const CflArgs &a, int precision, hipStream_t stream)
{
    if (a.n_cells < 1) return hipErrorInvalidValue;
    const dim3 grid(cfl_grid(a.n_cells)), block(256);
    if (precision == PREC_FP64) hipLaunchKernelGGL((k_cfl<PREC_FP64>), grid, block, 0, stream, a);
    else if (precision == PREC_MIXED) hipLaunchKernelGGL((k_cfl<PREC_MIXED>), grid, block, 0, stream, a);
    else return hipErrorNotSupported;
    return hipGetLastError();
}

hipError_t launch_fluct(const FluctArgs &a, int precision, int G, hipStream_t stream)
{
    if (a.n < 1) return hipSuccess;
    if (precision == PREC_FP64) return launch_fluct_prec<PREC_FP64>(a, G, stream);
    if (precision == PREC_MIXED) return launch_fluct_prec<PREC_MIXED>(a, G, stream);
    return hipErrorNotSupported;
}

hipError_t launch_cell_update(const double *Dm, const double *Dp, const double *dt, double,
                              double dx, int64_t N, double *h, double *q, double *z,
                              hipStream_t stream)
{
    if (N < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_update, dim3(blocks_for(N, 256)), dim3(256), 0, stream, Dm, Dp, dt, dx, N,
                       h, q, z);
    return hipGetLastError();
}

hipError_t launch_dt(const unsigned long long *amax, const ChanInfo *ch, int32_t C, double *dt,
                     hipStream_t stream)
{
    hipLaunchKernelGGL(k_dt, dim3(blocks_for(C, 256)), dim3(256), 0, stream, amax, ch, C, dt);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int *p, int64_t n, unsigned int v, hipStream_t s)
{
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace dsve

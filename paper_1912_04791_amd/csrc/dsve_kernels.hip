// dsve_kernels.hip -- HIP kernels of the A-DOT hot path for gfx950 (wave64).
//
// k_step      one fused kernel per time step over the flat edge space of all channels:
//             ghost cells (boundary conditions), DOT fluctuation of every edge, exchange of
//             D^- through LDS, cell update into the other ping-pong buffer, CFL speed of the
//             new state reduced per channel (DPP lane moves -> LDS -> one global atomic max
//             per workgroup into its CFL sub-slot).
// k_cfl       CFL maximum of a state (start of a run, and the cfl_reduce entry point).
// k_fluct     pairwise fluctuations (dot_edge_fluct entry point).
// k_update    cell update from given fluctuations (cell_update entry point).
//
// Every kernel comes in one closure form per bed-load law: CL_GRASS (the Grass law in closed
// form, the workloads of Sec. 4) and the other laws through b = xi dq_s/dq per state (Sec. 2,
// Sec. 5), and in three arithmetic forms: FP64 and mixed closed form (Sec. 3.3), and FP64 with
// the numerical eigen-decomposition of the original DOT solver (Sec. 3.1), the baseline of the
// closed form.
//
// Tiling of the step kernel: a workgroup of T threads takes T consecutive edges of the flat
// edge space and updates the T-1 cells whose two faces both lie in the tile; tile k starts at
// edge k (T-1), so consecutive tiles share one edge, which both compute.  Every cell is
// updated by exactly one thread and every value computed depends only on its own edge or
// cell, so results do not depend on T or on the number of workgroups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "dsve_dot.hpp"
#include "dsve_internal.hpp"
#include "dsve_math.hpp"

namespace dsve {

// Maximum over the 64 lanes of a wave of 32-bit values, read back to every lane.  DPP lane
// moves (swaps within quads, half-row and row mirrors: each lane then holds its row of 16; then
// the broadcasts of lane 15 of each row into the next row and of lane 31 into the upper half)
// leave the maximum in lane 63.  A lane whose DPP source lies outside the wave reads 0, the
// identity of the maximum, so every lane is written and no copy of the old value is needed.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_umax32(unsigned v)
{
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
    return o > v ? o : v;
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = dpp_umax32<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_umax32<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_umax32<0x141>(v);   // row_half_mirror
    v = dpp_umax32<0x140>(v);   // row_mirror
    v = dpp_umax32<0x142>(v);   // row_bcast:15
    v = dpp_umax32<0x143>(v);   // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
// Maximum over the wave of 64-bit patterns: the largest high word, then the largest low word among
// the lanes that hold it (one 32-bit maximum per step instead of a 64-bit compare and two selects).
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    const unsigned hi = (unsigned)(v >> 32), lo = (unsigned)v;
    const unsigned mh = wave_max_u32(hi);
    const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
    return ((unsigned long long)mh << 32) | ml;
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

// Atomic maximum of a workgroup's partial result into a per-channel slot, skipped when the slot
// already holds at least the value.  Slot values only grow while a kernel runs, so a load that
// returns an older (smaller) value only costs an atomic that was not needed; the load bypasses
// the compute unit's cache.  Most workgroups do not hold their channel's maximum, so most
// flushes skip the atomic, which would otherwise serialise on the one address at the end of
// the kernel.
__device__ __forceinline__ void flush_max(unsigned long long *slot, unsigned long long v)
{
    const unsigned long long cur = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v > cur) atomicMax(slot, v);
}

// CFL maximum of channel c: the largest of its S sub-slots, as a double.  The floating-point
// maximum drops a NaN sub-slot when another holds a number; a NaN state still shows, since its
// cells stay NaN and the host's check of the last slot orders bit patterns as unsigned
// integers, where NaN is the largest.
__device__ __forceinline__ double amax_of(const unsigned long long *__restrict__ AM, int c,
                                         int64_t stride, int split)
{
    double m = __longlong_as_double((long long)AM[c]);
#pragma unroll
    for (int s = 1; s < kAmaxSplitMax; ++s)
        if (s < split) m = fmax(m, __longlong_as_double((long long)AM[c + s * stride]));
    return m;
}

__device__ __forceinline__ void raise_flag(unsigned int *flags, unsigned bad)
{
    if (bad) atomicOr(&flags[0], bad);
}

// Edge fluctuation and cell speed for the chosen precision and closure form.
template <int G, int PREC, int CL>
__device__ __forceinline__ void edge_fluct(double hL, double qL, double zL, double hR, double qR,
                                           double zR, double g, const Closure &K, double Dm[3],
                                           double Dp[3], unsigned &bad)
{
    if constexpr (PREC == PREC_FP64) fluct64<G, CL>(hL, qL, zL, hR, qR, zR, g, K, Dm, Dp, bad);
    else if constexpr (PREC == PREC_MIXED) fluct_mixed<G, CL>(hL, qL, zL, hR, qR, zR, g, K, Dm, Dp, bad);
    else fluct_dot<G, CL>(hL, qL, zL, hR, qR, zR, g, K, Dm, Dp, bad);
}

template <int PREC, int CL>
__device__ __forceinline__ double cell_speed(double h, double q, double g, const Closure &K,
                                             unsigned &bad)
{
    if constexpr (PREC == PREC_FP64) return speed64<CL>(h, q, g, K, bad);
    else if constexpr (PREC == PREC_MIXED) return speed_mixed<CL>(h, q, g, K, bad);
    else return speed_dot<CL>(h, q, g, K, bad);
}

// Ghost states (boundary conditions): the state beyond edge 0 (left) or edge N (right) of a
// channel from the adjacent cell's and the end's boundary data b = {h, q, z, dz/dt}.
__device__ __forceinline__ double ghost_h(int bc, const double *b, double h)
{
    return (bc == BC_FIXED_DEPTH || bc == BC_INFLOW_QH || bc == BC_DIRICHLET) ? b[0] : h;
}
__device__ __forceinline__ double ghost_q(int bc, const double *b, double q)
{
    return (bc == BC_INFLOW_Q || bc == BC_INFLOW_QH || bc == BC_DIRICHLET) ? b[1] : q;
}
__device__ __forceinline__ double ghost_z(int bc, const double *b, double z, double t)
{
    return bc == BC_DIRICHLET ? fma(t, b[3], b[2]) : z;
}

// Index arithmetic of the step kernel: 32-bit when the context has fewer than 2^29 edges (then
// every byte offset into a state array fits in 32 bits and a load is an SGPR base plus a 32-bit
// VGPR offset), 64-bit otherwise.
template <bool WIDE> struct StepIdx { using type = int32_t; };
template <> struct StepIdx<true> { using type = int64_t; };

template <bool WIDE, typename I>
__device__ __forceinline__ double ldx(const double *__restrict__ p, I i)
{
    if constexpr (WIDE) return p[i];
    else return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(p) + ((uint32_t)i << 3));
}
template <bool WIDE, typename I>
__device__ __forceinline__ void stx(double *__restrict__ p, I i, double v)
{
    if constexpr (WIDE) p[i] = v;
    else *reinterpret_cast<double *>(reinterpret_cast<char *>(p) + ((uint32_t)i << 3)) = v;
}

// ---------------------------------------------------------------------------
template <int G, int PREC, int CL, bool WIDE>
__global__ __launch_bounds__(kMaxTile, step_min_waves(PREC, CL)) void k_step(StepArgs A, const ChanInfo *__restrict__ CH,
                                                                           const int64_t *__restrict__ EO,
                                                                           const int32_t *__restrict__ TC,
                                                                           const unsigned long long *__restrict__ AM)
{
    extern __shared__ double s_dm_all[];      // [2][3][T]: D^- of even and odd tiles
    __shared__ unsigned long long s_acc;
    using Idx = typename StepIdx<WIDE>::type;
    const int T = blockDim.x;
    const int t = threadIdx.x;
    const int lane = t & 63;

    // Each workgroup takes a contiguous run of tiles (the tiles split evenly over the grid: lo or
    // lo + 1 per workgroup, from the host; tile indices fit 32 bits, the host refuses 2^31
    // tiles), so consecutive tiles mostly share their home channel, the channel of the tile's
    // first edge.  The home channel's values (edge offsets, boundary codes, CFL maximum of W^n,
    // time step) are loaded when the run enters the channel, and every lane keeps the running
    // CFL maximum of its cells in it; the lanes are reduced across only when the run leaves the
    // channel, and at the end.  Cells of another channel (a tile that straddles a channel's
    // end) find their channel by a forward scan and go to its slot at once.
    const int wg = (int)blockIdx.x;
    const int k_first = wg * A.tiles_lo + (wg < A.tiles_rem ? wg : A.tiles_rem);
    const int k_end = k_first + A.tiles_lo + (wg < A.tiles_rem ? 1 : 0);
    if (t == 0) s_acc = 0ull;
    if (k_first >= k_end) return;   // the same for the whole workgroup
    // this workgroup's sub-slot of the CFL maxima it merges into (S is a power of two)
    unsigned long long *const amax_mine =
        A.amax_next + (int64_t)(blockIdx.x & (unsigned)(A.amax_split - 1)) * A.amax_stride;
    int home = -1;
    Idx eo0 = 0, eo1 = 0;
    int h_bcl = 0, h_bcr = 0;
    double am_home = 0.0, dt_home = 0.0, r_home = 0.0;
    unsigned long long lane_acc = 0ull;
    int nx_home = TC[k_first];
    for (int k = k_first; k < k_end; ++k) {
        const int tile_home = nx_home;
        if (k + 1 < k_end) nx_home = TC[k + 1];
        if (tile_home != home) {
            if (home >= 0) {
                // merge what the lanes hold for the channel the run leaves (two barriers, once
                // per channel, not per tile)
                const unsigned long long m = wave_max_u64(lane_acc);
                if (lane == 0 && m != 0ull) atomicMax(&s_acc, m);
                __syncthreads();
                if (t == 0) {
                    if (s_acc != 0ull) flush_max(&amax_mine[home], s_acc);
                    s_acc = 0ull;
                }
                __syncthreads();
                lane_acc = 0ull;
            }
            // (a channel's first cell and length follow from its edge offsets: eoff[c] = off[c] + c)
            home = tile_home;
            eo0 = (Idx)EO[home];
            eo1 = (Idx)EO[home + 1];
            h_bcl = CH[home].bcl;
            h_bcr = CH[home].bcr;
            am_home = amax_of(AM, home, A.amax_stride, A.amax_split);
            // dt = CFL dx / amax and dt/dx, as every lane of another channel computes them
            dt_home = CH[home].cfl_dx * rcp_h(am_home);
            r_home = dt_home * CH[home].inv_dx;
        }
        const Idx h_cell0 = eo0 - home, h_ncell = eo1 - eo0 - 1;
        double *const s_dm = s_dm_all + (int)(k & 1) * 3 * T;
        // lanes past the last edge (in the last tile only) compute the last edge again: their
        // results are never stored and no lane that updates a cell reads them
        const Idx ge_raw = (Idx)k * (Idx)(T - 1) + t;
        const bool have_edge = ge_raw < (Idx)A.n_edges;
        const Idx ge = have_edge ? ge_raw : (Idx)A.n_edges - 1;
        int c = home;
        Idx eoc = eo0, cell0 = h_cell0, ncell = h_ncell;
        int bcl = h_bcl, bcr = h_bcr;
        if (ge >= eo1) {
            c = home + 1;
            while (ge >= (Idx)EO[c + 1]) ++c;
            eoc = (Idx)EO[c];
            cell0 = eoc - c;
            ncell = (Idx)EO[c + 1] - eoc - 1;
            bcl = CH[c].bcl;
            bcr = CH[c].bcr;
        }
        // the home channel's record is the same for the whole workgroup (scalar loads); lanes
        // of another channel load their own
        const ChanInfo hci = CH[home];
        ChanInfo ci = hci;
        if (c != home) ci = CH[c];
        const Closure K = closure_of(ci);
        const Idx e = ge - eoc;
        unsigned bad = 0u;
        double Dm[3], Dp[3];
        const Idx N = ncell, base = cell0;
        const Idx il = (e == 0) ? (bcl == BC_PERIODIC ? base + N - 1 : base) : base + e - 1;
        const Idx ir = (e == N) ? (bcr == BC_PERIODIC ? base : base + N - 1) : base + e;
        double hL = ldx<WIDE>(A.h, il);
        double qL = ldx<WIDE>(A.q, il);
        double zL = ldx<WIDE>(A.z, il);
        const double hR = ldx<WIDE>(A.h, ir);
        const double qR = ldx<WIDE>(A.q, ir);
        const double zR = ldx<WIDE>(A.z, ir);
        {
            double hRe = hR, qRe = qR, zRe = zR;
            if (e == 0) {
                hL = ghost_h(ci.bcl, ci.bl, hL);
                qL = ghost_q(ci.bcl, ci.bl, qL);
                if (ci.bcl == BC_DIRICHLET) zL = ghost_z(ci.bcl, ci.bl, zL, A.t_cur[c]);
            } else if (e == N) {
                hRe = ghost_h(ci.bcr, ci.br, hR);
                qRe = ghost_q(ci.bcr, ci.br, qR);
                if (ci.bcr == BC_DIRICHLET) zRe = ghost_z(ci.bcr, ci.br, zR, A.t_cur[c]);
            }
            edge_fluct<G, PREC, CL>(hL, qL, zL, hRe, qRe, zRe, A.g, K, Dm, Dp, bad);
        }
        // D^- goes to the left neighbour through this tile's half of the LDS buffer; the next
        // tile writes the other half, so one barrier per tile orders every write after the
        // reads of the tile before
        s_dm[t] = Dm[0];
        s_dm[T + t] = Dm[1];
        s_dm[2 * T + t] = Dm[2];
        __syncthreads();
        const bool upd = have_edge && (t < T - 1) && (e < ncell);
        unsigned long long sp_bits = 0ull;
        if (upd) {
            double dt = dt_home, r = r_home;
            if (c != home) {
                dt = ci.cfl_dx * rcp_h(amax_of(AM, c, A.amax_stride, A.amax_split));
                r = dt * ci.inv_dx;
            }
            const Idx i = cell0 + e;
            // W_i^{n+1} = W_i^n - dt/dx (D^-_{i+1/2} + D^+_{i-1/2}) + dt S(W_i^n)
            // (Sec. 3, Eq. scheme; S from the friction slope when K_s is given)
            const double hn = hR - r * (s_dm[t + 1] + Dp[0]);
            double qn = qR - r * (s_dm[T + t + 1] + Dp[1]);
            const double zn = zR - r * (s_dm[2 * T + t + 1] + Dp[2]);
            if (ci.fric > 0.0) qn = fma(dt, friction_source(hR, qR, A.g, ci.fric), qn);
            stx<WIDE>(A.hn, i, hn);
            stx<WIDE>(A.qn, i, qn);
            stx<WIDE>(A.zn, i, zn);
            const double sp = fabs(cell_speed<PREC, CL>(hn, qn, A.g, K, bad));
            sp_bits = (unsigned long long)__double_as_longlong(sp);
            if (e == 0) {
                A.t_next[c] = A.t_cur[c] + dt;
                A.amax_clear[c] = 0ull;
#pragma unroll
                for (int s = 1; s < kAmaxSplitMax; ++s)
                    if (s < A.amax_split) A.amax_clear[c + s * A.amax_stride] = 0ull;
            }
        }
        raise_flag(A.flags, bad);
        const bool mine = upd && c == home;
        lane_acc = (mine && sp_bits > lane_acc) ? sp_bits : lane_acc;
        const bool other = upd && c != home;
        if (__ballot(other)) reduce_channel_max(sp_bits, c, other, -1, &s_acc, amax_mine);
    }
    const unsigned long long m = wave_max_u64(lane_acc);
    if (lane == 0 && m != 0ull) atomicMax(&s_acc, m);
    __syncthreads();
    if (t == 0 && s_acc != 0ull) flush_max(&amax_mine[home], s_acc);
}

// ---------------------------------------------------------------------------
// Maximum over the workgroup (uniform result): wave maxima through LDS.  `s_w` holds one entry
// per wave; consecutive calls are separated by at least one other barrier of the caller.
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v, unsigned long long *s_w)
{
    const unsigned long long m = wave_max_u64(v);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    unsigned long long r = 0ull;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) r = (s_w[w] > r) ? s_w[w] : r;
    return r;
}

// Channel-resident run: one workgroup of NT threads takes one channel of N < NT cells (thread i
// holds cell i and computes edge i, between cells i-1 and i) through all n steps of the run,
// with the state in registers, the neighbour states and D^- exchanged through LDS, and the
// channel's CFL maximum reduced within the workgroup; then the next channel.  Every value is
// computed as in k_step (same fluctuation, update and speed, same order of operations), so the
// results are bitwise those of the per-step kernels.
template <int G, int PREC, int CL, int NT>
__global__ __launch_bounds__(NT, step_min_waves(PREC, CL) < 3 ? step_min_waves(PREC, CL) : 3)
void k_resident(ResidentArgs A)
{
    __shared__ double s_st[3][NT];        // h, q, z of the cells
    __shared__ double s_dm[3][NT + 1];    // D^- of the edges
    __shared__ unsigned long long s_w[NT / 64];
    const int t = threadIdx.x;
    unsigned bad = 0u;
    for (int c = blockIdx.x; c < A.n_channels; c += gridDim.x) {
        const ChanInfo ci = A.ch[c];
        const Closure K = closure_of(ci);
        const int64_t cell0 = A.off[c];
        const int N = (int)(A.off[c + 1] - cell0);
        const bool has_cell = t < N, has_edge = t <= N;
        double h = 0.0, q = 0.0, z = 0.0;
        if (has_cell) {
            h = A.h[cell0 + t];
            q = A.q[cell0 + t];
            z = A.z[cell0 + t];
        }
        double tc = A.t[c];
        unsigned long long sp = 0ull;
        if (has_cell) sp = (unsigned long long)__double_as_longlong(fabs(cell_speed<PREC, CL>(h, q, A.g, K, bad)));
        unsigned long long amax_bits = block_max_u64(sp, s_w);
        for (int n = 0; n < A.n_steps; ++n) {
            const double dt = ci.cfl_dx * rcp_h(__longlong_as_double((long long)amax_bits));
            const double r = dt * ci.inv_dx;
            if (has_cell) {
                s_st[0][t] = h;
                s_st[1][t] = q;
                s_st[2][t] = z;
            }
            __syncthreads();
            double Dm[3] = {0.0, 0.0, 0.0}, Dp[3] = {0.0, 0.0, 0.0};
            if (has_edge) {
                const int il = (t == 0) ? (ci.bcl == BC_PERIODIC ? N - 1 : 0) : t - 1;
                const int ir = (t == N) ? (ci.bcr == BC_PERIODIC ? 0 : N - 1) : t;
                double hL = s_st[0][il], qL = s_st[1][il], zL = s_st[2][il];
                double hR = s_st[0][ir], qR = s_st[1][ir], zR = s_st[2][ir];
                if (t == 0) {
                    hL = ghost_h(ci.bcl, ci.bl, hL);
                    qL = ghost_q(ci.bcl, ci.bl, qL);
                    if (ci.bcl == BC_DIRICHLET) zL = ghost_z(ci.bcl, ci.bl, zL, tc);
                } else if (t == N) {
                    hR = ghost_h(ci.bcr, ci.br, hR);
                    qR = ghost_q(ci.bcr, ci.br, qR);
                    if (ci.bcr == BC_DIRICHLET) zR = ghost_z(ci.bcr, ci.br, zR, tc);
                }
                edge_fluct<G, PREC, CL>(hL, qL, zL, hR, qR, zR, A.g, K, Dm, Dp, bad);
                s_dm[0][t] = Dm[0];
                s_dm[1][t] = Dm[1];
                s_dm[2][t] = Dm[2];
            }
            __syncthreads();
            sp = 0ull;
            if (has_cell) {
                // W_i^{n+1} = W_i^n - dt/dx (D^-_{i+1/2} + D^+_{i-1/2}) + dt S(W_i^n) (Sec. 3, Eq. scheme)
                const double hn = h - r * (s_dm[0][t + 1] + Dp[0]);
                double qn = q - r * (s_dm[1][t + 1] + Dp[1]);
                const double zn = z - r * (s_dm[2][t + 1] + Dp[2]);
                if (ci.fric > 0.0) qn = fma(dt, friction_source(h, q, A.g, ci.fric), qn);
                h = hn;
                q = qn;
                z = zn;
                sp = (unsigned long long)__double_as_longlong(fabs(cell_speed<PREC, CL>(h, q, A.g, K, bad)));
            }
            amax_bits = block_max_u64(sp, s_w);
            tc += dt;
        }
        if (has_cell) {
            A.h[cell0 + t] = h;
            A.q[cell0 + t] = q;
            A.z[cell0 + t] = z;
        }
        if (t == 0) {
            A.t[c] = tc;
            A.amax[c] = amax_bits;
        }
        __syncthreads();   // the next channel reuses the LDS
    }
    raise_flag(A.flags, bad);
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
template <int PREC, int CL>
__global__ __launch_bounds__(kCflThreads) void k_cfl(CflArgs A)
{
    // Each workgroup takes a contiguous range of cells, kCflThreads at a time.  Every lane keeps
    // the running maximum of its cells in its wave's current channel `cur` (wave-uniform); the
    // lanes are reduced across only when one of them reaches another channel, and at the end.
    // The workgroup's home channel (that of its first cell) collects in LDS and is merged into
    // its slot once; other channels go to their slots directly.  Workgroups of 1024 threads keep
    // those end-of-kernel merges, which serialise on one address, to a few hundred.
    __shared__ unsigned long long s_acc;
    const int lane = threadIdx.x & 63;
    const int64_t per =
        ((A.n_cells + gridDim.x - 1) / gridDim.x + kCflThreads - 1) / kCflThreads * kCflThreads;
    const int64_t start = (int64_t)blockIdx.x * per;
    const int64_t end = start + per < A.n_cells ? start + per : A.n_cells;
    if (threadIdx.x == 0) s_acc = 0ull;
    __syncthreads();
    if (start >= end) return;   // the same for the whole workgroup
    const int home = find_channel(A.off, A.n_channels, start);
    int c = home;                  // channel of this lane's cell
    int cur = home;                // the wave's current channel
    unsigned long long acc = 0ull; // this lane's maximum over its cells in `cur`
    unsigned bad = 0u;
    // the lane's channel end and closure stay in registers until the lane leaves the channel,
    // so the common iteration waits only for its own cell's state
    int64_t c_end = A.off[c + 1];
    Closure K = closure_of(A.ch[c]);
    for (int64_t i0 = start; i0 < end; i0 += kCflThreads) {
        const int64_t i = i0 + threadIdx.x;
        const bool active = i < end;
        unsigned long long bits = 0ull;
        if (active) {
            if (i >= c_end) {
                do {
                    ++c;
                    c_end = A.off[c + 1];
                } while (i >= c_end);
                K = closure_of(A.ch[c]);
            }
            const double sp = fabs(cell_speed<PREC, CL>(A.h[i], A.q[i], A.g, K, bad));
            bits = (unsigned long long)__double_as_longlong(sp);
        }
        const unsigned long long moved = __ballot(active && c != cur);
        if (moved == 0ull) {
            if (active) acc = bits > acc ? bits : acc;
        } else {
            // the wave leaves `cur`: merge what its lanes hold for it, then this round's cells
            // by channel, and go on in the channel of its last active lane
            const unsigned long long m = wave_max_u64(acc);
            if (lane == 0 && m != 0ull) {
                if (cur == home) atomicMax(&s_acc, m);
                else flush_max(&A.amax[cur], m);
            }
            acc = 0ull;
            reduce_channel_max(bits, c, active, home, &s_acc, A.amax);
            const unsigned long long act = __ballot(active);
            cur = __shfl(c, 63 - __clzll((long long)act), 64);
        }
    }
    const unsigned long long m = wave_max_u64(acc);
    if (lane == 0 && m != 0ull) {
        if (cur == home) atomicMax(&s_acc, m);
        else flush_max(&A.amax[cur], m);
    }
    raise_flag(A.flags, bad);
    __syncthreads();
    if (threadIdx.x == 0 && s_acc != 0ull) flush_max(&A.amax[home], s_acc);
}

template <int G, int PREC, int CL>
__global__ __launch_bounds__(256) void k_fluct(FluctArgs A)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned bad = 0u;
    if (e < A.n) {
        double Dm[3], Dp[3];
        edge_fluct<G, PREC, CL>(A.hL[e], A.qL[e], A.zL[e], A.hR[e], A.qR[e], A.zR[e], A.g, closure_of(A.ci),
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
                                                const ChanInfo *ch, double g, int64_t N, double *h,
                                                double *q, double *z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t E = N + 1;
    const double dti = dt[0];
    const double r = dti * ch->inv_dx;
    const double fric = ch->fric;
    const double h0 = h[i], q0 = q[i];
    double qn = q0 - r * (Dm[E + i + 1] + Dp[E + i]);
    if (fric > 0.0) qn = fma(dti, friction_source(h0, q0, g, fric), qn);
    h[i] = h0 - r * (Dm[i + 1] + Dp[i]);
    q[i] = qn;
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

__global__ void k_copy_u64(unsigned long long *dst, const unsigned long long *src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Static device scratch of the allocation-free run (adot_step_noalloc): the ping-pong copy of
// the state and clocks and the rotating CFL slots of a run of at most kNoAllocCells cells in at
// most kNoAllocChannels channels.  Each device the library runs on holds its own copy until the
// process ends.  Host code never passes this name to a kernel: its device address comes from
// hipGetSymbolAddress, once per device (noalloc_scratch below).
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// ---------------------------------------------------------------------------
static inline unsigned int blocks_for(int64_t n, int bs)
{
    return (unsigned int)((n + bs - 1) / bs);
}

// CFL kernel grid: enough workgroups to fill the chip, few enough that the per-workgroup
// global atomics (serialised on one address per channel) stay cheap.
static inline unsigned int cfl_grid(int64_t n_cells)
{
    const unsigned int full = blocks_for(n_cells, kCflThreads);
    return full < 512u ? full : 512u;
}

// Dispatch over the compile-time variants: G in [1, 5] quadrature points, closure (law).
#define DSVE_DISPATCH_G_CL(G, CL, MACRO)                                                  \
    switch ((G) * 8 + (CL)) {                                                             \
    case 8: MACRO(1, CL_GRASS); break;                                                \
    case 9: MACRO(1, CL_GRASS_THR); break;                                            \
    case 10: MACRO(1, CL_POWER); break;                                               \
    case 11: MACRO(1, CL_MPM); break;                                                 \
    case 12: MACRO(1, CL_VANRIJN); break;                                             \
    case 13: MACRO(1, CL_POWER_INT); break;                                           \
    case 16: MACRO(2, CL_GRASS); break;                                               \
    case 17: MACRO(2, CL_GRASS_THR); break;                                           \
    case 18: MACRO(2, CL_POWER); break;                                               \
    case 19: MACRO(2, CL_MPM); break;                                                 \
    case 20: MACRO(2, CL_VANRIJN); break;                                             \
    case 21: MACRO(2, CL_POWER_INT); break;                                           \
    case 24: MACRO(3, CL_GRASS); break;                                               \
    case 25: MACRO(3, CL_GRASS_THR); break;                                           \
    case 26: MACRO(3, CL_POWER); break;                                               \
    case 27: MACRO(3, CL_MPM); break;                                                 \
    case 28: MACRO(3, CL_VANRIJN); break;                                             \
    case 29: MACRO(3, CL_POWER_INT); break;                                           \
    case 32: MACRO(4, CL_GRASS); break;                                               \
    case 33: MACRO(4, CL_GRASS_THR); break;                                           \
    case 34: MACRO(4, CL_POWER); break;                                               \
    case 35: MACRO(4, CL_MPM); break;                                                 \
    case 36: MACRO(4, CL_VANRIJN); break;                                             \
    case 37: MACRO(4, CL_POWER_INT); break;                                           \
    case 40: MACRO(5, CL_GRASS); break;                                               \
    case 41: MACRO(5, CL_GRASS_THR); break;                                           \
    case 42: MACRO(5, CL_POWER); break;                                               \
    case 43: MACRO(5, CL_MPM); break;                                                 \
    case 44: MACRO(5, CL_VANRIJN); break;                                             \
    case 45: MACRO(5, CL_POWER_INT); break;                                           \
    default: return hipErrorInvalidValue;                                                 \
    }

// Dispatch over the closure alone.
#define DSVE_DISPATCH_CL(CL, MACRO)                                                       \
    switch (CL) {                                                                         \
    case CL_GRASS: MACRO(CL_GRASS); break;                                                \
    case CL_GRASS_THR: MACRO(CL_GRASS_THR); break;                                        \
    case CL_POWER: MACRO(CL_POWER); break;                                                \
    case CL_MPM: MACRO(CL_MPM); break;                                                    \
    case CL_VANRIJN: MACRO(CL_VANRIJN); break;                                            \
    case CL_POWER_INT: MACRO(CL_POWER_INT); break;                                        \
    default: return hipErrorInvalidValue;                                                 \
    }

template <int PREC>
static hipError_t launch_fluct_prec(const FluctArgs &a, int G, int cl, hipStream_t stream)
{
    const dim3 grid(blocks_for(a.n, 256)), block(256);
#define DSVE_LAUNCH_FLUCT(GG, CC) hipLaunchKernelGGL((k_fluct<GG, PREC, CC>), grid, block, 0, stream, a)
    DSVE_DISPATCH_G_CL(G, cl, DSVE_LAUNCH_FLUCT)
#undef DSVE_LAUNCH_FLUCT
    return hipGetLastError();
}

template <int PREC, bool WIDE>
static hipError_t launch_step_prec(const StepArgs &a, int G, int cl, int tile, int grid, hipStream_t s)
{
    const size_t lds = sizeof(double) * 6 * (size_t)tile;
#define DSVE_LAUNCH_STEP(GG, CC) hipLaunchKernelGGL((k_step<GG, PREC, CC, WIDE>), dim3(grid), dim3(tile), lds, s, a, \
                                                   a.ch, a.eoff, a.tile_chan, a.amax_cur)
    DSVE_DISPATCH_G_CL(G, cl, DSVE_LAUNCH_STEP)
#undef DSVE_LAUNCH_STEP
    return hipGetLastError();
}

template <int PREC, bool WIDE>
static hipError_t occupancy_query(int G, int cl, int tile, int &n)
{
    const size_t lds = sizeof(double) * 6 * (size_t)tile;
    hipError_t e = hipErrorInvalidValue;
#define DSVE_OCC(GG, CC) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step<GG, PREC, CC, WIDE>, tile, lds)
    DSVE_DISPATCH_G_CL(G, cl, DSVE_OCC)
#undef DSVE_OCC
    return e;
}

template <bool WIDE>
static hipError_t occupancy_of(int precision, int G, int cl, int tile, int &n)
{
    return precision == PREC_MIXED ? occupancy_query<PREC_MIXED, WIDE>(G, cl, tile, n)
         : precision == PREC_DOT   ? occupancy_query<PREC_DOT, WIDE>(G, cl, tile, n)
                                   : occupancy_query<PREC_FP64, WIDE>(G, cl, tile, n);
}

int step_blocks_per_cu(int precision, int G, int cl, int tile, int64_t n_edges)
{
    int n = 0;
    const hipError_t e = step_needs_wide_index(n_edges) ? occupancy_of<true>(precision, G, cl, tile, n)
                                                       : occupancy_of<false>(precision, G, cl, tile, n);
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <bool WIDE>
static hipError_t launch_step_w(const StepArgs &a, int precision, int G, int cl, int tile, int grid,
                                hipStream_t stream)
{
    if (precision == PREC_FP64) return launch_step_prec<PREC_FP64, WIDE>(a, G, cl, tile, grid, stream);
    if (precision == PREC_MIXED) return launch_step_prec<PREC_MIXED, WIDE>(a, G, cl, tile, grid, stream);
    if (precision == PREC_DOT) return launch_step_prec<PREC_DOT, WIDE>(a, G, cl, tile, grid, stream);
    return hipErrorNotSupported;
}

hipError_t launch_step(const StepArgs &a, int precision, int G, int cl, int tile, int grid,
                       hipStream_t stream)
{
    if (tile < 64 || tile > kMaxTile || (tile & 63) || grid < 1) return hipErrorInvalidValue;
    // workgroup b takes tiles [b lo + min(b, rem), ...), lo + 1 of them for b < rem, else lo
    StepArgs b = a;
    b.tiles_lo = (int32_t)(a.n_tiles / grid);
    b.tiles_rem = (int32_t)(a.n_tiles % grid);
    return step_needs_wide_index(a.n_edges) ? launch_step_w<true>(b, precision, G, cl, tile, grid, stream)
                                            : launch_step_w<false>(b, precision, G, cl, tile, grid, stream);
}

template <int PREC>
static hipError_t launch_cfl_prec(const CflArgs &a, int cl, hipStream_t stream)
{
    const dim3 grid(cfl_grid(a.n_cells)), block(kCflThreads);
#define DSVE_LAUNCH_CFL(CC) hipLaunchKernelGGL((k_cfl<PREC, CC>), grid, block, 0, stream, a)
    DSVE_DISPATCH_CL(cl, DSVE_LAUNCH_CFL)
#undef DSVE_LAUNCH_CFL
    return hipGetLastError();
}

hipError_t launch_cfl(const CflArgs &a, int precision, int cl, hipStream_t stream)
{
    if (a.n_cells < 1) return hipErrorInvalidValue;
    if (precision == PREC_FP64) return launch_cfl_prec<PREC_FP64>(a, cl, stream);
    if (precision == PREC_MIXED) return launch_cfl_prec<PREC_MIXED>(a, cl, stream);
    if (precision == PREC_DOT) return launch_cfl_prec<PREC_DOT>(a, cl, stream);
    return hipErrorNotSupported;
}

hipError_t launch_fluct(const FluctArgs &a, int precision, int G, int cl, hipStream_t stream)
{
    if (a.n < 1) return hipSuccess;
    if (precision == PREC_FP64) return launch_fluct_prec<PREC_FP64>(a, G, cl, stream);
    if (precision == PREC_MIXED) return launch_fluct_prec<PREC_MIXED>(a, G, cl, stream);
    if (precision == PREC_DOT) return launch_fluct_prec<PREC_DOT>(a, G, cl, stream);
    return hipErrorNotSupported;
}

hipError_t launch_cell_update(const double *Dm, const double *Dp, const double *dt,
                              const ChanInfo *ch, double g, int64_t N, double *h, double *q,
                              double *z, hipStream_t stream)
{
    if (N < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_update, dim3(blocks_for(N, 256)), dim3(256), 0, stream, Dm, Dp, dt, ch, g,
                       N, h, q, z);
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

template <int PREC, int NT>
static hipError_t launch_resident_prec(const ResidentArgs &a, int G, int cl, int grid, hipStream_t s)
{
#define DSVE_LAUNCH_RES(GG, CC) hipLaunchKernelGGL((k_resident<GG, PREC, CC, NT>), dim3(grid), dim3(NT), 0, s, a)
    DSVE_DISPATCH_G_CL(G, cl, DSVE_LAUNCH_RES)
#undef DSVE_LAUNCH_RES
    return hipGetLastError();
}

template <int NT>
static hipError_t launch_resident_nt(const ResidentArgs &a, int precision, int G, int cl, int grid,
                                     hipStream_t stream)
{
    if (precision == PREC_FP64) return launch_resident_prec<PREC_FP64, NT>(a, G, cl, grid, stream);
    if (precision == PREC_MIXED) return launch_resident_prec<PREC_MIXED, NT>(a, G, cl, grid, stream);
    if (precision == PREC_DOT) return launch_resident_prec<PREC_DOT, NT>(a, G, cl, grid, stream);
    return hipErrorNotSupported;
}

hipError_t launch_resident(const ResidentArgs &a, int precision, int G, int cl, int threads, int grid,
                           hipStream_t stream)
{
    if (grid < 1 || a.n_channels < 1 || a.n_steps < 1) return hipErrorInvalidValue;
    if (threads == 256) return launch_resident_nt<256>(a, precision, G, cl, grid, stream);
    if (threads == 512) return launch_resident_nt<512>(a, precision, G, cl, grid, stream);
    return hipErrorInvalidValue;
}

int amax_split_of_kernels() { return kAmaxSplitMax; }

hipError_t launch_copy_u64(unsigned long long *dst, const unsigned long long *src, int64_t n,
                           hipStream_t s)
{
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_copy_u64, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per device (the device
// must be current; each device holds its own copy of the array at its own address).
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocMaxDevices];

hipError_t noalloc_scratch(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace dsve

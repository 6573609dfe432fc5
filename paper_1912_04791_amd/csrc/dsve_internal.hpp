// dsve_internal.hpp -- types shared by the HIP kernels and the host side of libdsve.
//
// Layout in HBM (all device memory):
//   state      h[N], q[N], z[N] float64 SoA, channels back to back (caller's arrays
//              plus one ping-pong copy owned by the context)
//   ChanInfo   one 96-byte record per channel (offsets, closure constants, CFL constant,
//              1/dx, boundary conditions)
//   eoff       int64 [C+1]: first edge of each channel in the flat edge space;
//              channel c has N_c + 1 edges, eoff[c] = off[c] + c, eoff[C] = total edges
//   tile_chan  int32 per tile: channel of the tile's first edge
//   amax       uint64 [3][C]: bit patterns of the per-channel CFL maximum, rotated
//              through three slots (read n%3, atomic-max (n+1)%3, clear (n+2)%3)
//   flags      uint32 [4]: [0] non-hyperbolic state seen
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsve {

enum { BC_TRANSMISSIVE = 0, BC_PERIODIC = 1, BC_INFLOW_Q = 2 };
enum { PREC_FP64 = 0, PREC_MIXED = 1 };

constexpr int kMaxGauss = 5;
constexpr int kMaxTile = 256;     // threads (= edges) per workgroup of the step kernel, at most
// Waves per SIMD the step kernel is compiled for (bounds its registers per lane).
#ifndef DSVE_MINW_FP64
#define DSVE_MINW_FP64 3
#endif
#ifndef DSVE_MINW_MIXED
#define DSVE_MINW_MIXED 4
#endif

struct alignas(16) ChanInfo {
    int64_t cell0;   // first cell of the channel in the concatenated state
    int64_t ncell;   // N_c
    double kqg;      // 3 xi A_g g: xi dq_s/dq = kqg Fr^2 for the Grass law
    double K1, K2;   // 1 + 3 kqg, 2 + 9 kqg (k1 = 3 + K1 Fr^2, k2 = Fr (18 - K2 Fr^2))
    double cfl_dx;   // cfl * dx  (dt = cfl_dx / amax)
    double inv_dx;   // 1 / dx
    double q_in;     // inflow discharge for BC_INFLOW_Q
    int32_t bcl, bcr;
    int32_t pad[6];
};
static_assert(sizeof(ChanInfo) == 96, "ChanInfo layout changed");

struct GaussRule {
    double s[kMaxGauss];
    double w[kMaxGauss];
};

struct StepArgs {
    const double *h, *q, *z;     // W^n
    double *hn, *qn, *zn;        // W^{n+1}
    const ChanInfo *ch;
    const int64_t *eoff;         // [C+1]
    const int32_t *tile_chan;    // [n_tiles]
    const unsigned long long *amax_cur;  // [C] CFL max of W^n
    unsigned long long *amax_next;       // [C] CFL max of W^{n+1} (pre-cleared)
    unsigned long long *amax_clear;      // [C] slot to clear for step n+1
    double *t;                   // [C] clocks
    unsigned int *flags;
    int64_t n_edges;
    int64_t n_tiles;
    int32_t n_channels;
    double g;
    GaussRule rule;
};

struct CflArgs {
    const double *h, *q, *z;
    const ChanInfo *ch;
    const int64_t *off;          // [C+1] cell offsets
    unsigned long long *amax;    // [C]
    unsigned int *flags;
    int64_t n_cells;
    int32_t n_channels;
    double g;
};

struct FluctArgs {
    const double *hL, *qL, *zL, *hR, *qR, *zR;
    double *Dm, *Dp;             // [3][n]
    unsigned int *flags;
    int64_t n;
    double g;
    ChanInfo ci;   // closure constants of the context (channel 0)
    GaussRule rule;
};

// Host-side launchers (dsve_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
hipError_t launch_step(const StepArgs &a, int precision, int G, int tile, int grid,
                       hipStream_t stream);
// Workgroups of the step kernel that fit on one compute unit at once (occupancy query).
int step_blocks_per_cu(int precision, int G, int tile);
hipError_t launch_cfl(const CflArgs &a, int precision, hipStream_t stream);
hipError_t launch_fluct(const FluctArgs &a, int precision, int G, hipStream_t stream);
hipError_t launch_cell_update(const double *Dm, const double *Dp, const double *dt,
                              double inv_dx_unused, double dx, int64_t N, double *h, double *q,
                              double *z, hipStream_t stream);
hipError_t launch_dt(const unsigned long long *amax, const ChanInfo *ch, int32_t n_channels,
                     double *dt, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t stream);
hipError_t launch_fill_u32(unsigned int *p, int64_t n, unsigned int v, hipStream_t stream);

}  // namespace dsve

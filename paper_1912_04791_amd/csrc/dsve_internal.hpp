// dsve_internal.hpp -- types shared by the HIP kernels and the host side of libdsve.
//
// Layout in HBM (all device memory):
//   state      h[N], q[N], z[N] float64 SoA, channels back to back (caller's arrays
//              plus one ping-pong copy owned by the context)
//   ChanInfo   one 160-byte record per channel (offsets, closure constants, CFL constant,
//              1/dx, friction, boundary conditions)
//   eoff       int64 [C+1]: first edge of each channel in the flat edge space;
//              channel c has N_c + 1 edges, eoff[c] = off[c] + c, eoff[C] = total edges
//   tile_chan  int32 per tile: channel of the tile's first edge
//   amax       uint64 [3][4][Cs]: bit patterns of the per-channel CFL maximum, rotated
//              through three slots (read n%3, atomic-max (n+1)%3, clear (n+2)%3); each slot
//              holds up to 4 sub-slots per channel, Cs = C rounded up to 512 entries (4 KiB)
//              apart, and the channel's maximum is the maximum over its sub-slots.  With S
//              sub-slots in use a workgroup merges its partial maximum into sub-slot
//              (workgroup index mod S), so the atomics of one step spread over S addresses
//              instead of queueing on one (S = 1, 2 or 4, a launch parameter).
//   clocks     float64 [C] twice (the caller's array and the context's copy): step n reads one
//              and writes t + dt to the other, so every thread sees the step's start time
//   flags      uint32 [4]: [0] deferred error bits (kFlag*) of the states and nodes seen
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsve {

enum { BC_TRANSMISSIVE = 0, BC_PERIODIC = 1, BC_INFLOW_Q = 2, BC_FIXED_DEPTH = 3, BC_INFLOW_QH = 4,
       BC_DIRICHLET = 5 };
// Arithmetic of a kernel: FP64 closed form, mixed FP32/FP64 closed form, or FP64 with the
// numerical eigen-decomposition of the original DOT solver (the baseline of the closed form).
enum { PREC_FP64 = 0, PREC_MIXED = 1, PREC_DOT = 2 };
enum { LAW_GRASS = 0, LAW_GRASS_THR = 1, LAW_POWER = 2, LAW_MPM = 3, LAW_VANRIJN = 4 };
// Kernel variants by closure, one per law: the Grass law in closed non-dimensional form
// (CL_GRASS), and each other law through the per-state coefficient b = xi dq_s/dq.  A context
// has one law, so its kernels are compiled for that law alone.
// CL_POWER_INT is the power law with an integer exponent beta - 1 in [0, 15] in every channel
// (then |u|^(beta - 1) is a short product instead of a general power).
enum { CL_GRASS = LAW_GRASS, CL_GRASS_THR = LAW_GRASS_THR, CL_POWER = LAW_POWER, CL_MPM = LAW_MPM,
       CL_VANRIJN = LAW_VANRIJN, CL_POWER_INT = 5, kNumClosures = 6 };

// Deferred device error bits, or-ed into flags[0] and read back by dsve_sync.
constexpr unsigned kFlagComplex = 1u;    // complex eigenvalues: arccos argument past 1 + tol, or k1 <= 0
constexpr unsigned kFlagCoalesce = 2u;   // a quadrature node whose arccos argument is +-1 to working
                                         // precision: two eigenvalues equal, R^-1 does not exist
constexpr unsigned kFlagNonfinite = 4u;  // a non-finite arccos argument (an overflowed or NaN state)

constexpr int kMaxGauss = 5;
constexpr int kMaxTile = 256;     // threads (= edges) per workgroup of the step kernel, at most
constexpr int kCflThreads = 1024;  // threads per workgroup of the CFL-maximum kernel
// Waves per SIMD the step kernel is compiled for (bounds its registers per lane).
#ifndef DSVE_MINW_FP64
#define DSVE_MINW_FP64 3
#endif
#ifndef DSVE_MINW_MIXED
#define DSVE_MINW_MIXED 4
#endif
// The other closures carry their laws' power and root evaluations: fewer waves, more
// registers per lane.
#ifndef DSVE_MINW_LAW_FP64
#define DSVE_MINW_LAW_FP64 2
#endif
#ifndef DSVE_MINW_LAW_MIXED
#define DSVE_MINW_LAW_MIXED 2
#endif
// The FP64 integer-exponent power law runs the 3 waves its 146 registers allow: capped for 4
// waves it spills 140 bytes and its ensemble steps 26% slower.  MPM and Van Rijn keep the floor
// of 2 and run 3 waves as well (157 registers).
#ifndef DSVE_MINW_POWINT_FP64
#define DSVE_MINW_POWINT_FP64 3
#endif
#ifndef DSVE_MINW_DOT
#define DSVE_MINW_DOT 2
#endif
constexpr int step_min_waves(int prec, int cl)
{
    return prec == PREC_DOT ? DSVE_MINW_DOT
         : cl == CL_GRASS ? (prec == PREC_FP64 ? DSVE_MINW_FP64 : DSVE_MINW_MIXED)
         : (cl == CL_POWER_INT && prec == PREC_FP64) ? DSVE_MINW_POWINT_FP64
                          : (prec == PREC_FP64 ? DSVE_MINW_LAW_FP64 : DSVE_MINW_LAW_MIXED);
}

// Law constants lp0, lp1 (b = xi dq_s/dq at a state with u = q/h, 1/h, |q|):
//   GRASS      lp0 = 3 xi A_g                        b = lp0 u^2 / h
//   GRASS_THR  lp0 = 3 xi A_g, lp1 = u_cr            b = lp0 (|u| - u_cr)^2 / h above u_cr
//   POWER      lp0 = xi A_g beta, lp1 = beta - 1     b = lp0 |u|^lp1 / h  (ipow = lp1 when it
//                                                    is an integer in [0, 15], else -1)
//   MPM        lp0 = 1 / (K_s^2 (S_g-1) d50),        theta = lp0 u^2 / h^(1/3),
//              lp1 = 24 xi sqrt(g (S_g-1) d50^3)     b = lp1 sqrt(theta - 0.047) theta / |q|
//   VANRIJN    lp0 = g / (K_s^2 u_*cr^2),            T + 1 = lp0 u^2 / h^(1/3),
//              lp1 = 4.2 xi 0.053 sqrt(g (S_g-1) d50^3) / D_*^0.3
//                                                    b = lp1 T^1.1 (T + 1) / |q|
struct alignas(16) ChanInfo {
    int64_t cell0;   // first cell of the channel in the concatenated state
    int64_t ncell;   // N_c
    double kqg;      // 3 xi A_g g: xi dq_s/dq = kqg Fr^2 for the Grass law
    double K1, K2h;   // 1 + 3 kqg, 1 + 4.5 kqg (k1 = 3 + K1 Fr^2, k2 / 2 = Fr (9 - K2h Fr^2))
    double cfl_dx;   // cfl * dx  (dt = cfl_dx / amax)
    double inv_dx;   // 1 / dx
    double fric;     // 1 / K_s^2 of the friction slope (0: no friction source)
    double lp0, lp1; // law constants (above)
    // Boundary data of the left / right end {h, q, z, dz/dt}: the ghost takes h from it for
    // FIXED_DEPTH, INFLOW_QH and DIRICHLET, q for INFLOW_Q, INFLOW_QH and DIRICHLET, and
    // z + t dz/dt for DIRICHLET; other components come from the adjacent cell.
    double bl[4], br[4];
    int32_t bcl, bcr;
    int32_t law;
    int32_t ipow;    // power law: integer exponent beta - 1 in [0, 15], else -1
};
static_assert(sizeof(ChanInfo) == 160, "ChanInfo layout changed");

// Gauss-Legendre rules on [0, 1] for G = 1..5 points (Sec. 3.1: the path integral of the
// fluctuations): nodes s = (1 + x)/2 of the Legendre roots x, from their closed forms, and
// weights halved so they sum to one, to 21 significant digits.  Compile-time constants of the
// kernels, which are instantiated per G.
template <int G> struct Gauss;
template <> struct Gauss<1> {
    static constexpr double s[1] = {5.000000000000000000000e-1};
    static constexpr double w[1] = {1.000000000000000000000e+0};
};
template <> struct Gauss<2> {
    static constexpr double s[2] = {2.113248654051871177454e-1, 7.886751345948128822546e-1};
    static constexpr double w[2] = {5.000000000000000000000e-1, 5.000000000000000000000e-1};
};
template <> struct Gauss<3> {
    static constexpr double s[3] = {1.127016653792583114821e-1, 5.000000000000000000000e-1,
                                    8.872983346207416885179e-1};
    static constexpr double w[3] = {2.777777777777777777778e-1, 4.444444444444444444444e-1,
                                    2.777777777777777777778e-1};
};
template <> struct Gauss<4> {
    static constexpr double s[4] = {6.943184420297371238803e-2, 3.300094782075718675987e-1,
                                    6.699905217924281324013e-1, 9.305681557970262876120e-1};
    static constexpr double w[4] = {1.739274225687269286865e-1, 3.260725774312730713135e-1,
                                    3.260725774312730713135e-1, 1.739274225687269286865e-1};
};
template <> struct Gauss<5> {
    static constexpr double s[5] = {4.691007703066800360119e-2, 2.307653449471584544818e-1,
                                    5.000000000000000000000e-1, 7.692346550528415455182e-1,
                                    9.530899229693319963988e-1};
    static constexpr double w[5] = {1.184634425280945437571e-1, 2.393143352496832340206e-1,
                                    2.844444444444444444444e-1, 2.393143352496832340206e-1,
                                    1.184634425280945437571e-1};
};

constexpr int kAmaxSplitMax = 4;   // CFL sub-slots per channel allocated in each slot
inline int64_t amax_stride(int64_t n_channels) { return (n_channels + 511) / 512 * 512; }

struct StepArgs {
    const double *h, *q, *z;     // W^n
    double *hn, *qn, *zn;        // W^{n+1}
    const ChanInfo *ch;
    const int64_t *eoff;         // [C+1]
    const int32_t *tile_chan;    // [n_tiles]
    const unsigned long long *amax_cur;  // [S][Cs] CFL max of W^n
    unsigned long long *amax_next;       // [S][Cs] CFL max of W^{n+1} (pre-cleared)
    unsigned long long *amax_clear;      // [S][Cs] slot to clear for step n+1
    int64_t amax_stride;                 // Cs
    int32_t amax_split;                  // S: sub-slots in use (1, 2 or 4)
    const double *t_cur;         // [C] clocks at the start of the step
    double *t_next;              // [C] clocks after it
    unsigned int *flags;
    int64_t n_edges;
    int64_t n_tiles;
    int32_t tiles_lo, tiles_rem; // n_tiles / grid and n_tiles % grid (set at launch)
    int32_t n_channels;
    double g;
};

// Channel-resident runs: every channel of at most kResidentCells cells is held by one
// workgroup of 256 threads, or 512 when a channel has more than 255 cells (one edge and one
// cell per thread), for all steps of a run, with its state in registers and LDS, so the run
// is one launch.
constexpr int kResidentCells = 511;
constexpr int kResidentSmall = 255;   // channels up to this length use 256-thread workgroups

struct ResidentArgs {
    double *h, *q, *z;           // state, updated in place
    double *t;                   // [C] clocks
    const ChanInfo *ch;
    const int64_t *off;          // [C+1] cell offsets
    unsigned long long *amax;    // [C] CFL maximum of the final state (bit patterns)
    unsigned int *flags;
    int32_t n_channels;
    int32_t n_steps;
    double g;
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
};

// Host-side launchers (dsve_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch; `precision` is one of PREC_*.
hipError_t launch_step(const StepArgs &a, int precision, int G, int cl, int tile, int grid,
                       hipStream_t stream);
// Workgroups of the step kernel that fit on one compute unit at once (occupancy query).
int step_blocks_per_cu(int precision, int G, int cl, int tile, int64_t n_edges);
// The step kernel indexes cells and edges in 32 bits below 2^29 edges (byte offsets into the
// state arrays then fit in 32 bits), in 64 bits from there on.
inline bool step_needs_wide_index(int64_t n_edges) { return n_edges >= (int64_t(1) << 29); }
hipError_t launch_cfl(const CflArgs &a, int precision, int cl, hipStream_t stream);
hipError_t launch_fluct(const FluctArgs &a, int precision, int G, int cl, hipStream_t stream);
// Cell update of one channel from given fluctuations; ch is the channel's record on the device
// (its 1/dx and friction coefficient are used).
hipError_t launch_cell_update(const double *Dm, const double *Dp, const double *dt,
                              const ChanInfo *ch, double g, int64_t N, double *h, double *q,
                              double *z, hipStream_t stream);
hipError_t launch_dt(const unsigned long long *amax, const ChanInfo *ch, int32_t n_channels,
                     double *dt, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t stream);
hipError_t launch_fill_u32(unsigned int *p, int64_t n, unsigned int v, hipStream_t stream);
// All n_steps of a run of channels of at most kResidentCells cells in one launch, with
// workgroups of `threads` (256 or 512) threads, more than the longest channel has cells.
hipError_t launch_resident(const ResidentArgs &a, int precision, int G, int cl, int threads, int grid,
                           hipStream_t stream);
// kAmaxSplitMax as compiled into the kernels (the host code checks it against its own).
int amax_split_of_kernels();
hipError_t launch_copy_u64(unsigned long long *dst, const unsigned long long *src, int64_t n,
                           hipStream_t stream);

// Allocation-free runs (adot_step_noalloc): limits and layout of the static device scratch that
// replaces the context's ping-pong state, clocks and CFL slots.
constexpr int64_t kNoAllocCells = int64_t(1) << 20;
constexpr int64_t kNoAllocChannels = 4096;
constexpr int kNoAllocMaxDevices = 64;
constexpr int64_t kNoAllocSlotEntries = 3 * kAmaxSplitMax * ((kNoAllocChannels + 511) / 512 * 512);
constexpr int64_t kNoAllocOffAmax = 0;                                              // uint64 [3][4][Cs]
constexpr int64_t kNoAllocOffClock = kNoAllocOffAmax + 8 * kNoAllocSlotEntries;     // double [C]
constexpr int64_t kNoAllocOffState = kNoAllocOffClock + 8 * kNoAllocChannels;       // double [3][N]
constexpr int64_t kNoAllocScratchBytes = kNoAllocOffState + 3 * 8 * kNoAllocCells;
static_assert(kNoAllocOffClock % 256 == 0 && kNoAllocOffState % 256 == 0, "scratch alignment");
// Device address of the scratch on `device`, which must be the current device.
hipError_t noalloc_scratch(int device, void **ptr);

}  // namespace dsve

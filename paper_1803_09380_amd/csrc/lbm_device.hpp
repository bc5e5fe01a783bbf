// Device-side descriptors and lattice helpers of the gfx950 IB-LBM library.
//
// Population storage (per simulation): row-blocked.  The lattice rows
// y = -1 .. ny (rows -1 and ny are a ghost layer) are stored one after the
// other, `rstride` elements each.  A row is a sequence of `nblk` blocks of
// kBlk consecutive nodes; a block holds the nine populations of its nodes,
// population i in elements i * kBlk .. i * kBlk + kBlk - 1.  Block 0 is a
// ghost block whose last element is x = -1; block b >= 1 holds
// x = kBlk (b - 1) .. kBlk b - 1, and x = nx (a ghost cell) lies in the last
// block.  One wavefront's access to one population of one block is one
// contiguous 256-byte (FP32) segment, as with separate planes, but the nine
// segments a node's update touches sit together, which keeps the sweep's
// HBM stream as local as a plain copy.  The ghost layer receives populations
// that leave through a non-periodic side and holds the post-stream values
// that the boundary kernel writes for the next sweep to read.
//
// In-place AA access pattern: `swapped` = 0 ("natural") means the post-stream
// population f_i(x) lives in slot i of cell x; `swapped` = 1 means it lives
// in slot opp(i) of cell x - e_i.  A sweep on a natural state reads its own
// cell and writes the post-collision f*_i into slot opp(i) of the same cell
// (result: swapped); a sweep on a swapped state reads slot opp(i) of x - e_i
// and writes f*_i into slot i of x + e_i (result: natural).  Every slot is
// read once and written once per sweep, by the same thread.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmib {

constexpr int Q = 9;
constexpr int kBlk = 64;  // nodes per block of the population layout

// Blocks per stored row for nx nodes (ghost block, data blocks, x = nx inside).
__host__ __device__ constexpr int blocks_per_row(int nx) { return ((nx + kBlk) / kBlk) + 1; }
// Element offset of x within a stored row (population 0); x >= -1.
__host__ __device__ __forceinline__ int col_off(int x) { return ((x + kBlk) / kBlk) * (Q * kBlk) + ((x + kBlk) % kBlk); }

// D2Q9 order fixed by the j_x and j_y rows of the moment matrix (Eq. 5).
__host__ __device__ constexpr int ex_of(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int ey_of(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
// mirror in y (specular reflection on a south/north wall)
__host__ __device__ constexpr int mirror_y(int i) {
    return i == 2 ? 4 : i == 4 ? 2 : i == 5 ? 8 : i == 8 ? 5 : i == 6 ? 7 : i == 7 ? 6 : i;
}
template <typename T>
__host__ __device__ constexpr T weight_of(int i) {
    return i == 0 ? T(4) / T(9) : (i <= 4 ? T(1) / T(9) : T(1) / T(36));
}

enum : int32_t {
    BC_PERIODIC = 0,
    BC_WALL = 1,
    BC_FREESLIP = 2,
    BC_VELOCITY = 3,
    BC_OUTFLOW = 4,
    BC_PRESSURE = 5,
    BC_DIRICHLET = 6
};
enum : int32_t { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
enum : int32_t { BODY_FIXED = 0, BODY_FREE = 1 };

// status bits (sticky, per simulation)
enum : uint32_t { ST_UNSTABLE = 1u, ST_PLAN_OVERFLOW = 2u };

struct BodyDev {
    int32_t kind, n, m0, used;  // marker count, offset into the simulation's marker arrays
    double xc[2], U[2], omega, theta, R, rho_s;
    double Uprev[2], omega_prev;
    double F[2], T, resid, maxslip;  // outputs of the last step
};

struct SimDev {
    void* pop;           // T* base of the stored rows
    int64_t rstride;     // elements per stored row (nblk * 9 * kBlk)
    int32_t nblk;        // blocks per stored row
    int32_t edges;       // bit per side (W, E, S, N) whose wall or free-slip rule the sweep applies
    int32_t nx, ny;
    int32_t bc[4];       // W, E, S, N
    int32_t px, py;      // periodic axes
    double omega;        // 1 / tau
    double rho0;         // reference density
    double rho_base;     // 0 (FP64 stores f) or rho0 (FP32 stores f - w rho0)
    double u_in[2];
    double gravity[2];
    int32_t collision;   // 0 BGK, 1 MRT
    int32_t delta;       // 2, 3 or 4: discrete delta function
    double mrt_s[9];     // MRT relaxation rates in the order of the moment matrix
    const double* ubound;  // DIRICHLET box: (u, v) per perimeter node
    int32_t swapped;     // AA state of the populations (see above)
    int32_t active;      // batch: still stepping
    int64_t steps_left;  // batch: < 0 means unlimited
    int64_t steps_done;
    uint32_t* status;    // sticky status bits
    int32_t nperim;      // boundary nodes the boundary kernel rebuilds each step (inlet and
                         // outlet columns, or the perimeter of a prescribed-velocity box)
    int32_t nbody;
    int32_t ib_iters;    // correction sweeps per step
    int32_t pad_;
    BodyDev* bodies;     // [LBM_MAX_BODIES]
    double *mX, *mY, *mU, *mV, *mds;  // markers of all bodies, FP64
};

// One group of bodies whose delta stencils may share nodes; one workgroup
// corrects a group.  Plan arrays describe the band (the union of the markers'
// 4 x 4 stencils): band nodes in ascending cell order, and for each band node
// the run of stencil entries touching it in ascending marker order.
struct GroupDev {
    int32_t sim;              // index into the simulation table
    int32_t nbody;
    int32_t body[8];          // body slots, ascending
    int32_t M;                // markers in the group
    int32_t dynamic;          // 1: plan rebuilt on the device every step
    int32_t nband, nent;      // static plan sizes
    int32_t cap_nodes, cap_ent;
    int32_t* node_cell;       // [cap_nodes] cell key y * nx + x
    int32_t* node_run;        // [cap_nodes + 1] first entry of each node
    int32_t* ent;             // [cap_ent] (group marker << 4) | (ky << 2) | kx
    int32_t* mnode;           // [M * 16] band node of each stencil slot, -1 if dropped
    int32_t* flags;           // [1] device flag: stencil weights of a static plan are current
    void* node4;              // T [cap_nodes * 4]: rho, 1/rho, j_x, j_y of each band node
                              // (used when the band does not fit in LDS)
    void* ent_D;              // [cap_ent] packed (marker, delta weight D) of every stencil entry:
                              // {int, float} for FP32, {int, int, double} for FP64
    void* m_phi;              // T [M * 8]: phi_x[4], phi_y[4]
    void* m_wtot;             // T [M * 5]: per-sweep ds*dm (first 2M), then ds * (sum dm, sum dPi)
    unsigned short* m_rows;   // [M * 4] first band node of each stencil row, 0xFFFF where the
                              // row's nodes are not 4 consecutive band nodes (fixed plans)
    double* m_red;            // [M * 5] per-marker Fx, Fy, T, |dm|^2, slip for the reductions
    // Colour classes of a fixed plan whose stencil rows are all four consecutive
    // band nodes: no two markers of a class share a band node, so a class
    // spreads into the band without conflicts (ncolor = 0: no such plan).
    int32_t ncolor;
    // 1: the correction workgroup gathers and applies the band itself (plans
    // rebuilt on the device, and fixed plans of at most kFuseBandNodes nodes);
    // 0: the band kernels do, over all CUs
    int32_t in_kernel;
    unsigned short* cord;     // [2 M] group marker at each position (by class, then marker),
                              // then the position of each group marker
    int32_t* coff;            // [ncolor + 1] first position of each class
};

// Work counts of a batch, read by persistent kernels so that a captured graph
// stays valid while the tables change.
// Sweep tiles are stored grouped by XCD: tiles [xcd_start[k], xcd_start[k+1])
// are swept by the blocks with blockIdx.x % 8 == k (workgroups are dealt to
// the eight XCDs round-robin), so x-neighbouring tiles, which share cache lines
// through the shifted accesses of the swapped sweep, meet in one L2.
struct BatchHeader {
    int32_t nsims, ntiles, nbc, ngroups;
    int32_t xcd_start[9];
    int32_t nchunks;  // band chunks (group, first node) of the band kernels
};

// ---------------------------------------------------------------- indexing

__device__ __forceinline__ int wrap(int v, int n, int periodic) {
    if (periodic) {
        if (v < 0) return v + n;
        if (v >= n) return v - n;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T* slot(const SimDev& S, int i, int x, int y) {
    return reinterpret_cast<T*>(S.pop) + (int64_t)(y + 1) * S.rstride + col_off(x) + i * kBlk;
}

// Where the post-stream f_i(x, y) lives for AA state `sw`.
template <typename T>
__device__ __forceinline__ T* loc(const SimDev& S, int i, int x, int y, int sw) {
    if (sw) {
        int sx = wrap(x - ex_of(i), S.nx, S.px), sy = wrap(y - ey_of(i), S.ny, S.py);
        return slot<T>(S, opp_of(i), sx, sy);
    }
    return slot<T>(S, i, x, y);
}

// Where the post-collision f*_i(x, y) of the sweep that produced state `sw` lives.
template <typename T>
__device__ __forceinline__ T* pc(const SimDev& S, int i, int x, int y, int sw) {
    if (sw) return slot<T>(S, opp_of(i), x, y);
    int tx = wrap(x + ex_of(i), S.nx, S.px), ty = wrap(y + ey_of(i), S.ny, S.py);
    return slot<T>(S, i, tx, ty);
}

}  // namespace lbmib

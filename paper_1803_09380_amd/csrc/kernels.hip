// gfx950 kernels of the distribution-function-correction IB-LBM.
//
//   k_sweep        fused collision (BGK or MRT) + streaming, in place (AA
//                  pattern), SoA planes, one workgroup per tile; HBM-bound.
//   k_boundary     rules for populations entering through non-periodic sides.
//   k_band_gather  band records (rho, 1/rho, j) of groups with fixed plans.
//   k_ib           one workgroup per body group: plan and weights of moving
//                  bodies, N Jacobi sweeps of the correction of Sec. 2.3 on the
//                  band's (rho, j), per-marker totals, FP64 force/torque
//                  reductions and the rigid-body update.  Fixed bands are
//                  spread by colour classes of markers that share no band
//                  node; other bands through per-node entry lists.
//   k_band_apply   one final spread of the accumulated deviation into the nine
//                  populations of every band node.
//   k_advance      per-simulation step bookkeeping of batches.
//
// T = double stores f_i; T = float stores h_i = f_i - w_i rho0 (rho_base).
// The equilibrium is written in terms of S = sum_i h_i = rho - rho_base and
// j = sum_i e_i h_i, which covers both: h_i^eq = w_i (S + 3 e.j + 4.5 (e.j)^2/rho
// - 1.5 j.j/rho) (Eq. 3 with c_s^2 = 1/3 and rho u = j).
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace lbmib {

// Tilings 8..15 repeat 0..7 with non-temporal loads and stores (streamed
// data is not kept in the caches); 16..19 are block tiles (tx = 0: ty waves
// of one block each, rpt rounds).  None of them changes the arithmetic.
const Tiling kTilings[kNumTilings] = {
    {64, 4, 1, 0}, {64, 4, 2, 0}, {128, 2, 2, 0}, {256, 1, 2, 0}, {256, 1, 4, 0}, {64, 4, 4, 0},
    {256, 1, 1, 0}, {128, 2, 1, 0}, {64, 4, 1, 1}, {64, 4, 2, 1}, {128, 2, 2, 1}, {256, 1, 2, 1},
    {256, 1, 4, 1}, {64, 4, 4, 1}, {256, 1, 1, 1}, {128, 2, 1, 1}, {0, 4, 1, 1}, {0, 4, 2, 1},
    {0, 8, 1, 1}, {0, 4, 1, 0}};

// Typed accessors: LDS-resident arrays are read with ds_read, device memory
// with global loads and stores (never the flat path of generic pointers, whose
// counters also hold back LDS waits).
#define LBM_AS3 __attribute__((address_space(3)))
#define LBM_AS1 __attribute__((address_space(1)))
template <bool LDS, typename T>
__device__ __forceinline__ T ldm(const T* p) {
    if constexpr (LDS)
        return *(const LBM_AS3 T*)(p);
    else
        return *(const LBM_AS1 T*)(p);
}
template <bool LDS, typename T>
__device__ __forceinline__ void stm(T* p, T v) {
    if constexpr (LDS)
        *(LBM_AS3 T*)(p) = v;
    else
        *(LBM_AS1 T*)(p) = v;
}

// device-memory accesses of the sweep, optionally non-temporal
template <bool NTMP, typename T>
__device__ __forceinline__ T ldg(const LBM_AS1 T* p) {
    if constexpr (NTMP)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NTMP, typename T>
__device__ __forceinline__ void stg(LBM_AS1 T* p, T v) {
    if constexpr (NTMP)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <typename T>
__device__ __forceinline__ LBM_AS1 T* gptr(T* p) {
    return (LBM_AS1 T*)p;
}

// ---------------------------------------------------------------- collision

// The equilibrium (Eq. 3) is evaluated in FP64 whatever the storage
// precision; moments, relaxation and storage stay in T.  In FP32 the rounding
// of the equilibrium is a fixed bias of a steady state, which its slowest
// hydrodynamic mode amplifies by about 1/(nu k^2): it made FP32 and FP64
// Couette fields differ by 1.3e-5 (256^2) and 5.4e-5 (512^2); evaluated in
// FP64 the difference is 3.7e-7 and 1.2e-6, at no measurable cost in time.
template <typename T>
__device__ __forceinline__ void bgk(T h[9], T rho_base, T omega, uint32_t& bad) {
    const T S = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const T jx = (h[1] + h[5] + h[8]) - (h[3] + h[6] + h[7]);
    const T jy = (h[2] + h[5] + h[6]) - (h[4] + h[7] + h[8]);
    const T rho = rho_base + S;
    if (!(rho > T(0)) || !isfinite(jx + jy)) bad = 1u;
    const T inv = T(1) / rho;
    const T ux = jx * inv, uy = jy * inv;
    const double ju = 1.5 * (double(jx) * double(ux) + double(jy) * double(uy));
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double ej = double(ex_of(i)) * double(jx) + double(ey_of(i)) * double(jy);
        const double eu = double(ex_of(i)) * double(ux) + double(ey_of(i)) * double(uy);
        const T heq = T(weight_of<double>(i) * (double(S) + 3.0 * ej + 4.5 * ej * eu - ju));
        h[i] = h[i] + omega * (heq - h[i]);
    }
}

// MRT collision of Eq. 2 with the moment matrix M of Eq. 5 (rows: rho, e,
// epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy) and the diagonal rates of Eq. 6.
// The rows of M are orthogonal, so M^-1 = M^T diag(1/|row|^2).  Shifting f by
// w rho_base moves only the equilibrium of e and epsilon by the same amount as
// the moments themselves, so m - m^eq is formed directly from h.
__host__ __device__ constexpr int mrt_row(int k, int i) {
    // rows of Eq. 5
    return k == 0   ? 1
           : k == 1 ? (i == 0 ? -4 : (i <= 4 ? -1 : 2))
           : k == 2 ? (i == 0 ? 4 : (i <= 4 ? -2 : 1))
           : k == 3 ? ex_of(i)
           : k == 4 ? (i == 0 ? 0 : (i <= 4 ? -2 * ex_of(i) : ex_of(i)))
           : k == 5 ? ey_of(i)
           : k == 6 ? (i == 0 ? 0 : (i <= 4 ? -2 * ey_of(i) : ey_of(i)))
           : k == 7 ? (i == 1 || i == 3 ? 1 : (i == 2 || i == 4 ? -1 : 0))
                    : (i == 5 || i == 7 ? 1 : (i == 6 || i == 8 ? -1 : 0));
}
__host__ __device__ constexpr int mrt_norm2(int k) {
    return k == 0 ? 9 : k == 1 || k == 2 ? 36 : k == 3 || k == 5 ? 6 : k == 4 || k == 6 ? 12 : 4;
}

// As bgk(): each moment of h and its equilibrium (and so m - m^eq) in FP64,
// one moment at a time; the relaxation back to the populations and the
// storage in T.
template <typename T>
__device__ __forceinline__ void mrt(T h[9], T rho_base, const T rate[9], uint32_t& bad) {
    const T S = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const T jx = (h[1] + h[5] + h[8]) - (h[3] + h[6] + h[7]);
    const T jy = (h[2] + h[5] + h[6]) - (h[4] + h[7] + h[8]);
    const double Sd = S, jxd = jx, jyd = jy;
    const double rho = double(rho_base) + Sd;
    if (!(rho > 0.0) || !isfinite(jxd + jyd)) bad = 1u;
    const double inv = 1.0 / rho;
    T d[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (k == 0 || k == 3 || k == 5) {  // conserved moments do not relax
            d[k] = T(0);
            continue;
        }
        double m = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (mrt_row(k, i) != 0) m += double(mrt_row(k, i)) * double(h[i]);
        // equilibrium moments of h (Eq. 3 in moment space)
        const double jj = (jxd * jxd + jyd * jyd) * inv;
        const double meq = k == 1   ? -2.0 * Sd + 3.0 * jj
                           : k == 2 ? Sd - 3.0 * jj
                           : k == 4 ? -jxd
                           : k == 6 ? -jyd
                           : k == 7 ? (jxd * jxd - jyd * jyd) * inv
                                    : jxd * jyd * inv;
        d[k] = T(double(rate[k]) * (m - meq) / double(mrt_norm2(k)));
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        T c = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (mrt_row(k, i) != 0 && k != 0 && k != 3 && k != 5) c += T(mrt_row(k, i)) * d[k];
        h[i] = h[i] - c;
    }
}

// ---------------------------------------------------------------- sweep

// Kernels on a lane's critical path (boundary rules, band gather and apply,
// correction) raise their waves' issue priority above the sweep's: when two
// lanes overlap, their waves share SIMDs with streaming sweep waves that mostly
// wait on memory, and the latency-bound kernels would otherwise queue behind them.
__device__ __forceinline__ void raise_wave_priority() { __builtin_amdgcn_s_setprio(2); }

// Wall (half-way bounce-back, Fig. 2) and free-slip (specular) rules for the
// post-collision populations h that node (x, y) sends out of the lattice,
// written where the next sweep reads the populations they become: the
// reversed one at the same node, or the mirrored one at (x + e_x, y).  No
// other thread reads or writes those slots during the sweep (their source
// lies outside the lattice), so the sweep applies them itself.  A population
// leaving through a west/east side follows that side's rule (corners
// included); the inlet and outlet rules of those sides are left to
// k_boundary.  In AA terms, after a natural sweep (sw = 0) the reversed
// population lives in slot k of the ghost cell x + e_k and the mirrored one in
// slot opp(mirror(k)) of (x, y + e_y); after a swapped sweep, in slot opp(k)
// of the node itself and in slot mirror(k) of (x + e_x, y).  R0, Rs, Rn are
// rows y, y - 1, y + 1 and c0, cl, cr the offsets of x, x - 1, x + 1 (wrapped
// on periodic axes, ghost cells otherwise).
template <typename T, bool NTMP>
__device__ __forceinline__ void edge_rules(const SimDev& S, int x, int y, int sw, const T h[9],
                                           LBM_AS1 T* __restrict__ R0, LBM_AS1 T* __restrict__ Rs,
                                           LBM_AS1 T* __restrict__ Rn, int c0, int cl, int cr) {
    constexpr int B = kBlk;
    const bool wx = !S.px && x == 0, ex = !S.px && x == S.nx - 1;
    const bool sy = !S.py && y == 0, ny = !S.py && y == S.ny - 1;
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const bool outx = (ex_of(k) < 0 && wx) || (ex_of(k) > 0 && ex);
        const bool outy = (ey_of(k) < 0 && sy) || (ey_of(k) > 0 && ny);
        if (!outx && !outy) continue;
        const int side = outx ? S.bc[ex_of(k) < 0 ? SIDE_W : SIDE_E] : S.bc[ey_of(k) < 0 ? SIDE_S : SIDE_N];
        const int cx = ex_of(k) < 0 ? cl : (ex_of(k) > 0 ? cr : c0);
        LBM_AS1 T* __restrict__ Ry = ey_of(k) < 0 ? Rs : (ey_of(k) > 0 ? Rn : R0);
        if (side == BC_WALL) {
            if (!sw)
                stg<NTMP>(&Ry[cx + k * B], h[k]);
            else
                stg<NTMP>(&R0[c0 + opp_of(k) * B], h[k]);
        } else if (side == BC_FREESLIP) {  // south/north only
            if (!sw)
                stg<NTMP>(&Ry[c0 + opp_of(mirror_y(k)) * B], h[k]);
            else
                stg<NTMP>(&R0[cx + mirror_y(k) * B], h[k]);
        }
    }
}

// One node of the sweep: collision and streaming of node (x, y) of a
// simulation whose stored row y = 0 starts at P (rows rs elements apart).
template <typename T, bool NTMP>
__device__ __forceinline__ void sweep_node(const SimDev& S, LBM_AS1 T* __restrict__ P, int64_t rs, int nx, int ny,
                                           int px, int py, int x, int y, int sw, T rho_base, T omega, bool use_mrt,
                                           const T rate[9], uint32_t& bad) {
    constexpr int B = kBlk;
    const int em = S.edges;
    const bool edge = em != 0 && (((em & 1) && x == 0) || ((em & 2) && x == nx - 1) || ((em & 4) && y == 0) ||
                                  ((em & 8) && y == ny - 1));
    const int c0 = col_off(x);
    LBM_AS1 T* __restrict__ R0 = P + (int64_t)y * rs;
    T h[9];
    if (!sw) {
        // natural state: own slots; write f*_i into slot opp(i)
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = ldg<NTMP>(&R0[c0 + i * B]);
        if (use_mrt)
            mrt<T>(h, rho_base, rate, bad);
        else
            bgk<T>(h, rho_base, omega, bad);
#pragma unroll
        for (int i = 0; i < 9; ++i) stg<NTMP>(&R0[c0 + opp_of(i) * B], h[i]);
        if (edge) {
            LBM_AS1 T* __restrict__ Rs = P + (int64_t)wrap(y - 1, ny, py) * rs;
            LBM_AS1 T* __restrict__ Rn = P + (int64_t)wrap(y + 1, ny, py) * rs;
            edge_rules<T, NTMP>(S, x, y, 0, h, R0, Rs, Rn, c0, col_off(wrap(x - 1, nx, px)), col_off(wrap(x + 1, nx, px)));
        }
        return;
    }
    // swapped state: f_i(x) = slot opp(i) of x - e_i; element offsets of
    // x - 1 and x + 1 within a stored row, rows y - 1 and y + 1.  A wave's
    // load shifted by one node in x takes one element from the cache line the
    // neighbouring block's wave also reads, so those six loads stay cached
    // (a non-temporal load lets the line go before the neighbour gets it).
    const int cm = col_off(wrap(x - 1, nx, px)), cp = col_off(wrap(x + 1, nx, px));
    LBM_AS1 T* __restrict__ Rm = P + (int64_t)wrap(y - 1, ny, py) * rs;
    LBM_AS1 T* __restrict__ Rp = P + (int64_t)wrap(y + 1, ny, py) * rs;
    h[0] = ldg<NTMP>(&R0[c0 + 0 * B]);
    h[1] = ldg<false>(&R0[cm + 3 * B]);
    h[2] = ldg<NTMP>(&Rm[c0 + 4 * B]);
    h[3] = ldg<false>(&R0[cp + 1 * B]);
    h[4] = ldg<NTMP>(&Rp[c0 + 2 * B]);
    h[5] = ldg<false>(&Rm[cm + 7 * B]);
    h[6] = ldg<false>(&Rm[cp + 8 * B]);
    h[7] = ldg<false>(&Rp[cp + 5 * B]);
    h[8] = ldg<false>(&Rp[cm + 6 * B]);
    if (use_mrt)
        mrt<T>(h, rho_base, rate, bad);
    else
        bgk<T>(h, rho_base, omega, bad);
    // f*_i goes to slot i of x + e_i
    stg<NTMP>(&R0[c0 + 0 * B], h[0]);
    stg<NTMP>(&R0[cp + 1 * B], h[1]);
    stg<NTMP>(&Rp[c0 + 2 * B], h[2]);
    stg<NTMP>(&R0[cm + 3 * B], h[3]);
    stg<NTMP>(&Rm[c0 + 4 * B], h[4]);
    stg<NTMP>(&Rp[cp + 5 * B], h[5]);
    stg<NTMP>(&Rp[cm + 6 * B], h[6]);
    stg<NTMP>(&Rm[cm + 7 * B], h[7]);
    stg<NTMP>(&Rm[cp + 8 * B], h[8]);
    if (edge) edge_rules<T, NTMP>(S, x, y, 1, h, R0, Rm, Rp, c0, cm, cp);
}

template <typename T, bool MRT>
constexpr int kSweepMinWaves = MRT ? 1 : (sizeof(T) == 4 ? 7 : 6);

// Tile range of workgroup blockIdx.x: with a batch header and a grid that is a
// multiple of 8, the tiles dealt to its XCD; otherwise a grid-stride loop over
// every tile.
__device__ __forceinline__ void tile_range(const BatchHeader* hdr, int ntiles_arg, int& t0, int& t1, int& dt) {
    t0 = blockIdx.x;
    t1 = hdr ? hdr->ntiles : ntiles_arg;
    dt = gridDim.x;
    if (hdr && (gridDim.x & 7) == 0) {
        const int xcd = blockIdx.x & 7;
        t0 = hdr->xcd_start[xcd] + (blockIdx.x >> 3);
        t1 = hdr->xcd_start[xcd + 1];
        dt = gridDim.x >> 3;
    }
}

// At most seven waves per SIMD: the sweep streams at a higher rate than with
// eight (measured), and each SIMD keeps a wave slot for the other kernels.  At
// least seven (FP32) or six (FP64) for BGK only: register budgets of 72 and
// 80, which its code fits without spilling, and more waves in flight hide
// more of the memory latency.
// MRT = false: BGK only (the launch holds no MRT simulation), which leaves out
// the MRT code and its registers; MRT = true: each simulation's own collision.
// Rectangular tiles: TX x TY threads, RPT rows per thread, tile (sim, x0, y0).
template <typename T, int TX, int TY, int RPT, bool NTMP, bool MRT>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(kSweepMinWaves<T, MRT>, 7)))
    k_sweep(const SimDev* __restrict__ sims, const int4* __restrict__ tiles,
            const BatchHeader* __restrict__ hdr, int ntiles_arg, int parity) {
    int t0, t1, dt;
    tile_range(hdr, ntiles_arg, t0, t1, dt);
    for (int t = t0; t < t1; t += dt) {
        const int4 tile = tiles[t];
        const SimDev& S = sims[tile.x];
        if (!S.active) continue;
        const int sw = parity >= 0 ? parity : S.swapped;
        LBM_AS1 T* __restrict__ P = gptr(reinterpret_cast<T*>(S.pop)) + S.rstride;  // stored row of y = 0
        const T rho_base = T(S.rho_base), omega = T(S.omega);
        const bool use_mrt = MRT && S.collision != 0;
        T rate[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) rate[k] = T(S.mrt_s[k]);
        const int x = tile.y + threadIdx.x;
        uint32_t bad = 0;
        if (x < S.nx) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int y = tile.z + threadIdx.y * RPT + r;
                if (y >= S.ny) break;
                sweep_node<T, NTMP>(S, P, S.rstride, S.nx, S.ny, S.px, S.py, x, y, sw, rho_base, omega, use_mrt,
                                    rate, bad);
            }
        }
        if (bad) atomicOr(S.status, ST_UNSTABLE);
    }
}

// Block tiles: every wave takes whole blocks of kBlk nodes of one row; a tile
// (sim, k0) is the W * R consecutive blocks k0 .. k0 + W R - 1 of the
// simulation in row-major order (block k: row k / nbx, nodes
// kBlk (k % nbx) ..), round r giving wave w block k0 + r W + w.  Short rows
// then leave no whole waves idle, and a workgroup's blocks are adjacent in
// memory.
template <typename T, int W, int R, bool NTMP, bool MRT>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kSweepMinWaves<T, MRT>, 7)))
    k_sweep_blk(const SimDev* __restrict__ sims, const int4* __restrict__ tiles,
                const BatchHeader* __restrict__ hdr, int ntiles_arg, int parity) {
    int t0, t1, dt;
    tile_range(hdr, ntiles_arg, t0, t1, dt);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int t = t0; t < t1; t += dt) {
        const int4 tile = tiles[t];
        const SimDev& S = sims[tile.x];
        if (!S.active) continue;
        const int sw = parity >= 0 ? parity : S.swapped;
        LBM_AS1 T* __restrict__ P = gptr(reinterpret_cast<T*>(S.pop)) + S.rstride;
        const T rho_base = T(S.rho_base), omega = T(S.omega);
        const bool use_mrt = MRT && S.collision != 0;
        T rate[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) rate[k] = T(S.mrt_s[k]);
        const int nbx = (S.nx + kBlk - 1) / kBlk, nb = nbx * S.ny;
        uint32_t bad = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = tile.y + r * W + w;
            if (k >= nb) break;
            const int y = k / nbx;
            const int x = (k - y * nbx) * kBlk + lane;
            if (x < S.nx)
                sweep_node<T, NTMP>(S, P, S.rstride, S.nx, S.ny, S.px, S.py, x, y, sw, rho_base, omega, use_mrt,
                                    rate, bad);
        }
        if (bad) atomicOr(S.status, ST_UNSTABLE);
    }
}

// ---------------------------------------------------------------- boundary rules

// Perimeter node k of a prescribed-velocity box: south row, north row, then
// the west and east columns without the corners already counted (the order of
// lbm_set_boundary_velocity).
__device__ __forceinline__ void perim_node(const SimDev& S, int k, int& x, int& y) {
    const int nx = S.nx, ny = S.ny;
    if (k < nx) {
        x = k;
        y = 0;
        return;
    }
    if (k < 2 * nx) {
        x = k - nx;
        y = ny - 1;
        return;
    }
    k -= 2 * nx;
    if (k < ny - 2) {
        x = 0;
        y = 1 + k;
    } else {
        x = nx - 1;
        y = 1 + k - (ny - 2);
    }
}

// Post-stream f_i at an interior-in-x node, applying the south/north rule when
// the source lies outside in y.  Reads post-collision values only.
template <typename T>
__device__ __forceinline__ T post_stream(const SimDev& S, int i, int x, int y, int sw) {
    const int sx = wrap(x - ex_of(i), S.nx, S.px), sy = wrap(y - ey_of(i), S.ny, S.py);
    if (sy >= 0 && sy < S.ny) return ldm<false>(pc<T>(S, i, sx, sy, sw));
    const int side = sy < 0 ? S.bc[SIDE_S] : S.bc[SIDE_N];
    if (side == BC_WALL) return ldm<false>(pc<T>(S, opp_of(i), x, y, sw));
    return ldm<false>(pc<T>(S, mirror_y(i), wrap(x - ex_of(i), S.nx, S.px), y, sw));
}

// h^eq_i for shifted sum S (= rho - rho_base), density rho and momentum j,
// evaluated in FP64 (see bgk()).
template <typename T>
__device__ __forceinline__ T heq_i(int i, T S_, T rho, T jx, T jy) {
    const double jxd = jx, jyd = jy;
    const double ej = double(ex_of(i)) * jxd + double(ey_of(i)) * jyd;
    return T(weight_of<double>(i) *
             (double(S_) + 3.0 * ej + (4.5 * ej * ej - 1.5 * (jxd * jxd + jyd * jyd)) / double(rho)));
}

// Boundary rules of one item (simulation item.x, boundary nodes item.y ..
// item.y + 255), node item.y + t for thread t of the 256 serving the item.
template <typename T>
__device__ __forceinline__ void boundary_item(const SimDev* __restrict__ sims, int2 item, int t, int parity) {
    const SimDev& S = sims[item.x];
    if (!S.active) return;
    const int k = item.y + t;
    if (k >= S.nperim) return;
    const int sw = 1 - (parity >= 0 ? parity : S.swapped);  // state after this step's sweep
    const int nx = S.nx, ny = S.ny;
    int x, y;
    if (S.bc[SIDE_W] == BC_DIRICHLET) {
        perim_node(S, k, x, y);
        // prescribed velocity: non-equilibrium extrapolation from the inward
        // neighbour (diagonal at corners), which is interior on both axes
        const int xn = x < 1 ? 1 : (x > nx - 2 ? nx - 2 : x);
        const int yn = y < 1 ? 1 : (y > ny - 2 ? ny - 2 : y);
        T fn[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) fn[i] = ldm<false>(pc<T>(S, i, xn - ex_of(i), yn - ey_of(i), sw));
        const T Sn = ((fn[0] + fn[1]) + (fn[2] + fn[3])) + ((fn[4] + fn[5]) + (fn[6] + fn[7])) + fn[8];
        const T jxn = (fn[1] + fn[5] + fn[8]) - (fn[3] + fn[6] + fn[7]);
        const T jyn = (fn[2] + fn[5] + fn[6]) - (fn[4] + fn[7] + fn[8]);
        const T rhon = T(S.rho_base) + Sn;
        const T jxb = rhon * T(ldm<false>(S.ubound + 2 * k)), jyb = rhon * T(ldm<false>(S.ubound + 2 * k + 1));
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const T v = heq_i<T>(i, Sn, rhon, jxb, jyb) + (fn[i] - heq_i<T>(i, Sn, rhon, jxn, jyn));
            stm<false>(loc<T>(S, i, x, y, sw), v);
        }
        return;
    }
    // inlet column (west) first, then the outlet column (east)
    const bool inlet = S.bc[SIDE_W] == BC_VELOCITY;
    x = inlet && k < ny ? 0 : nx - 1;
    y = inlet && k >= ny ? k - ny : k;
    if (x == 0) {
        // non-equilibrium extrapolation from column 1 (every population)
        T f1[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f1[i] = post_stream<T>(S, i, 1, y, sw);
        const T S1 = ((f1[0] + f1[1]) + (f1[2] + f1[3])) + ((f1[4] + f1[5]) + (f1[6] + f1[7])) + f1[8];
        const T jx1 = (f1[1] + f1[5] + f1[8]) - (f1[3] + f1[6] + f1[7]);
        const T jy1 = (f1[2] + f1[5] + f1[6]) - (f1[4] + f1[7] + f1[8]);
        const T rho1 = T(S.rho_base) + S1;
        const T jxb = rho1 * T(S.u_in[0]), jyb = rho1 * T(S.u_in[1]);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const T v = heq_i<T>(i, S1, rho1, jxb, jyb) + (f1[i] - heq_i<T>(i, S1, rho1, jx1, jy1));
            stm<false>(loc<T>(S, i, 0, y, sw), v);
        }
        return;
    }
    if (S.bc[SIDE_E] == BC_PRESSURE) {
        // non-equilibrium extrapolation from column nx-2 at density rho0
        T f2[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f2[i] = post_stream<T>(S, i, nx - 2, y, sw);
        const T S2 = ((f2[0] + f2[1]) + (f2[2] + f2[3])) + ((f2[4] + f2[5]) + (f2[6] + f2[7])) + f2[8];
        const T jx2 = (f2[1] + f2[5] + f2[8]) - (f2[3] + f2[6] + f2[7]);
        const T jy2 = (f2[2] + f2[5] + f2[6]) - (f2[4] + f2[7] + f2[8]);
        const T rho2 = T(S.rho_base) + S2;
        const T rhob = T(S.rho0), Sb = T(S.rho0 - S.rho_base);
        const T jxb = rhob * (jx2 / rho2), jyb = rhob * (jy2 / rho2);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const T v = heq_i<T>(i, Sb, rhob, jxb, jyb) + (f2[i] - heq_i<T>(i, S2, rho2, jx2, jy2));
            stm<false>(loc<T>(S, i, nx - 1, y, sw), v);
        }
        return;
    }
    // zero-gradient outlet: the populations entering from the east copy the
    // post-stream values of column nx-2
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (ex_of(i) < 0) stm<false>(loc<T>(S, i, nx - 1, y, sw), post_stream<T>(S, i, nx - 2, y, sw));
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_boundary(const SimDev* __restrict__ sims, const int2* __restrict__ items,
               const BatchHeader* __restrict__ hdr, int nitems_arg, int parity) {
    raise_wave_priority();
    const int nitems = hdr ? hdr->nbc : nitems_arg;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) boundary_item<T>(sims, items[it], threadIdx.x, parity);
}

// ---------------------------------------------------------------- correction sweeps

// One-dimensional discrete delta functions of Eq. 15: (a) two-point hat,
// (b) three-point, (c) four-point cosine.  All three vanish outside the 4 x 4
// stencil floor(X)-1 .. floor(X)+2, so one stencil layout serves every kernel.
template <typename T>
__device__ __forceinline__ T delta_w(int kind, T r) {
    const T a = fabs(r);
    if (kind == 2) return a <= T(1) ? T(1) - a : T(0);
    if (kind == 3) {
        if (a < T(0.5)) return (T(1) + sqrt(T(1) - T(3) * a * a)) / T(3);
        if (a < T(1.5)) return (T(5) - T(3) * a - sqrt(T(1) - T(3) * (T(1) - a) * (T(1) - a))) / T(6);
        return T(0);
    }
    return a <= T(2) ? T(0.25) * (T(1) + cos(T(M_PI) * a * T(0.5))) : T(0);
}

// group marker g -> index into the simulation's marker arrays, and its body slot
__device__ __forceinline__ int marker_index(const SimDev& S, const GroupDev& G, int g, int& body) {
    int base = 0;
    for (int b = 0; b < G.nbody; ++b) {
        const BodyDev& B = S.bodies[G.body[b]];
        if (g < base + B.n) {
            body = G.body[b];
            return B.m0 + (g - base);
        }
        base += B.n;
    }
    body = G.body[0];
    return 0;
}

__device__ __forceinline__ bool stencil_cell(const SimDev& S, double X, double Y, int kx, int ky, int& cell) {
    int x = (int)floor(X) - 1 + kx, y = (int)floor(Y) - 1 + ky;
    x = wrap(x, S.nx, S.px);
    y = wrap(y, S.ny, S.py);
    if (x < 0 || x >= S.nx || y < 0 || y >= S.ny) return false;
    cell = y * S.nx + x;
    return true;
}

// Block-wide exclusive scan of one int per thread (NT threads); returns the
// prefix and the total in *total.  A shuffle scan inside each wave, then the
// wave totals in order; tmp holds NT / 64 + 1 ints.
template <int NT>
__device__ __forceinline__ int block_scan(int v, int* tmp, int* total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int k = 0; k < NT / 64; ++k) {
            const int t = tmp[k];
            tmp[k] = run;
            run += t;
        }
        tmp[NT / 64] = run;
    }
    __syncthreads();
    const int incl = x + tmp[w];
    *total = tmp[NT / 64];
    __syncthreads();
    return incl - v;
}

// Rebuild a group's plan on the device: stencil entries (cell, marker, kx, ky)
// sorted by cell then marker, runs of equal cells are the band nodes.
template <int NT>
__device__ void build_plan(const SimDev& S, const GroupDev& G, unsigned long long* keys, int* scan_tmp,
                           int& nband_out, int& nent_out) {
    const int tid = threadIdx.x;
    const int NE = 16 * G.M;
    int P2 = 16;
    while (P2 < NE) P2 <<= 1;
    for (int e = tid; e < P2; e += NT) {
        unsigned long long key = ~0ull;
        if (e < NE) {
            const int g = e >> 4, s = e & 15, kx = s & 3, ky = s >> 2;
            int body;
            const int mi = marker_index(S, G, g, body);
            int cell;
            if (stencil_cell(S, S.mX[mi], S.mY[mi], kx, ky, cell))
                key = ((unsigned long long)(unsigned)cell << 32) | (unsigned)((g << 4) | (ky << 2) | kx);
        }
        keys[e] = key;
    }
    for (int e = tid; e < NE; e += NT) G.mnode[e] = -1;
    __syncthreads();
    // bitonic sort, ascending
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int e = tid; e < P2; e += NT) {
                const int p = e ^ j;
                if (p > e) {
                    const unsigned long long a = keys[e], b = keys[p];
                    const bool up = (e & k) == 0;
                    if ((a > b) == up) {
                        keys[e] = b;
                        keys[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // run starts -> band node indices (contiguous segment per thread, then scan)
    const int per = (NE + NT - 1) / NT;
    const int e0 = tid * per, e1 = min(NE, e0 + per);
    int cnt = 0, valid = 0;
    for (int e = e0; e < e1; ++e) {
        const unsigned long long key = keys[e];
        if (key == ~0ull) continue;
        ++valid;
        if (e == 0 || (keys[e - 1] >> 32) != (key >> 32)) ++cnt;
    }
    int total;
    int node = block_scan<NT>(cnt, scan_tmp, &total) - 1;
    int nvalid;
    block_scan<NT>(valid, scan_tmp, &nvalid);
    for (int e = e0; e < e1; ++e) {
        const unsigned long long key = keys[e];
        if (key == ~0ull) continue;
        const int cell = (int)(key >> 32);
        if (e == 0 || (keys[e - 1] >> 32) != (key >> 32)) {
            ++node;
            G.node_cell[node] = cell;
            G.node_run[node] = e;
        }
        const int low = (int)(key & 0xffffffffu);
        G.ent[e] = low;
        G.mnode[low] = node;  // low = 16 * marker + stencil slot
    }
    if (tid == 0) G.node_run[total] = nvalid;
    nband_out = total;
    nent_out = nvalid;
    __syncthreads();
}

// Faster rebuild for groups whose stencils fit a small bounding box (the usual
// case for moving particles): count stencil entries per box cell in LDS, scan
// the counts into band-node indices and entry offsets, drop each entry into
// its cell's run, and order every run by marker (insertion sort of a handful of
// entries) so the plan is the same whatever order the atomics came in.  The
// markers' stencil corners, the counts and the entries stay in LDS; the plan is
// written to device memory once.  Returns false, without touching the plan,
// when the box or its LDS arrays are too large.
constexpr int kBinCells = 16384;
// LDS arena of the correction kernel (plan build, then the band's working arrays)
constexpr int kIbArenaBytes = 148 * 1024;
// ... and of the lean correction kernel (dynamic LDS, so that the compiler
// budgets registers for four waves per SIMD)
constexpr int kIbLeanArenaBytes = 96 * 1024;

template <int NT>
__device__ bool build_plan_binned(const SimDev& S, const GroupDev& G, int* lds, int arena_bytes, int* scan_tmp,
                                  int* bbox, int& nband_out, int& nent_out) {
    const int tid = threadIdx.x;
    const int M = G.M, NE = 16 * M;
    if (M == 0 || 2L * M * (int)sizeof(int) > arena_bytes) return false;
    if (tid == 0) {
        bbox[0] = 0x7fffffff;
        bbox[1] = 0x7fffffff;
        bbox[2] = -0x7fffffff;
        bbox[3] = -0x7fffffff;
    }
    __syncthreads();
    // lower-left stencil corner of every marker, kept for the passes below
    int* mfx = lds;
    int* mfy = lds + M;
    int lx = 0x7fffffff, ly = 0x7fffffff, hx = -0x7fffffff, hy = -0x7fffffff;
    for (int g = tid; g < M; g += NT) {
        int body;
        const int mi = marker_index(S, G, g, body);
        const int fx = (int)floor(S.mX[mi]) - 1, fy = (int)floor(S.mY[mi]) - 1;
        mfx[g] = fx;
        mfy[g] = fy;
        lx = min(lx, fx);
        ly = min(ly, fy);
        hx = max(hx, fx + 3);
        hy = max(hy, fy + 3);
    }
    if (lx <= hx) {
        atomicMin(&bbox[0], lx);
        atomicMin(&bbox[1], ly);
        atomicMax(&bbox[2], hx);
        atomicMax(&bbox[3], hy);
    }
    __syncthreads();
    const int x0 = bbox[0], y0 = bbox[1];
    const long W = (long)bbox[2] - x0 + 1, H = (long)bbox[3] - y0 + 1;
    const long words = 2L * M + 2 * W * H + NE;
    if (W * H > kBinCells || words * (long)sizeof(int) > arena_bytes || (S.px && W >= S.nx) || (S.py && H >= S.ny))
        return false;
    const int ncell = (int)(W * H);
    int* count = lds + 2 * M;  // per box cell: entries, then band-node index
    int* start = count + ncell;  // per box cell: first entry, then fill position
    int* ents = start + ncell;   // entries by run
    for (int c = tid; c < ncell; c += NT) count[c] = 0;
    for (int e = tid; e < NE; e += NT) G.mnode[e] = -1;
    __syncthreads();
    for (int e = tid; e < NE; e += NT) {
        const int g = e >> 4, sl = e & 15;
        const int ux = mfx[g] + (sl & 3), uy = mfy[g] + (sl >> 2);
        const int x = wrap(ux, S.nx, S.px), y = wrap(uy, S.ny, S.py);
        if (x < 0 || x >= S.nx || y < 0 || y >= S.ny) continue;
        atomicAdd(&count[(uy - y0) * (int)W + (ux - x0)], 1);
    }
    __syncthreads();
    // scan cells (contiguous segment per thread): entry offsets and band-node indices
    const int per = (ncell + NT - 1) / NT;
    const int c0 = tid * per, c1 = min(ncell, c0 + per);
    int ecnt = 0, ncnt = 0;
    for (int c = c0; c < c1; ++c) {
        ecnt += count[c];
        ncnt += count[c] > 0;
    }
    int etotal, ntotal;
    int ebase = block_scan<NT>(ecnt, scan_tmp, &etotal);
    int nbase = block_scan<NT>(ncnt, scan_tmp, &ntotal);
    for (int c = c0; c < c1; ++c) {
        const int n = count[c];
        start[c] = ebase;
        if (n > 0) {
            const int ux = x0 + c % (int)W, uy = y0 + c / (int)W;
            const int x = wrap(ux, S.nx, S.px), y = wrap(uy, S.ny, S.py);
            G.node_cell[nbase] = y * S.nx + x;
            G.node_run[nbase] = ebase;
            count[c] = nbase;
            ++nbase;
        }
        ebase += n;
    }
    if (tid == 0) G.node_run[ntotal] = etotal;
    __syncthreads();
    for (int e = tid; e < NE; e += NT) {
        const int g = e >> 4, sl = e & 15;
        const int ux = mfx[g] + (sl & 3), uy = mfy[g] + (sl >> 2);
        const int x = wrap(ux, S.nx, S.px), y = wrap(uy, S.ny, S.py);
        if (x < 0 || x >= S.nx || y < 0 || y >= S.ny) continue;
        const int slot = atomicAdd(&start[(uy - y0) * (int)W + (ux - x0)], 1);
        ents[slot] = e;  // e = 16 * marker + (ky << 2 | kx)
    }
    __syncthreads();
    // each non-empty cell's run ends at its fill position and holds count
    // entries no more; order it by marker and write the plan
    for (int c = tid; c < ncell; c += NT) {
        const int e1 = start[c];
        const int e0 = c == 0 ? 0 : start[c - 1];
        if (e1 == e0) continue;
        const int k = count[c];
        for (int a = e0 + 1; a < e1; ++a) {
            const int v = ents[a];
            int b = a - 1;
            while (b >= e0 && ents[b] > v) {
                ents[b + 1] = ents[b];
                --b;
            }
            ents[b + 1] = v;
        }
        for (int e = e0; e < e1; ++e) {
            G.ent[e] = ents[e];
            G.mnode[ents[e]] = k;
        }
    }
    nband_out = ntotal;
    nent_out = etotal;
    __syncthreads();
    return true;
}

// Deterministic FP64 reduction over markers [0, n) of a body: five sums and
// one maximum of per-marker values v[l * 5 + c] (c = 0..3 summed, c = 4 maxed
// with the |dm|^2 slot kept at index 3).  Markers are taken 256 at a time; each
// 64-marker slice is reduced by a fixed xor-shuffle tree, the four slices and
// the chunks are added in order by thread 0.  The order depends only on the
// marker index, never on the workgroup size.
__device__ void body_reduce(int n, const double* v, double* part, double out[5]) {
    const int tid = threadIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < n; c0 += 256) {
        if (tid < 256) {
            const int l = c0 + tid;
            double x[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) x[c] = l < n ? v[l * 5 + c] : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                for (int c = 0; c < 4; ++c) x[c] += __shfl_xor(x[c], off, 64);
                x[4] = fmax(x[4], __shfl_xor(x[4], off, 64));
            }
            if ((tid & 63) == 0)
#pragma unroll
                for (int c = 0; c < 5; ++c) part[(tid >> 6) * 5 + c] = x[c];
        }
        __syncthreads();
        if (tid == 0)
            for (int w = 0; w < 4; ++w) {
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += part[w * 5 + c];
                acc[4] = fmax(acc[4], part[w * 5 + 4]);
            }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = acc[c];  // valid on thread 0
}

// Eq. 39 with the numerator gap read as xi.
__device__ void collision_force(double xi0, double xi1, double xj0, double xj1, double Ri, double Rj,
                                double cij, double gap, double& fx, double& fy) {
    const double dx = xi0 - xj0, dy = xi1 - xj1;
    const double d = sqrt(dx * dx + dy * dy);
    if (d > Ri + Rj + gap || d <= 0.0) return;
    const double g = (d - Ri - Rj - gap) / gap;
    const double mag = cij / 0.01 * g * g;
    fx += mag * dx / d;
    fy += mag * dy / d;
}

// LDS arena of the correction kernel.  In order of use per sweep, the band's
// (rho, j), the per-marker weights, the band's run offsets, the stencil node
// indices (16-bit), the per-marker phi values and the stencil entries are
// placed here while they fit; the rest stay in the group's global scratch
// (generic pointers serve both).  A plan rebuilt on the device first uses the
// arena for its sort keys or bins.

struct Bump {
    char* base;
    int off;
    int cap;  // arena bytes
    __device__ void* take(long bytes) {
        const long a = (bytes + 15) & ~15L;
        if (off + a <= cap) {
            void* p = base + off;
            off += (int)a;
            return p;
        }
        return nullptr;
    }
};

// group marker -> body slot and index into the simulation's marker arrays
struct GroupLookup {
    int nb;
    int body[8];
    int m0[8];
    int gbase[9];
};

__device__ __forceinline__ int lookup(const GroupLookup& L, int g, int& body) {
    int b = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < L.nb && g >= L.gbase[k]) b = k;
    body = L.body[b];
    return L.m0[b] + g - L.gbase[b];
}

// native vectors for 8- and 16-byte LDS/global accesses
template <typename T>
using nv2 = T __attribute__((ext_vector_type(2)));
template <typename T>
using nv4 = T __attribute__((ext_vector_type(4)));

// Where a group's working arrays live for one step.  CORE (band (rho, j),
// per-marker weights, run offsets, 16-bit stencil indices) in LDS or global;
// EXTRA (phi, 16-bit entries, entry weights) in LDS or global.
template <typename T>
struct Band {
    T* node;                 // band records rho, 1/rho, j_x, j_y (rho is fixed during the sweeps)
    T* wt;                   // per-marker weights ds * dm of the current sweep (2 per marker)
    unsigned short* run16;   // band run offsets (LDS) ...
    const int* run32;        // ... or global
    unsigned short* rows;    // per marker: first band node of each stencil row (LDS);
                             // 0xFFFF when the row's nodes are not 4 consecutive band nodes
    const int* mn32;         // per marker: band node of each of the 16 stencil slots (global)
    T* phi;
    unsigned short* ent16;   // packed entries (marker << 4 | ky << 2 | kx) in LDS; D from phi
    const void* entpk;       // ... or packed (marker, D) records in device memory
};

// marker pass: interpolate (rho, j, jj/rho) at marker g from the band,
// deviation dm = rho* U - j*, dPi = rho* U U - Pi*
template <typename T, bool CORE, bool EXTRA>
__device__ __forceinline__ void interp_marker(const Band<T> B, int g, T U, T V, T& dmx, T& dmy, T& dpxx,
                                              T& dpxy, T& dpyy, T& rs) {
    // stencil node indices and weights: vector reads, no branches, so all
    // sixteen band records below are requested at once (a dropped node reads
    // record 0 with weight 0, which adds exact zeros)
    int k[16];
    if constexpr (CORE) {
        const nv2<unsigned> rv = ldm<true>(reinterpret_cast<const nv2<unsigned>*>(B.rows + g * 4));
        const int rs[4] = {(int)(rv.x & 0xffffu), (int)(rv.x >> 16), (int)(rv.y & 0xffffu), (int)(rv.y >> 16)};
#pragma unroll
        for (int ky = 0; ky < 4; ++ky) {
            if (rs[ky] != 0xFFFF) {
#pragma unroll
                for (int kx = 0; kx < 4; ++kx) k[ky * 4 + kx] = rs[ky] + kx;
            } else {  // a row cut by a lattice edge or wrapped across a periodic one
#pragma unroll
                for (int kx = 0; kx < 4; ++kx) k[ky * 4 + kx] = ldm<false>(B.mn32 + g * 16 + ky * 4 + kx);
            }
        }
    } else {
        const nv4<int>* m = reinterpret_cast<const nv4<int>*>(B.mn32 + g * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const nv4<int> v = ldm<false>(m + q);
            k[4 * q] = v.x;
            k[4 * q + 1] = v.y;
            k[4 * q + 2] = v.z;
            k[4 * q + 3] = v.w;
        }
    }
    T px[4], py[4];
    {
        const nv4<T>* ph = reinterpret_cast<const nv4<T>*>(B.phi + g * 8);
        const nv4<T> a = ldm<EXTRA>(ph), c = ldm<EXTRA>(ph + 1);
        px[0] = a.x;
        px[1] = a.y;
        px[2] = a.z;
        px[3] = a.w;
        py[0] = c.x;
        py[1] = c.y;
        py[2] = c.z;
        py[3] = c.w;
    }
    const nv4<T>* node = reinterpret_cast<const nv4<T>*>(B.node);
    T r = 0, jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0;
    // two stencil rows at a time: eight band records requested together
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        nv4<T> nd[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kk = k[half * 8 + q];
            nd[q] = ldm<CORE>(node + (kk < 0 ? 0 : kk));
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kx = q & 3, ky = half * 2 + (q >> 2);
            const T D = k[half * 8 + q] < 0 ? T(0) : px[kx] * py[ky];
            const T nr = nd[q].x, inv = nd[q].y, nx = nd[q].z, ny = nd[q].w;
            r += D * nr;
            jx += D * nx;
            jy += D * ny;
            pxx += D * nx * nx * inv;
            pxy += D * nx * ny * inv;
            pyy += D * ny * ny * inv;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    dmx = r * U - jx;
    dmy = r * V - jy;
    dpxx = r * U * U - pxx;
    dpxy = r * U * V - pxy;
    dpyy = r * V * V - pyy;
    rs = r;
}

// Packed stencil entry in device memory: marker index g and weight D, one
// 8-byte (FP32) or 16-byte (FP64) load per entry.
template <typename T>
__device__ __forceinline__ void store_entry(void* base, int e, int g, T d) {
    if constexpr (sizeof(T) == 4) {
        nv2<unsigned> v;
        v.x = (unsigned)g;
        v.y = __builtin_bit_cast(unsigned, d);
        stm<false>(reinterpret_cast<nv2<unsigned>*>(base) + e, v);
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, d);
        nv4<unsigned> v;
        v.x = (unsigned)g;
        v.y = 0u;
        v.z = (unsigned)(b & 0xffffffffull);
        v.w = (unsigned)(b >> 32);
        stm<false>(reinterpret_cast<nv4<unsigned>*>(base) + e, v);
    }
}
template <typename T>
__device__ __forceinline__ void load_entry(const void* base, int e, int& g, T& d) {
    if constexpr (sizeof(T) == 4) {
        const nv2<unsigned> v = ldm<false>(reinterpret_cast<const nv2<unsigned>*>(base) + e);
        // through plain scalars: a bit cast applied to a vector element
        // expression reinterprets the wrong element
        const unsigned gx = v.x, dy = v.y;
        g = (int)gx;
        d = __builtin_bit_cast(T, dy);
    } else {
        const nv4<unsigned> v = ldm<false>(reinterpret_cast<const nv4<unsigned>*>(base) + e);
        const unsigned gx = v.x, lo = v.z, hi = v.w;
        g = (int)gx;
        d = __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}

// node pass: sum over the node's stencil entries (ascending marker) of
// D * w[stride * g + c] for C components
template <typename T, bool CORE, bool EXTRA, int C>
__device__ __forceinline__ void spread_node(const Band<T> B, const T* w, int stride, int e0, int e1, T out[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = T(0);
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        int g[4];
        T d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (EXTRA) {
                const int p = ldm<true>(B.ent16 + e + q);
                g[q] = p >> 4;
                d[q] = ldm<true>(B.phi + g[q] * 8 + (p & 3)) * ldm<true>(B.phi + g[q] * 8 + 4 + ((p >> 2) & 3));
            } else {
                load_entry<T>(B.entpk, e + q, g[q], d[q]);
            }
        }
        T wv[4][C];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < C; ++c) wv[q][c] = ldm<CORE>(w + stride * g[q] + c);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < C; ++c) out[c] += d[q] * wv[q][c];
    }
    for (; e < e1; ++e) {
        int g;
        T d;
        if constexpr (EXTRA) {
            const int p = ldm<true>(B.ent16 + e);
            g = p >> 4;
            d = ldm<true>(B.phi + g * 8 + (p & 3)) * ldm<true>(B.phi + g * 8 + 4 + ((p >> 2) & 3));
        } else {
            load_entry<T>(B.entpk, e, g, d);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) out[c] += d * ldm<CORE>(w + stride * g + c);
    }
}

#ifdef LBMIB_TRACE_IB
// phase timestamps (100 MHz wall clock) of the first group, for profiling builds only
__device__ long long lbmib_ib_trace[64];
}  // namespace lbmib
extern "C" int lbm_debug_ib_trace(long long* out) {
    return hipMemcpyFromSymbol(out, HIP_SYMBOL(lbmib::lbmib_ib_trace), sizeof(long long) * 64) == hipSuccess ? 0 : 3;
}
namespace lbmib {
#define IB_MARK(k)                                  \
    do {                                            \
        if (gi == 0 && tid == 0) {                  \
            lbmib_ib_trace[(k)] = wall_clock64();   \
            lbmib_ib_trace[32 + (k)] = clock64();   \
        }                                           \
    } while (0)
#else
#define IB_MARK(k) \
    do {           \
    } while (0)
#endif

template <typename T, bool CORE>
__device__ __forceinline__ int run_at(const Band<T>& B, int k) {
    if constexpr (CORE)
        return ldm<true>(B.run16 + k);
    else
        return ldm<false>(B.run32 + k);
}

// The four stencil rows of marker i as band node indices: the first node of
// each row, or 0xFFFF where the row's nodes are not 4 consecutive band nodes
// (cut by a lattice edge or wrapped across a periodic one).
__device__ __forceinline__ nv2<unsigned> stencil_rows(const GroupDev& G, int i) {
    int m[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) m[q] = ldm<false>(G.mnode + i * 16 + q);
    unsigned short r[4];
#pragma unroll
    for (int ky = 0; ky < 4; ++ky) {
        const int a = m[ky * 4];
        const bool reg = a >= 0 && a < 0xFFFF && m[ky * 4 + 1] == a + 1 && m[ky * 4 + 2] == a + 2 && m[ky * 4 + 3] == a + 3;
        r[ky] = reg ? (unsigned short)a : (unsigned short)0xFFFF;
    }
    nv2<unsigned> rv;
    rv.x = (unsigned)r[0] | ((unsigned)r[1] << 16);
    rv.y = (unsigned)r[2] | ((unsigned)r[3] << 16);
    return rv;
}

// Band record of one node: rho, 1/rho, j_x, j_y of its post-stream populations.
template <typename T>
__device__ __forceinline__ nv4<T> band_record(const T f[9], T rho_base) {
    const T Ssum = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const T rho = rho_base + Ssum;
    nv4<T> rec;
    rec.x = rho;
    rec.y = T(1) / rho;
    rec.z = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
    rec.w = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
    return rec;
}

// Outputs of marker g after the sweeps: force and torque of its accumulated
// deviation, the mismatch left (dmx, dmy) and the slip relative to the
// interpolated density rs, for the FP64 reductions; and the totals of the
// sweeps (ds times the sums of dm and dPi) for the final spread (k_band_apply).
template <typename T>
__device__ __forceinline__ void marker_outputs(const SimDev& S, const GroupDev& G, const GroupLookup& L, int g,
                                               const T acc[5], T dmx, T dmy, T rs) {
    int body;
    const int mi = lookup(L, g, body);
    const double ds = ldm<false>(S.mds + mi);
    const BodyDev& Bd = S.bodies[body];
    const double Fx = -ds * (double)acc[0], Fy = -ds * (double)acc[1];
    const double r2 = (double)dmx * (double)dmx + (double)dmy * (double)dmy;
    double* mr = G.m_red + g * 5;
    mr[0] = Fx;
    mr[1] = Fy;
    mr[2] = (S.mX[mi] - Bd.xc[0]) * Fy - (S.mY[mi] - Bd.xc[1]) * Fx;
    mr[3] = r2;
    mr[4] = sqrt(r2) / (double)rs;
#pragma unroll
    for (int c = 0; c < 5; ++c) stm<false>(reinterpret_cast<T*>(G.m_wtot) + g * 5 + c, T(ds * (double)acc[c]));
}

// Eq. 28 on the nine populations f of one node, given the spread totals t
// (ds-weighted sums of dm_x, dm_y, dPi_xx, dPi_xy, dPi_yy): f_i += delta f_i.
// No multiply-add is fused here, so every caller (band kernel, correction
// workgroup, whatever the code around it) rounds the same way.
template <typename T>
__device__ __forceinline__ void correct_pops(const T t[5], T f[9]) {
#pragma clang fp contract(off)
    const T trB = T(1.5) * (t[2] + t[4]);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T ex = T(ex_of(i)), ey = T(ey_of(i));
        const T d = weight_of<T>(i) *
                    (T(3) * (ex * t[0] + ey * t[1]) + T(4.5) * (ex * ex * t[2] + T(2) * ex * ey * t[3] + ey * ey * t[4]) - trB);
        f[i] = f[i] + d;
    }
}

// Eq. 28 at node (x, y), in place.
template <typename T>
__device__ __forceinline__ void correct_node(const SimDev& S, int x, int y, int sw, const T t[5]) {
    T f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = ldm<false>(loc<T>(S, i, x, y, sw));
    correct_pops<T>(t, f);
#pragma unroll
    for (int i = 0; i < 9; ++i) stm<false>(loc<T>(S, i, x, y, sw), f[i]);
}

// Steps 2-5 of a group's correction (gather, N sweeps on (rho, j), per-marker
// totals of the sweeps) for one placement of its working arrays.  Groups with
// fixed plans have their band records gathered beforehand (gather_band in the
// same workgroup, or k_band_gather for large bands); the final spread and
// correction of the populations follow (apply_band, or k_band_apply).
template <typename T, int NT, int MPT, bool CORE, bool EXTRA>
__device__ __forceinline__ void correct_group(const SimDev& S, const GroupDev& G, const GroupLookup& L, Band<T> B,
                                              const T* phi_g, int M, int nband, int nent, int sw,
                                              int gi) {
    const int tid = threadIdx.x;
    if constexpr (CORE) {
        // one pass issues every copy's loads together
        const int len = max(max(nband + 1, M), EXTRA ? max(8 * M, nent) : 0);
        for (int i = tid; i < len; i += NT) {
            if (i <= nband) stm<true>(B.run16 + i, (unsigned short)ldm<false>(G.node_run + i));
            if (i < M) {
                const nv2<unsigned> rv = G.dynamic ? stencil_rows(G, i)
                                                   : ldm<false>(reinterpret_cast<const nv2<unsigned>*>(G.m_rows) + i);
                stm<true>(reinterpret_cast<nv2<unsigned>*>(B.rows + i * 4), rv);
            }
            if constexpr (EXTRA) {
                if (i < 8 * M) stm<true>(B.phi + i, ldm<false>(phi_g + i));
                if (i < nent) stm<true>(B.ent16 + i, (unsigned short)ldm<false>(G.ent + i));
            }
        }
        if (!G.dynamic) {  // band records gathered by gather_band or k_band_gather; four in flight
            const nv4<T>* src = reinterpret_cast<const nv4<T>*>(G.node4);
            nv4<T>* dst = reinterpret_cast<nv4<T>*>(B.node);
            for (int k0 = tid; k0 < nband; k0 += 4 * NT) {
                nv4<T> rec[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (k0 + u * NT < nband) rec[u] = ldm<false>(src + k0 + u * NT);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (k0 + u * NT < nband) stm<true>(dst + k0 + u * NT, rec[u]);
            }
        }
    }
    IB_MARK(2);
    // gather (rho, j) of a rebuilt band from the post-stream populations, four
    // nodes per thread in flight
    const T rho_base = T(S.rho_base);
    for (int k0 = tid; G.dynamic && k0 < nband; k0 += 4 * NT) {
        T h[4][9];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * NT;
            if (k < nband) {
                const int cell = ldm<false>(G.node_cell + k);
                const int x = cell % S.nx, y = cell / S.nx;
#pragma unroll
                for (int i = 0; i < 9; ++i) h[u][i] = ldm<false>(loc<T>(S, i, x, y, sw));
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * NT;
            if (k < nband) stm<CORE>(reinterpret_cast<nv4<T>*>(B.node) + k, band_record<T>(h[u], rho_base));
        }
    }
    // per-thread markers: velocities, arc lengths and running sums over the
    // sweeps in registers (storage precision; the reductions over markers are FP64)
    T mu[MPT], mv[MPT], mds[MPT];
    T acc[MPT][5];
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int g = tid + q * NT;
        mu[q] = mv[q] = mds[q] = T(0);
        if (g < M) {
            int body;
            const int mi = lookup(L, g, body);
            mu[q] = T(ldm<false>(S.mU + mi));
            mv[q] = T(ldm<false>(S.mV + mi));
            mds[q] = T(ldm<false>(S.mds + mi));
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[q][c] = T(0);
    }
    __syncthreads();
    IB_MARK(3);
    const int iters = S.ib_iters;
    for (int n = 0; n < iters; ++n) {
#pragma unroll
        for (int q = 0; q < MPT; ++q) {
            const int g = tid + q * NT;
            if (g < M) {
                T dmx, dmy, dpxx, dpxy, dpyy, rs;
                interp_marker<T, CORE, EXTRA>(B, g, mu[q], mv[q], dmx, dmy, dpxx, dpxy, dpyy, rs);
                acc[q][0] += dmx;
                acc[q][1] += dmy;
                acc[q][2] += dpxx;
                acc[q][3] += dpxy;
                acc[q][4] += dpyy;
                stm<CORE>(B.wt + 2 * g, mds[q] * dmx);
                stm<CORE>(B.wt + 2 * g + 1, mds[q] * dmy);
            }
        }
        __syncthreads();
        if (n < 2) IB_MARK(28 + n);
        // Eqs. 26-27 on the momentum: j(x) += sum_l D(x - X_l) ds_l dm_l, ascending l
        for (int k = tid; k < nband; k += NT) {
            T inc[2];
            spread_node<T, CORE, EXTRA, 2>(B, B.wt, 2, run_at<T, CORE>(B, k), run_at<T, CORE>(B, k + 1), inc);
            nv2<T>* jp = reinterpret_cast<nv2<T>*>(B.node + 4 * k + 2);
            nv2<T> j = ldm<CORE>(jp);
            j.x += inc[0];
            j.y += inc[1];
            stm<CORE>(jp, j);
        }
        __syncthreads();
        IB_MARK(4 + (n < 20 ? n : 19));
    }
    // mismatch left after the sweeps, per-marker force and torque, totals
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int g = tid + q * NT;
        if (g < M) {
            T dmx, dmy, dpxx, dpxy, dpyy, rs;
            interp_marker<T, CORE, EXTRA>(B, g, mu[q], mv[q], dmx, dmy, dpxx, dpxy, dpyy, rs);
            marker_outputs<T>(S, G, L, g, acc[q], dmx, dmy, rs);
        }
    }
    if (tid == 0) G.flags[1] = nband;
    IB_MARK(24);
}

// Colour-class form of a fixed band whose stencil rows are all four consecutive
// band nodes.  Markers are coloured so that no two of a class share a band
// node; the node pass then walks the classes in order, one thread per stencil
// row (marker, ky) adding D * (ds dm) into its four nodes, with no conflicts
// inside a class and a fixed order of the classes at every node.  rho enters
// the sweeps only through each marker's interpolated density, which does not
// change during them and stays in a register; the band keeps 1/rho and j.
// Per-marker arrays are stored by position (class, then marker).  Everything
// the sweeps read is in LDS.
template <typename T>
struct ColBand {
    T* inv;                 // 1/rho per band node
    nv2<T>* j;              // j per band node
    T* wt;                  // per-position weights ds * dm of the current sweep
    T* phi;                 // [8 M] phi_x[4], phi_y[4] per position
    unsigned short* rows;   // [4 M] first band node of each stencil row per position
};

__device__ __forceinline__ void row_starts(nv2<unsigned> rv, int rs[4]) {
    rs[0] = (int)(rv.x & 0xffffu);
    rs[1] = (int)(rv.x >> 16);
    rs[2] = (int)(rv.y & 0xffffu);
    rs[3] = (int)(rv.y >> 16);
}

// density interpolated at marker g from the band records in device memory
// (the same weights and order as the sweeps' interpolation)
template <typename T>
__device__ __forceinline__ T interp_rho(const nv4<T>* node4, nv2<unsigned> rv, const T* phi_g, int g) {
    int rs[4];
    row_starts(rv, rs);
    const nv4<T> a = ldm<false>(reinterpret_cast<const nv4<T>*>(phi_g + g * 8));
    const nv4<T> c = ldm<false>(reinterpret_cast<const nv4<T>*>(phi_g + g * 8) + 1);
    const T px[4] = {a.x, a.y, a.z, a.w}, py[4] = {c.x, c.y, c.z, c.w};
    T rho[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) rho[q] = ldm<false>(reinterpret_cast<const T*>(node4 + rs[q >> 2] + (q & 3)));
    T r = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) r += (px[q & 3] * py[q >> 2]) * rho[q];
    return r;
}

// marker pass on the class band for the marker at position p with row starts
// rv: deviation dm = r U - j*, dPi = r U U - Pi*
template <typename T>
__device__ __forceinline__ void interp_marker_col(const ColBand<T>& B, nv2<unsigned> rv, int p, T r, T U, T V, T& dmx,
                                                  T& dmy, T& dpxx, T& dpxy, T& dpyy) {
    int rs[4];
    row_starts(rv, rs);
    const nv4<T> a = ldm<true>(reinterpret_cast<const nv4<T>*>(B.phi + p * 8));
    const nv4<T> c = ldm<true>(reinterpret_cast<const nv4<T>*>(B.phi + p * 8) + 1);
    const T px[4] = {a.x, a.y, a.z, a.w}, py[4] = {c.x, c.y, c.z, c.w};
    T jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        nv2<T> jv[8];
        T iv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kk = rs[half * 2 + (q >> 2)] + (q & 3);
            jv[q] = ldm<true>(B.j + kk);
            iv[q] = ldm<true>(B.inv + kk);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const T D = px[q & 3] * py[half * 2 + (q >> 2)];
            const T nx = jv[q].x, ny = jv[q].y, inv = iv[q];
            jx += D * nx;
            jy += D * ny;
            pxx += D * nx * nx * inv;
            pxy += D * nx * ny * inv;
            pyy += D * ny * ny * inv;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    dmx = r * U - jx;
    dmy = r * V - jy;
    dpxx = r * U * U - pxx;
    dpxy = r * U * V - pxy;
    dpyy = r * V * V - pyy;
}

// One stencil row of the class spread: D * (ds dm) of the marker at position p
// added to the four band nodes from k0.  With two rows they are requested together.
template <typename T, int R>
__device__ __forceinline__ void class_rows(const ColBand<T>& B, const int p[R], const int ky[R], const int k0[R],
                                           const bool on[R]) {
    nv4<T> px[R];
    T py[R];
    nv2<T> w[R], jv[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!on[r]) continue;
        px[r] = ldm<true>(reinterpret_cast<const nv4<T>*>(B.phi + p[r] * 8));
        py[r] = ldm<true>(B.phi + p[r] * 8 + 4 + ky[r]);
        w[r] = ldm<true>(reinterpret_cast<const nv2<T>*>(B.wt) + p[r]);
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) jv[r][kx] = ldm<true>(B.j + k0[r] + kx);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!on[r]) continue;
        const T pxa[4] = {px[r].x, px[r].y, px[r].z, px[r].w};
#pragma unroll
        for (int kx = 0; kx < 4; ++kx) {
            const T D = pxa[kx] * py[r];
            jv[r][kx].x += D * w[r].x;
            jv[r][kx].y += D * w[r].y;
            stm<true>(B.j + k0[r] + kx, jv[r][kx]);
        }
    }
}

// Steps 3-5 of the correction on a class band whose records were gathered by
// k_band_gather, for groups of at most MPT NT markers.  The marker pass takes
// the markers in their own order (their stencils overlap from lane to lane);
// the node pass walks the classes, with the first nodes of the thread's rows
// held in registers when there are at most kRegClasses classes of at most two
// rows per thread.
constexpr int kRegClasses = 8;

template <typename T, int NT, int MPT>
__device__ __forceinline__ void correct_group_col(const SimDev& S, const GroupDev& G, const GroupLookup& L,
                                                  ColBand<T> B, const int* coff, const T* phi_g, int M, int nband,
                                                  int gi) {
    const int tid = threadIdx.x;
    const nv4<T>* node4 = reinterpret_cast<const nv4<T>*>(G.node4);
    // band records into LDS, four per thread in flight
    for (int i0 = tid; i0 < nband; i0 += 4 * NT) {
        nv4<T> rec[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * NT < nband) rec[u] = ldm<false>(node4 + i0 + u * NT);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * NT;
            if (i < nband) {
                nv2<T> jj;
                jj.x = rec[u].z;
                jj.y = rec[u].w;
                stm<true>(B.inv + i, rec[u].y);
                stm<true>(B.j + i, jj);
            }
        }
    }
    for (int i = tid; i < M; i += NT) {
        const int g = ldm<false>(G.cord + i);
        const nv4<T>* src = reinterpret_cast<const nv4<T>*>(phi_g + g * 8);
        nv4<T>* dst = reinterpret_cast<nv4<T>*>(B.phi + i * 8);
        stm<true>(dst, ldm<false>(src));
        stm<true>(dst + 1, ldm<false>(src + 1));
        stm<true>(reinterpret_cast<nv2<unsigned>*>(B.rows + i * 4),
                  ldm<false>(reinterpret_cast<const nv2<unsigned>*>(G.m_rows) + g));
    }
    IB_MARK(2);
    // the thread's markers g = tid + q NT and their positions
    int pm[MPT];
    T mu[MPT], mv[MPT], mds[MPT], rr[MPT];
    nv2<unsigned> rw[MPT];
    T acc[MPT][5];
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int g = tid + q * NT;
        pm[q] = 0;
        mu[q] = mv[q] = mds[q] = rr[q] = T(0);
        rw[q].x = rw[q].y = 0u;
        if (g < M) {
            int body;
            const int mi = lookup(L, g, body);
            pm[q] = ldm<false>(G.cord + M + g);
            mu[q] = T(ldm<false>(S.mU + mi));
            mv[q] = T(ldm<false>(S.mV + mi));
            mds[q] = T(ldm<false>(S.mds + mi));
            rw[q] = ldm<false>(reinterpret_cast<const nv2<unsigned>*>(G.m_rows) + g);
            rr[q] = interp_rho<T>(node4, rw[q], phi_g, g);
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[q][c] = T(0);
    }
    __syncthreads();
    // the class offsets one per lane, and the first nodes of the thread's rows
    // (4 p + ky = 4 coff[c] + tid + h NT) of every class, two 16-bit halves
    const int ncolor = G.ncolor;
    const int coffv = (tid & 63) <= ncolor ? coff[tid & 63] : 0;
    bool reg = ncolor <= kRegClasses;
    for (int c = 0; c < ncolor; ++c) reg = reg && 4 * (coff[c + 1] - coff[c]) <= 2 * NT;
    unsigned k0h[kRegClasses];
#pragma unroll
    for (int c = 0; c < kRegClasses; ++c) {
        k0h[c] = 0u;
        if (reg && c < ncolor) {
            const int base = 4 * coff[c], nrow = 4 * (coff[c + 1] - coff[c]);
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (tid + h * NT < nrow) k0h[c] |= (unsigned)ldm<true>(B.rows + base + tid + h * NT) << (16 * h);
        }
    }
    IB_MARK(3);
    const int iters = S.ib_iters;
    for (int n = 0; n < iters; ++n) {
#pragma unroll
        for (int q = 0; q < MPT; ++q) {
            const int g = tid + q * NT;
            if (g < M) {
                T dmx, dmy, dpxx, dpxy, dpyy;
                interp_marker_col<T>(B, rw[q], pm[q], rr[q], mu[q], mv[q], dmx, dmy, dpxx, dpxy, dpyy);
                acc[q][0] += dmx;
                acc[q][1] += dmy;
                acc[q][2] += dpxx;
                acc[q][3] += dpxy;
                acc[q][4] += dpyy;
                nv2<T> w;
                w.x = mds[q] * dmx;
                w.y = mds[q] * dmy;
                stm<true>(reinterpret_cast<nv2<T>*>(B.wt) + pm[q], w);
            }
        }
        __syncthreads();
        if (n < 2) IB_MARK(28 + n);
        // Eqs. 26-27 on the momentum, class by class
        if (reg) {
#pragma unroll
            for (int c = 0; c < kRegClasses; ++c) {
                if (c < ncolor) {
                    const int c0 = __builtin_amdgcn_readlane(coffv, c), c1 = __builtin_amdgcn_readlane(coffv, c + 1);
                    int p[2], ky[2], k0[2];
                    bool on[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int t = tid + h * NT, pk = 4 * c0 + t;
                        on[h] = t < 4 * (c1 - c0);
                        p[h] = pk >> 2;
                        ky[h] = pk & 3;
                        k0[h] = (int)((k0h[c] >> (16 * h)) & 0xFFFFu);
                    }
                    class_rows<T, 2>(B, p, ky, k0, on);
                    __syncthreads();
                }
            }
        } else {
            for (int c = 0; c < ncolor; ++c) {
                const int p0 = coff[c], rows_c = 4 * (coff[c + 1] - p0);
                for (int t = tid; t < rows_c; t += NT) {
                    const int pk = 4 * p0 + t;
                    const int p[1] = {pk >> 2}, ky[1] = {pk & 3}, k0[1] = {(int)ldm<true>(B.rows + pk)};
                    const bool on[1] = {true};
                    class_rows<T, 1>(B, p, ky, k0, on);
                }
                __syncthreads();
            }
        }
        IB_MARK(4 + (n < 20 ? n : 19));
    }
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int g = tid + q * NT;
        if (g < M) {
            T dmx, dmy, dpxx, dpxy, dpyy;
            interp_marker_col<T>(B, rw[q], pm[q], rr[q], mu[q], mv[q], dmx, dmy, dpxx, dpxy, dpyy);
            marker_outputs<T>(S, G, L, g, acc[q], dmx, dmy, rr[q]);
        }
    }
    if (tid == 0) G.flags[1] = nband;
    IB_MARK(24);
}

// Correction of a group of free bodies planned, swept and applied inside the
// workgroup, for groups whose stencils lie in one box of kBinCells nodes or
// fewer inside the lattice (no wrap across a periodic side, no node outside):
// the box's cells are counted, scanned and filled as in build_plan_binned, but
// the plan (band nodes in ascending cell order, each node's entries in
// ascending marker order, the band node of every stencil row) stays in LDS,
// the weights of Eq. 15 are computed into LDS, and the final spread and Eq. 28
// correction of the populations follow the sweeps in the same workgroup.  The
// arithmetic and its order are those of correct_group and k_band_apply on the
// same plan.  Returns false, having written nothing to device memory, when the
// group does not qualify or its arrays do not fit the arena.
template <typename T, int NT, int MPT>
__device__ bool correct_free_lds(const SimDev& S, const GroupDev& G, const GroupLookup& L, char* arena,
                                 int arena_bytes, int* scan_tmp, int* bbox, int sw, int gi) {
    const int tid = threadIdx.x;
    const int M = G.M, NE = 16 * M;
    if (M == 0 || M > MPT * NT || NE > 0xFFFF) return false;
    Bump bp;
    bp.base = arena;
    bp.off = 0;
    bp.cap = arena_bytes;
    int* mfx = reinterpret_cast<int*>(bp.take(4L * M));
    int* mfy = reinterpret_cast<int*>(bp.take(4L * M));
    T* phi = reinterpret_cast<T*>(bp.take(8L * M * sizeof(T)));
    T* wt = reinterpret_cast<T*>(bp.take(2L * M * sizeof(T)));
    T* tot = reinterpret_cast<T*>(bp.take(5L * M * sizeof(T)));
    unsigned short* rows = reinterpret_cast<unsigned short*>(bp.take(2L * 4 * M));
    unsigned short* ents = reinterpret_cast<unsigned short*>(bp.take(2L * NE));
    if (!mfx || !mfy || !phi || !wt || !tot || !rows || !ents) return false;
    // stencil corners and the weights of Eq. 15 (the same expressions as the
    // weights of a plan in device memory); the box of the stencils by a
    // reduction in each wave and one LDS atomic per wave
    if (tid < 4) bbox[tid] = tid < 2 ? 0x7fffffff : -0x7fffffff;
    __syncthreads();
    int lx = 0x7fffffff, ly = 0x7fffffff, hx = -0x7fffffff, hy = -0x7fffffff;
    for (int g = tid; g < M; g += NT) {
        int body;
        const int mi = lookup(L, g, body);
        const double X = S.mX[mi], Y = S.mY[mi];
        const double fxd = floor(X) - 1.0, fyd = floor(Y) - 1.0;
        const int fx = (int)fxd, fy = (int)fyd;
        mfx[g] = fx;
        mfy[g] = fy;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            phi[g * 8 + q] = delta_w<T>(S.delta, T(fxd + q - X));
            phi[g * 8 + 4 + q] = delta_w<T>(S.delta, T(fyd + q - Y));
        }
        lx = min(lx, fx);
        ly = min(ly, fy);
        hx = max(hx, fx + 3);
        hy = max(hy, fy + 3);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lx = min(lx, __shfl_xor(lx, off, 64));
        ly = min(ly, __shfl_xor(ly, off, 64));
        hx = max(hx, __shfl_xor(hx, off, 64));
        hy = max(hy, __shfl_xor(hy, off, 64));
    }
    if ((tid & 63) == 0 && lx <= hx) {
        atomicMin(&bbox[0], lx);
        atomicMin(&bbox[1], ly);
        atomicMax(&bbox[2], hx);
        atomicMax(&bbox[3], hy);
    }
    __syncthreads();
    IB_MARK(1);
    const int x0 = bbox[0], y0 = bbox[1];
    const long W = (long)bbox[2] - x0 + 1, H = (long)bbox[3] - y0 + 1;
    const long ncell_l = W * H;
    // per box cell: the count of entries, then the band node (-1 for none);
    // the first entry, then the fill position.  The band records of the
    // sweeps take this space over once the plan is built, when they fit.
    char* plan = reinterpret_cast<char*>(bp.take(8L * ncell_l));
    if (x0 < 0 || y0 < 0 || bbox[2] >= S.nx || bbox[3] >= S.ny || ncell_l > kBinCells || !plan) return false;
    const int ncell = (int)ncell_l, Wi = (int)W;
    int* count = reinterpret_cast<int*>(plan);
    int* start = count + ncell;
    for (int c = tid; c < ncell; c += NT) count[c] = 0;
    __syncthreads();
    for (int e = tid; e < NE; e += NT) {
        const int g = e >> 4, sl = e & 15;
        atomicAdd(&count[(mfy[g] + (sl >> 2) - y0) * Wi + (mfx[g] + (sl & 3) - x0)], 1);
    }
    __syncthreads();
    // one scan of (band nodes << 16 | entries): both totals fit 16 bits
    const int per = (ncell + NT - 1) / NT;
    const int c0 = tid * per, c1 = min(ncell, c0 + per);
    int packed = 0;
    for (int c = c0; c < c1; ++c) packed += (count[c] > 0 ? 1 << 16 : 0) + count[c];
    int ptotal;
    const int pbase = block_scan<NT>(packed, scan_tmp, &ptotal);
    int ebase = pbase & 0xffff, nbase = pbase >> 16;
    const int nband = ptotal >> 16;
    for (int c = c0; c < c1; ++c) {
        const int n = count[c];
        start[c] = ebase;
        count[c] = n > 0 ? nbase++ : -1;
        ebase += n;
    }
    // the band's arrays, sized now that the band is known (the same on every thread)
    unsigned short* run16 = reinterpret_cast<unsigned short*>(bp.take(2L * (nband + 1)));
    int* cells = reinterpret_cast<int*>(bp.take(4L * nband));
    const long rec_bytes = 4L * nband * (long)sizeof(T);
    T* node = rec_bytes <= 8L * ncell_l ? reinterpret_cast<T*>(plan) : reinterpret_cast<T*>(bp.take(rec_bytes));
    if (!run16 || !cells || !node) return false;
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
        const int k = count[c];
        if (k >= 0) {
            cells[k] = c;
            run16[k] = (unsigned short)start[c];
        }
    }
    if (tid == 0) run16[nband] = (unsigned short)NE;
    __syncthreads();
    IB_MARK(30);
    for (int e = tid; e < NE; e += NT) {
        const int g = e >> 4, sl = e & 15;
        const int slot = atomicAdd(&start[(mfy[g] + (sl >> 2) - y0) * Wi + (mfx[g] + (sl & 3) - x0)], 1);
        ents[slot] = (unsigned short)e;  // e = 16 * marker + (ky << 2 | kx)
    }
    // band node of the first cell of each stencil row: its four cells are
    // consecutive cells of the box, all in the band, so consecutive band nodes
    for (int i = tid; i < 4 * M; i += NT) {
        const int g = i >> 2, ky = i & 3;
        rows[i] = (unsigned short)count[(mfy[g] + ky - y0) * Wi + (mfx[g] - x0)];
    }
    __syncthreads();
    // each run ends at its cell's fill position; order it by marker
    for (int k = tid; k < nband; k += NT) {
        const int e0 = run16[k], e1 = run16[k + 1];
        for (int a = e0 + 1; a < e1; ++a) {
            const unsigned short v = ents[a];
            int b = a - 1;
            while (b >= e0 && ents[b] > v) {
                ents[b + 1] = ents[b];
                --b;
            }
            ents[b + 1] = v;
        }
    }
    __syncthreads();
    IB_MARK(2);
    // band records from the post-stream populations (over the counts when
    // they fit there), four nodes per thread in flight
    const T rho_base = T(S.rho_base);
    for (int k0 = tid; k0 < nband; k0 += 4 * NT) {
        T h[4][9];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * NT;
            if (k < nband) {
                const int c = cells[k];
                const int x = x0 + c % Wi, y = y0 + c / Wi;
#pragma unroll
                for (int i = 0; i < 9; ++i) h[u][i] = ldm<false>(loc<T>(S, i, x, y, sw));
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * NT;
            if (k < nband) stm<true>(reinterpret_cast<nv4<T>*>(node) + k, band_record<T>(h[u], rho_base));
        }
    }
    Band<T> B;
    B.node = node;
    B.wt = wt;
    B.run16 = run16;
    B.run32 = nullptr;
    B.rows = rows;
    B.mn32 = nullptr;
    B.phi = phi;
    B.ent16 = ents;
    B.entpk = nullptr;
    T mu[MPT], mv[MPT], mds[MPT];
    T acc[MPT][5];
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int g = tid + q * NT;
        mu[q] = mv[q] = mds[q] = T(0);
        if (g < M) {
            int body;
            const int mi = lookup(L, g, body);
            mu[q] = T(ldm<false>(S.mU + mi));
            mv[q] = T(ldm<false>(S.mV + mi));
            mds[q] = T(ldm<false>(S.mds + mi));
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[q][c] = T(0);
    }
    __syncthreads();
    IB_MARK(3);
    const int iters = S.ib_iters;
    for (int n = 0; n < iters; ++n) {
#pragma unroll
        for (int q = 0; q < MPT; ++q) {
            const int g = tid + q * NT;
            if (g < M) {
                T dmx, dmy, dpxx, dpxy, dpyy, rs;
                interp_marker<T, true, true>(B, g, mu[q], mv[q], dmx, dmy, dpxx, dpxy, dpyy, rs);
                acc[q][0] += dmx;
                acc[q][1] += dmy;
                acc[q][2] += dpxx;
                acc[q][3] += dpxy;
                acc[q][4] += dpyy;
                stm<true>(wt + 2 * g, mds[q] * dmx);
                stm<true>(wt + 2 * g + 1, mds[q] * dmy);
            }
        }
        __syncthreads();
        // Eqs. 26-27 on the momentum: j(x) += sum_l D(x - X_l) ds_l dm_l, ascending l
        for (int k = tid; k < nband; k += NT) {
            T inc[2];
            spread_node<T, true, true, 2>(B, wt, 2, run16[k], run16[k + 1], inc);
            nv2<T>* jp = reinterpret_cast<nv2<T>*>(node + 4 * k + 2);
            nv2<T> j = ldm<true>(jp);
            j.x += inc[0];
            j.y += inc[1];
            stm<true>(jp, j);
        }
        __syncthreads();
        IB_MARK(4 + (n < 20 ? n : 19));
    }
    // mismatch left after the sweeps, per-marker force and torque (device
    // memory, for the FP64 reductions) and the totals of the sweeps (LDS)
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int g = tid + q * NT;
        if (g < M) {
            T dmx, dmy, dpxx, dpxy, dpyy, rs;
            interp_marker<T, true, true>(B, g, mu[q], mv[q], dmx, dmy, dpxx, dpxy, dpyy, rs);
            int body;
            const int mi = lookup(L, g, body);
            const double ds = ldm<false>(S.mds + mi);
            const BodyDev& Bd = S.bodies[body];
            const double Fx = -ds * (double)acc[q][0], Fy = -ds * (double)acc[q][1];
            const double r2 = (double)dmx * (double)dmx + (double)dmy * (double)dmy;
            double* mr = G.m_red + g * 5;
            mr[0] = Fx;
            mr[1] = Fy;
            mr[2] = (S.mX[mi] - Bd.xc[0]) * Fy - (S.mY[mi] - Bd.xc[1]) * Fx;
            mr[3] = r2;
            mr[4] = sqrt(r2) / (double)rs;
#pragma unroll
            for (int c = 0; c < 5; ++c) stm<true>(tot + g * 5 + c, T(ds * (double)acc[q][c]));
        }
    }
    __syncthreads();
    IB_MARK(24);
    // final spread of the totals and Eq. 28 at every band node
    for (int k = tid; k < nband; k += NT) {
        T t[5];
        spread_node<T, true, true, 5>(B, tot, 5, run16[k], run16[k + 1], t);
        const int c = cells[k];
        correct_node<T>(S, x0 + c % Wi, y0 + c / Wi, sw, t);
    }
    (void)gi;
    return true;
}

// Band records of a plan in device memory (node cells, records in node4),
// from the post-stream populations, four nodes per thread in flight (their
// four cells requested together, then their 36 populations).
template <typename T, int NT>
__device__ void gather_band(const SimDev& S, const GroupDev& G, int nband, int sw) {
    const T rho_base = T(S.rho_base);
    nv4<T>* node4 = reinterpret_cast<nv4<T>*>(G.node4);
    for (int k0 = threadIdx.x; k0 < nband; k0 += 4 * NT) {
        int cell[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cell[u] = k0 + u * NT < nband ? ldm<false>(G.node_cell + k0 + u * NT) : 0;
        T h[4][9];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (k0 + u * NT < nband) {
                const int x = cell[u] % S.nx, y = cell[u] / S.nx;
#pragma unroll
                for (int i = 0; i < 9; ++i) h[u][i] = ldm<false>(loc<T>(S, i, x, y, sw));
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * NT;
            if (k < nband) stm<false>(node4 + k, band_record<T>(h[u], rho_base));
        }
    }
}

// Final spread of a plan in device memory and Eq. 28 at its band nodes,
// inside the workgroup that corrected the group (after correct_group or
// correct_group_col, which leave the per-marker totals in m_wtot).  Groups
// never share a band node, and every (node, population) pair has a slot of
// its own in either AA state, so the groups of a launch apply side by side.
// U nodes per thread at a time: their run bounds and cells are requested
// together before the spreads (one node per round left the workgroup waiting
// on their loads too); each node's spread and Eq. 28 then follow as in
// k_band_apply (loading the populations before the spreads as well measured
// slower).
template <typename T, int NT, int U>
__device__ void apply_band(const SimDev& S, const GroupDev& G, int nband, int sw) {
    Band<T> B;
    B.entpk = G.ent_D;
    B.run32 = G.node_run;
    for (int k0 = threadIdx.x; k0 < nband; k0 += U * NT) {
        int e0[U], e1[U], cell[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * NT;
            e0[u] = e1[u] = cell[u] = 0;
            if (k < nband) {
                e0[u] = ldm<false>(G.node_run + k);
                e1[u] = ldm<false>(G.node_run + k + 1);
                cell[u] = ldm<false>(G.node_cell + k);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u * NT < nband) {
                T t[5];
                spread_node<T, false, false, 5>(B, reinterpret_cast<const T*>(G.m_wtot), 5, e0[u], e1[u], t);
                correct_node<T>(S, cell[u] % S.nx, cell[u] / S.nx, sw, t);
            }
        }
    }
}

// The correction of every group of a launch, one workgroup per group at a
// time (k_ib and k_ib_lean).
// bc_items (batches): the lane's boundary items (hdr->nbc of them), taken by
// every workgroup after its groups, 256 threads per item, when no band of the
// lane comes near a non-periodic side (the rules and the correction then touch
// disjoint populations); nullptr: none.
template <typename T, int NT, int MPT>
__device__ __forceinline__ void ib_groups(const SimDev* __restrict__ sims, GroupDev* __restrict__ groups,
                                          const BatchHeader* __restrict__ hdr, int ngroups_arg, int parity,
                                          char* arena, int arena_bytes, const int2* __restrict__ bc_items) {
    __shared__ double part[4 * 5];
    __shared__ int scan_tmp[NT];
    __shared__ double body_out[8][5];
    __shared__ GroupLookup L;
    __shared__ int bbox[4];
    __shared__ int coff_s[kMaxColors + 1];
    raise_wave_priority();
    const int ngroups = hdr ? hdr->ngroups : ngroups_arg;
    const int tid = threadIdx.x;
    for (int gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
        const GroupDev& G = groups[gi];
        const SimDev& S = sims[G.sim];
        if (!S.active) continue;
        const int sw = 1 - (parity >= 0 ? parity : S.swapped);
        const int M = G.M;
        int nband = G.nband, nent = G.nent;
        IB_MARK(0);
        // body lookup of the group: the first wave reads every body at once
        // and scans their marker counts
        if (tid < 64) {
            const int nb = G.nbody;
            int n = 0;
            if (tid < nb) {
                const int b = G.body[tid];
                const BodyDev& Bd = S.bodies[b];
                L.body[tid] = b;
                L.m0[tid] = Bd.m0;
                n = Bd.n;
            }
            int incl = n;
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                const int y = __shfl_up(incl, off, 64);
                if (tid >= off) incl += y;
            }
            if (tid <= nb) L.gbase[tid] = incl - n;
            if (tid == 0) L.nb = nb;
        }
        __syncthreads();
        IB_MARK(31);
        if (G.dynamic && correct_free_lds<T, NT, MPT>(S, G, L, arena, arena_bytes, scan_tmp, bbox, sw, gi)) {
            __syncthreads();
            IB_MARK(25);
        } else {
            if (G.dynamic && !build_plan_binned<NT>(S, G, reinterpret_cast<int*>(arena), arena_bytes, scan_tmp, bbox, nband, nent))
                build_plan<NT>(S, G, reinterpret_cast<unsigned long long*>(arena), scan_tmp, nband, nent);
            IB_MARK(30);
            T* phi_g = reinterpret_cast<T*>(G.m_phi);
            // stencil weights of Eq. 15: phi per marker, D per stencil entry (static plans: once)
            const bool fresh = G.dynamic || G.flags[0] == 0;
            __syncthreads();
            if (fresh) {
                for (int g = tid; g < M; g += NT) {
                    int body;
                    const int mi = lookup(L, g, body);
                    const double X = S.mX[mi], Y = S.mY[mi];
                    const double fx = floor(X) - 1.0, fy = floor(Y) - 1.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        phi_g[g * 8 + q] = delta_w<T>(S.delta, T(fx + q - X));
                        phi_g[g * 8 + 4 + q] = delta_w<T>(S.delta, T(fy + q - Y));
                    }
                }
                __syncthreads();
                for (int e = tid; e < nent; e += NT) {
                    const int p = G.ent[e];
                    const int g = p >> 4;
                    store_entry<T>(G.ent_D, e, g, phi_g[g * 8 + (p & 3)] * phi_g[g * 8 + 4 + ((p >> 2) & 3)]);
                }
                if (!G.dynamic)
                    for (int g = tid; g < M; g += NT)
                        stm<false>(reinterpret_cast<nv2<unsigned>*>(G.m_rows) + g, stencil_rows(G, g));
                __syncthreads();
                if (tid == 0 && !G.dynamic) G.flags[0] = 1;
            }
            IB_MARK(1);
            // band records (rho, 1/rho, j) of a fixed plan from the post-stream
            // populations (a rebuilt plan gathers its own in correct_group)
            if (!G.dynamic && G.in_kernel) {
                gather_band<T, NT>(S, G, nband, sw);
                __syncthreads();
            }
            // placement of the working arrays (the same decision on every thread):
            // the segment band when the plan has one and it fits, else the entry band
            bool done = false;
            // (two markers per thread at most in the wide kernels, whose larger
            // groups never fit the class band; the 256-thread kernels keep all
            // of theirs, at most 1280 markers, whose class band fits the arena;
            // the 512-thread lean kernel carries one)
            constexpr int MPTC = NT <= 256 ? MPT : (MPT < 2 ? MPT : 2);
            if (G.ncolor > 0 && M <= MPTC * NT) {
                Bump cb;
                cb.base = arena;
                cb.off = 0;
                cb.cap = arena_bytes;
                ColBand<T> CB;
                CB.inv = reinterpret_cast<T*>(cb.take((long)nband * sizeof(T)));
                CB.j = reinterpret_cast<nv2<T>*>(cb.take(2L * nband * sizeof(T)));
                CB.wt = reinterpret_cast<T*>(cb.take(2L * M * sizeof(T)));
                CB.phi = reinterpret_cast<T*>(cb.take(8L * M * sizeof(T)));
                CB.rows = reinterpret_cast<unsigned short*>(cb.take(2L * 4 * M));
                if (CB.inv && CB.j && CB.wt && CB.phi && CB.rows) {
                    if (tid <= G.ncolor) coff_s[tid] = G.coff[tid];
                    __syncthreads();
                    correct_group_col<T, NT, MPTC>(S, G, L, CB, coff_s, phi_g, M, nband, gi);
                    done = true;
                }
            }
            Bump bump;
            bump.base = arena;
            bump.off = 0;
            bump.cap = arena_bytes;
            Band<T> B;
            T* lnode = reinterpret_cast<T*>(bump.take(4L * nband * sizeof(T)));
            T* lwt = reinterpret_cast<T*>(bump.take(2L * M * sizeof(T)));
            unsigned short* lrun = reinterpret_cast<unsigned short*>(bump.take(2L * (nband + 1)));
            unsigned short* lrows = reinterpret_cast<unsigned short*>(bump.take(2L * 4 * M));
            const bool core = nband < 0xFFFF && nent < 0xFFFF && lnode && lwt && lrun && lrows;
            T* lphi = core ? reinterpret_cast<T*>(bump.take(8L * M * sizeof(T))) : nullptr;
            unsigned short* lent = core ? reinterpret_cast<unsigned short*>(bump.take(2L * nent)) : nullptr;
            const bool extra = core && lphi && lent && M < 4096;
            B.mn32 = G.mnode;
            B.entpk = G.ent_D;
            B.run32 = G.node_run;
            if (core) {
                B.node = lnode;
                B.wt = lwt;
                B.run16 = lrun;
                B.rows = lrows;
            } else {
                B.node = reinterpret_cast<T*>(G.node4);
                B.wt = reinterpret_cast<T*>(G.m_wtot);
                B.run16 = nullptr;
                B.rows = nullptr;
            }
            if (extra) {
                B.phi = lphi;
                B.ent16 = lent;
            } else {
                B.phi = phi_g;
                B.ent16 = nullptr;
            }
            if (done) {
                // corrected on the class band
            } else if (extra) {
                correct_group<T, NT, MPT, true, true>(S, G, L, B, phi_g, M, nband, nent, sw, gi);
            } else if (core) {
                correct_group<T, NT, MPT, true, false>(S, G, L, B, phi_g, M, nband, nent, sw, gi);
            } else {
                correct_group<T, NT, MPT, false, false>(S, G, L, B, phi_g, M, nband, nent, sw, gi);
            }
            __syncthreads();
            if (G.in_kernel) {
                apply_band<T, NT, MPT == 1 ? 2 : 4>(S, G, nband, sw);
                __syncthreads();
            }
            IB_MARK(25);
        }
        // FP64 reductions per body (order fixed by the marker index)
        for (int b = 0; b < G.nbody; ++b) {
            const int nb = L.gbase[b + 1] - L.gbase[b];
            double o[5];
            body_reduce(nb, G.m_red + L.gbase[b] * 5, part, o);
            if (tid == 0) {
                body_out[b][0] = o[0];
                body_out[b][1] = o[1];
                body_out[b][2] = o[2];
                body_out[b][3] = sqrt(o[3] / nb);
                body_out[b][4] = o[4];
            }
        }
        __syncthreads();
        IB_MARK(26);
        // outputs, then the rigid-body update of free circles (Eqs. 37, 39-42):
        // collision forces from the positions before any body moves, one body per thread
        BodyDev* bodies = S.bodies;
        if (tid < G.nbody) {
            BodyDev& Bd = bodies[G.body[tid]];
            Bd.F[0] = body_out[tid][0];
            Bd.F[1] = body_out[tid][1];
            Bd.T = body_out[tid][2];
            Bd.resid = body_out[tid][3];
            Bd.maxslip = body_out[tid][4];
            double fx = 0.0, fy = 0.0;
            if (Bd.kind == BODY_FREE) {
                const double gmag = sqrt(S.gravity[0] * S.gravity[0] + S.gravity[1] * S.gravity[1]);
                const double V = M_PI * Bd.R * Bd.R;
                const double cij = (Bd.rho_s * V - S.rho0 * V) * gmag;  // buoyancy-reduced weight
                const double gap = 0.1 * Bd.R;                          // xi = 0.05 D
                for (int c = 0; c < G.nbody; ++c) {
                    const BodyDev& O = bodies[G.body[c]];
                    if (c == tid || O.kind != BODY_FREE) continue;
                    collision_force(Bd.xc[0], Bd.xc[1], O.xc[0], O.xc[1], Bd.R, O.R, cij, gap, fx, fy);
                }
                // walls act through mirror particles of the same radius; walls sit half
                // a spacing outside the first and last nodes
                if (S.bc[SIDE_W] == BC_WALL || S.bc[SIDE_W] == BC_FREESLIP)
                    collision_force(Bd.xc[0], Bd.xc[1], -1.0 - Bd.xc[0], Bd.xc[1], Bd.R, Bd.R, cij, gap, fx, fy);
                if (S.bc[SIDE_E] == BC_WALL || S.bc[SIDE_E] == BC_FREESLIP)
                    collision_force(Bd.xc[0], Bd.xc[1], 2.0 * S.nx - 1.0 - Bd.xc[0], Bd.xc[1], Bd.R, Bd.R, cij, gap,
                                    fx, fy);
                if (S.bc[SIDE_S] == BC_WALL || S.bc[SIDE_S] == BC_FREESLIP)
                    collision_force(Bd.xc[0], Bd.xc[1], Bd.xc[0], -1.0 - Bd.xc[1], Bd.R, Bd.R, cij, gap, fx, fy);
                if (S.bc[SIDE_N] == BC_WALL || S.bc[SIDE_N] == BC_FREESLIP)
                    collision_force(Bd.xc[0], Bd.xc[1], Bd.xc[0], 2.0 * S.ny - 1.0 - Bd.xc[1], Bd.R, Bd.R, cij, gap,
                                    fx, fy);
            }
            body_out[tid][0] = fx;
            body_out[tid][1] = fy;
        }
        __syncthreads();
        if (tid < G.nbody) {
            BodyDev& Bd = bodies[G.body[tid]];
            if (Bd.kind == BODY_FREE) {
                const double rho_f = S.rho0;
                const double V = M_PI * Bd.R * Bd.R, Ms = Bd.rho_s * V, Is = 0.5 * Ms * Bd.R * Bd.R;
                const double Ftx = Bd.F[0] + rho_f * V * (Bd.U[0] - Bd.Uprev[0]) + body_out[tid][0] + (Ms - rho_f * V) * S.gravity[0];
                const double Fty = Bd.F[1] + rho_f * V * (Bd.U[1] - Bd.Uprev[1]) + body_out[tid][1] + (Ms - rho_f * V) * S.gravity[1];
                const double Tt = Bd.T + (rho_f / Bd.rho_s) * Is * (Bd.omega - Bd.omega_prev);
                // Eq. 42 advances positions with the level-n velocities, Eq. 41 the velocities
                Bd.xc[0] += Bd.U[0] + 0.5 * Ftx / Ms;
                Bd.xc[1] += Bd.U[1] + 0.5 * Fty / Ms;
                Bd.theta += Bd.omega + 0.5 * Tt / Is;
                Bd.Uprev[0] = Bd.U[0];
                Bd.Uprev[1] = Bd.U[1];
                Bd.omega_prev = Bd.omega;
                Bd.U[0] += Ftx / Ms;
                Bd.U[1] += Fty / Ms;
                Bd.omega += Tt / Is;
            }
        }
        __syncthreads();
        // regenerate the markers of free circles for the next step
        for (int g = tid; g < M; g += NT) {
            int body;
            const int mi = lookup(L, g, body);
            const BodyDev& B = S.bodies[body];
            if (B.kind != BODY_FREE) continue;
            const int l = mi - B.m0;
            const double a = 2.0 * M_PI * l / B.n + B.theta;
            const double X = B.xc[0] + B.R * cos(a), Y = B.xc[1] + B.R * sin(a);
            S.mX[mi] = X;
            S.mY[mi] = Y;
            S.mU[mi] = B.U[0] - B.omega * (Y - B.xc[1]);
            S.mV[mi] = B.U[1] + B.omega * (X - B.xc[0]);
        }
        __syncthreads();
        IB_MARK(27);
    }
    if (bc_items) {
        constexpr int per = NT / 256;  // items per workgroup and round
        const int nbc = hdr->nbc;
        for (int it = blockIdx.x * per + tid / 256; it < nbc; it += gridDim.x * per)
            boundary_item<T>(sims, bc_items[it], tid % 256, parity);
    }
}

template <typename T, int NT, int MPT>
__global__ void __launch_bounds__(NT)
    k_ib(const SimDev* __restrict__ sims, GroupDev* __restrict__ groups, const BatchHeader* __restrict__ hdr,
         int ngroups_arg, int parity, const int2* bc_items) {
    __shared__ __align__(16) char arena[kIbArenaBytes];
    ib_groups<T, NT, MPT>(sims, groups, hdr, ngroups_arg, parity, arena, kIbArenaBytes, bc_items);
}

// Workgroups that find room on a CU once a few sweep waves per SIMD have
// finished there, so the correction of one lane runs while the other lane's
// sweep streams (a 768-thread k_ib needs a CU with no sweep wave left).
// MPT = 1 (groups of at most 256 markers): 512 threads, two waves per SIMD of
// at most 128 VGPRs and a 96 KiB arena, room once four sweep waves per SIMD are
// gone (256 threads: 0.210 against 0.198 ms per step on the served mix in
// halves); MPT = 2 and 5 (at most 512 and 1280 markers): 256 threads, one
// wave per SIMD of up to 256 VGPRs (a tighter cap spills, and measured slower)
// and the full arena, room once four are gone.
template <int MPT>
constexpr int kLeanArenaBytes = MPT == 1 ? kIbLeanArenaBytes : kIbArenaBytes;
template <int MPT>
constexpr int kLeanThreads = MPT == 1 ? 512 : 256;

template <typename T, int MPT>
__global__ void __launch_bounds__(kLeanThreads<MPT>) __attribute__((amdgpu_waves_per_eu(MPT == 1 ? 4 : 2, 8)))
    k_ib_lean(const SimDev* __restrict__ sims, GroupDev* __restrict__ groups, const BatchHeader* __restrict__ hdr,
              int ngroups_arg, int parity, const int2* bc_items) {
    extern __shared__ __align__(16) char lean_arena[];  // kLeanArenaBytes<MPT> at launch
    ib_groups<T, kLeanThreads<MPT>, MPT>(sims, groups, hdr, ngroups_arg, parity, lean_arena, kLeanArenaBytes<MPT>,
                                         bc_items);
}

// ---------------------------------------------------------------- bookkeeping and I/O

// Work of the band kernels: chunks of 256 band nodes (group, first node) of
// the groups with large fixed plans, whose band one workgroup would gather and
// apply slowly (each node's populations lie in nine cache lines); k_ib
// gathers and applies every other band itself.

// Band records (rho, 1/rho, j) of the groups with fixed plans, from the
// post-stream populations, before the correction sweeps.
template <typename T>
__global__ void __launch_bounds__(256)
    k_band_gather(const SimDev* __restrict__ sims, const GroupDev* __restrict__ groups,
                  const int2* __restrict__ chunks, const BatchHeader* __restrict__ hdr, int nchunks_arg, int parity) {
    raise_wave_priority();
    const int nchunks = hdr ? hdr->nchunks : nchunks_arg;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int2 ch = chunks[c];
        const GroupDev& G = groups[ch.x];
        const SimDev& S = sims[G.sim];
        if (!S.active || G.in_kernel) continue;
        const int k = ch.y + threadIdx.x;
        if (k >= G.nband) continue;
        const int sw = 1 - (parity >= 0 ? parity : S.swapped);
        const int cell = ldm<false>(G.node_cell + k);
        const int x = cell % S.nx, y = cell / S.nx;
        T f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = ldm<false>(loc<T>(S, i, x, y, sw));
        stm<false>(reinterpret_cast<nv4<T>*>(G.node4) + k, band_record<T>(f, T(S.rho_base)));
    }
}

// Final spread of the summed corrections and correction of the populations
// (Eqs. 26-27; Eq. 28 is linear in dm and dPi, so the N sweeps' deviations
// are spread once from their per-marker totals), one band node per thread of
// the groups with large fixed plans (k_ib applies the others itself); each
// node sums its stencil entries in ascending marker order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_band_apply(const SimDev* __restrict__ sims, const GroupDev* __restrict__ groups,
                 const int2* __restrict__ chunks, const BatchHeader* __restrict__ hdr, int nchunks_arg, int parity) {
    raise_wave_priority();
    const int nchunks = hdr ? hdr->nchunks : nchunks_arg;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int2 ch = chunks[c];
        const GroupDev& G = groups[ch.x];
        const SimDev& S = sims[G.sim];
        if (!S.active || G.in_kernel) continue;  // applied by k_ib itself
        const int k = ch.y + threadIdx.x;
        if (k >= G.nband) continue;
        const int sw = 1 - (parity >= 0 ? parity : S.swapped);
        Band<T> B;
        B.entpk = G.ent_D;
        B.run32 = G.node_run;
        T t[5];
        spread_node<T, false, false, 5>(B, reinterpret_cast<const T*>(G.m_wtot), 5, ldm<false>(G.node_run + k),
                                        ldm<false>(G.node_run + k + 1), t);
        const int cell = ldm<false>(G.node_cell + k);
        correct_node<T>(S, cell % S.nx, cell / S.nx, sw, t);
    }
}

__global__ void k_advance(SimDev* sims, const BatchHeader* hdr, int nsims_arg) {
    const int nsims = hdr ? hdr->nsims : nsims_arg;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsims; s += gridDim.x * blockDim.x) {
        SimDev& S = sims[s];
        if (!S.active) continue;
        S.swapped ^= 1;
        S.steps_done += 1;
        if (S.steps_left > 0) {
            S.steps_left -= 1;
            if (S.steps_left == 0) S.active = 0;
        }
    }
}

// Fields of rows y0 .. y0 + gridDim.y - 1, written from index 0 of the outputs.
template <typename T>
__global__ void k_fields(const SimDev* sim, int sw, int y0, double* rho, double* ux, double* uy) {
    const SimDev& S = *sim;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
    if (x >= S.nx) return;
    double h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = (double)*loc<T>(S, i, x, y, sw);
    const double Ssum = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const double r = S.rho_base + Ssum;
    const double jx = (h[1] + h[5] + h[8]) - (h[3] + h[6] + h[7]);
    const double jy = (h[2] + h[5] + h[6]) - (h[4] + h[7] + h[8]);
    const int64_t c = (int64_t)(y - y0) * S.nx + x;
    if (rho) rho[c] = r;
    if (ux) ux[c] = jx / r;
    if (uy) uy[c] = jy / r;
}

template <typename T>
__global__ void k_get_pop(const SimDev* sim, int sw, double* f) {
    const SimDev& S = *sim;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= S.nx) return;
    const int64_t np = (int64_t)S.nx * S.ny, c = (int64_t)y * S.nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i * np + c] = (double)*loc<T>(S, i, x, y, sw) + weight_of<double>(i) * S.rho_base;
}

template <typename T>
__global__ void k_set_pop(const SimDev* sim, int sw, const double* f) {
    const SimDev& S = *sim;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= S.nx) return;
    const int64_t np = (int64_t)S.nx * S.ny, c = (int64_t)y * S.nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) *loc<T>(S, i, x, y, sw) = T(f[i * np + c] - weight_of<double>(i) * S.rho_base);
}

template <typename T>
__global__ void k_set_eq(const SimDev* sim, int sw, const double* rho, const double* ux, const double* uy,
                         double rho0, double u0x, double u0y) {
    const SimDev& S = *sim;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= S.nx) return;
    const int64_t c = (int64_t)y * S.nx + x;
    const double r = rho ? rho[c] : rho0, u = ux ? ux[c] : u0x, v = uy ? uy[c] : u0y;
    const double uu = u * u + v * v;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double eu = ex_of(i) * u + ey_of(i) * v;
        const double feq = weight_of<double>(i) * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        *loc<T>(S, i, x, y, sw) = T(feq - weight_of<double>(i) * S.rho_base);
    }
}

// ---------------------------------------------------------------- launchers

template <typename T, bool MRT, int TX, int TY, int RPT, bool NTMP>
static hipError_t sweep_t(const SimDev* sims, const int4* tiles, const BatchHeader* hdr, int ntiles, int grid,
                          int parity, hipStream_t st) {
    hipLaunchKernelGGL((k_sweep<T, TX, TY, RPT, NTMP, MRT>), dim3(grid), dim3(TX, TY), 0, st, sims, tiles, hdr, ntiles,
                       parity);
    return hipGetLastError();
}

template <typename T, bool MRT, int W, int R, bool NTMP>
static hipError_t sweep_b(const SimDev* sims, const int4* tiles, const BatchHeader* hdr, int ntiles, int grid,
                          int parity, hipStream_t st) {
    hipLaunchKernelGGL((k_sweep_blk<T, W, R, NTMP, MRT>), dim3(grid), dim3(64 * W), 0, st, sims, tiles, hdr, ntiles,
                       parity);
    return hipGetLastError();
}

template <typename T, bool MRT>
static hipError_t sweep_tt(int tiling, const SimDev* sims, const int4* tiles, const BatchHeader* hdr, int ntiles,
                           int grid, int parity, hipStream_t st) {
    switch (tiling) {
        case 16: return sweep_b<T, MRT, 4, 1, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 17: return sweep_b<T, MRT, 4, 2, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 18: return sweep_b<T, MRT, 8, 1, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 19: return sweep_b<T, MRT, 4, 1, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 0: return sweep_t<T, MRT, 64, 4, 1, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 1: return sweep_t<T, MRT, 64, 4, 2, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 2: return sweep_t<T, MRT, 128, 2, 2, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 3: return sweep_t<T, MRT, 256, 1, 2, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 4: return sweep_t<T, MRT, 256, 1, 4, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 5: return sweep_t<T, MRT, 64, 4, 4, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 6: return sweep_t<T, MRT, 256, 1, 1, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 7: return sweep_t<T, MRT, 128, 2, 1, false>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 8: return sweep_t<T, MRT, 64, 4, 1, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 9: return sweep_t<T, MRT, 64, 4, 2, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 10: return sweep_t<T, MRT, 128, 2, 2, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 11: return sweep_t<T, MRT, 256, 1, 2, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 12: return sweep_t<T, MRT, 256, 1, 4, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 13: return sweep_t<T, MRT, 64, 4, 4, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 14: return sweep_t<T, MRT, 256, 1, 1, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        case 15: return sweep_t<T, MRT, 128, 2, 1, true>(sims, tiles, hdr, ntiles, grid, parity, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(bool f64, bool mrt, int tiling, const SimDev* sims, const int4* tiles, const BatchHeader* hdr,
                        int ntiles, int grid, int parity, hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    if (mrt)
        return f64 ? sweep_tt<double, true>(tiling, sims, tiles, hdr, ntiles, grid, parity, stream)
                   : sweep_tt<float, true>(tiling, sims, tiles, hdr, ntiles, grid, parity, stream);
    return f64 ? sweep_tt<double, false>(tiling, sims, tiles, hdr, ntiles, grid, parity, stream)
               : sweep_tt<float, false>(tiling, sims, tiles, hdr, ntiles, grid, parity, stream);
}

hipError_t launch_boundary(bool f64, const SimDev* sims, const int2* items, const BatchHeader* hdr, int nitems,
                           int grid, int parity, hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_boundary<double>, dim3(grid), dim3(256), 0, stream, sims, items, hdr, nitems, parity);
    else
        hipLaunchKernelGGL(k_boundary<float>, dim3(grid), dim3(256), 0, stream, sims, items, hdr, nitems, parity);
    return hipGetLastError();
}

template <typename T, int NT, int MPT>
static hipError_t ib_t(const SimDev* sims, GroupDev* groups, const BatchHeader* hdr, int ngroups, int grid,
                       int parity, hipStream_t stream, const int2* bc_items) {
    hipLaunchKernelGGL((k_ib<T, NT, MPT>), dim3(grid), dim3(NT), 0, stream, sims, groups, hdr, ngroups, parity,
                       bc_items);
    return hipGetLastError();
}

template <typename T, int MPT>
static hipError_t ib_lean_t(const SimDev* sims, GroupDev* groups, const BatchHeader* hdr, int ngroups, int grid,
                            int parity, hipStream_t stream, const int2* bc_items) {
    static const hipError_t attr =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ib_lean<T, MPT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLeanArenaBytes<MPT>);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_ib_lean<T, MPT>), dim3(grid), dim3(kLeanThreads<MPT>), kLeanArenaBytes<MPT>, stream, sims,
                       groups, hdr, ngroups, parity, bc_items);
    return hipGetLastError();
}

int ib_variant(bool f64, int max_markers, bool lean) {
    if (f64) return max_markers <= 8 * 256 ? 0 : 1;
    if (lean && max_markers <= 1280) return max_markers <= 256 ? 4 : (max_markers <= 512 ? 5 : 6);
    return max_markers <= 3 * 768 ? 2 : 3;
}

hipError_t launch_ib(bool f64, int max_markers, const SimDev* sims, GroupDev* groups, const BatchHeader* hdr,
                     int ngroups, int grid, int parity, hipStream_t stream, bool lean, const int2* bc_items) {
    if (bc_items && !hdr) return hipErrorInvalidValue;  // the item count comes from the header
    if (grid <= 0) return hipSuccess;
    if (max_markers > kMaxGroupMarkers) return hipErrorInvalidValue;
    // each thread keeps up to MPT markers' running sums in registers
    if (f64)
        return max_markers <= 8 * 256
                   ? ib_t<double, 256, 8>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items)
                   : ib_t<double, 256, 16>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items);
    if (lean && max_markers <= 256)
        return ib_lean_t<float, 1>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items);
    if (lean && max_markers <= 512)
        return ib_lean_t<float, 2>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items);
    if (lean && max_markers <= 1280)
        return ib_lean_t<float, 5>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items);
    return max_markers <= 3 * 768 ? ib_t<float, 768, 3>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items)
                                  : ib_t<float, 512, 8>(sims, groups, hdr, ngroups, grid, parity, stream, bc_items);
}

hipError_t launch_band(bool f64, bool apply, const SimDev* sims, const GroupDev* groups, const int2* chunks,
                       const BatchHeader* hdr, int nchunks, int grid, int parity, hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    if (apply) {
        if (f64)
            hipLaunchKernelGGL(k_band_apply<double>, dim3(grid), dim3(256), 0, stream, sims, groups, chunks, hdr, nchunks, parity);
        else
            hipLaunchKernelGGL(k_band_apply<float>, dim3(grid), dim3(256), 0, stream, sims, groups, chunks, hdr, nchunks, parity);
    } else {
        if (f64)
            hipLaunchKernelGGL(k_band_gather<double>, dim3(grid), dim3(256), 0, stream, sims, groups, chunks, hdr, nchunks, parity);
        else
            hipLaunchKernelGGL(k_band_gather<float>, dim3(grid), dim3(256), 0, stream, sims, groups, chunks, hdr, nchunks, parity);
    }
    return hipGetLastError();
}

hipError_t launch_advance(SimDev* sims, const BatchHeader* hdr, int nsims, hipStream_t stream) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, stream, sims, hdr, nsims);
    return hipGetLastError();
}

#define IO_LAUNCH(kern, ...)                                                                             \
    do {                                                                                                 \
        dim3 grid((nx + 127) / 128, ny), block(128);                                                     \
        if (f64)                                                                                         \
            hipLaunchKernelGGL(kern<double>, grid, block, 0, stream, __VA_ARGS__);                       \
        else                                                                                             \
            hipLaunchKernelGGL(kern<float>, grid, block, 0, stream, __VA_ARGS__);                        \
        return hipGetLastError();                                                                        \
    } while (0)

hipError_t launch_fields(bool f64, const SimDev* sim, int nx, int ny, int sw, double* rho, double* ux, double* uy,
                         hipStream_t stream) {
    IO_LAUNCH(k_fields, sim, sw, 0, rho, ux, uy);
}
hipError_t launch_fields_rows(bool f64, const SimDev* sim, int nx, int y0, int rows, int sw, double* rho, double* ux,
                              double* uy, hipStream_t stream) {
    const int ny = rows;
    IO_LAUNCH(k_fields, sim, sw, y0, rho, ux, uy);
}
hipError_t launch_get_pop(bool f64, const SimDev* sim, int nx, int ny, int sw, double* f, hipStream_t stream) {
    IO_LAUNCH(k_get_pop, sim, sw, f);
}
hipError_t launch_set_pop(bool f64, const SimDev* sim, int nx, int ny, int sw, const double* f,
                          hipStream_t stream) {
    IO_LAUNCH(k_set_pop, sim, sw, f);
}
hipError_t launch_set_eq(bool f64, const SimDev* sim, int nx, int ny, int sw, const double* rho, const double* ux,
                         const double* uy, double rho0, double u0x, double u0y, hipStream_t stream) {
    IO_LAUNCH(k_set_eq, sim, sw, rho, ux, uy, rho0, u0x, u0y);
}

}  // namespace lbmib

// ---------------------------------------------------------------- static staging

// Device staging of lbm_fields_noalloc, for callers that cannot allocate:
// kStaticScratchDoubles doubles on every device the library runs on, held
// until the process ends.  Host code never uses the array's name as an
// address: static_scratch() takes the device address once per device with
// hipGetSymbolAddress and hands out that pointer.
static __device__ __align__(256) double scratch[lbmib::kStaticScratchDoubles];

namespace lbmib {

hipError_t static_scratch(double** out) {
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace lbmib

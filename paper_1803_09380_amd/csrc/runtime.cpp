// Host runtime and C ABI of the gfx950 IB-LBM library (declared in include/lbmib.h).
//
// A simulation owns its device state: the nine population planes with a ghost
// layer (see lbm_device.hpp), a one-entry descriptor table, its body and
// marker arrays, the work tables of its own steps (sweep tiles, boundary
// chunks, body groups) and each group's plan and scratch.  Plans of groups
// without free bodies are built here once, when markers are set; groups with
// free bodies rebuild theirs on the device every step.  A batch concatenates
// the work tables of its admitted simulations into device-resident tables and
// replays captured HIP graphs of kernels that read their work counts from
// those tables (one workgroup per sweep tile, persistent workgroups for the
// boundary chunks and body groups).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <utility>
#include <string>
#include <vector>

#include "../../include/lbmib.h"
#include "kernels.hpp"

using namespace lbmib;

namespace {

// 64 x 4 threads, one row each, non-temporal: the fastest tiling for the served
// mix of 400-wide requests (0.211 against 0.229 ms per step for 256 x 1 threads
// with two rows each) and often the autotuner's pick for the batched set
constexpr int kTileDefault = 8;

template <typename... A>
std::string fmt(const char* f, A... a) {
    char buf[512];
    snprintf(buf, sizeof buf, f, a...);
    return buf;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t alloc(size_t n) {
        release();
        if (n == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = n;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};

struct HostBody {
    bool used = false;
    int kind = 0, n = 0;
    std::vector<double> X, Y, U, V, ds;
    ib_body b{};
};

// One group's plan and scratch on the device plus its host descriptor.
struct Group {
    GroupDev d{};
    DevBuf node_cell, node_run, ent, mnode, flags, node4, ent_D, m_phi, m_wtot, m_rows, m_red, cord, coff;
};

}  // namespace

struct lbm_sim {
    lbm_params p{};
    bool f64 = true;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    DevBuf pop, desc, status, bodies, markers, tiles, bcitems, groups, ubound, chunks;
    SimDev h{};                // host mirror of the descriptor
    HostBody body[LBM_MAX_BODIES];
    std::vector<Group*> grp;
    std::vector<int4> h_tiles;
    std::vector<int2> h_bc;
    std::vector<int2> h_chunks;  // band chunks (group, first node)
    int tiling = kTileDefault;
    int64_t steps = 0;
    int mcount = 0;
    int max_group = 0;  // markers of the largest body group
    // some band node lies within three nodes of a non-periodic side (or a band
    // is rebuilt on the device): the boundary rules and the correction may
    // touch the same populations, so they run in order
    bool band_near_edge = false;
    lbm_batch* batch = nullptr;
    ~lbm_sim() {
        for (Group* g : grp) delete g;
    }
};

// One lane of a batch: the work tables of a subset of its simulations
// (contiguous in the batch's simulation table), replayed on its own stream.
struct Lane {
    DevBuf d_tiles, d_bc, d_groups, d_hdr, d_chunks;
    size_t cap_tiles = 0, cap_bc = 0, cap_groups = 0, cap_chunks = 0;
    int sim0 = 0, nsims = 0, ntiles = 0, nbc = 0, ngroups = 0, nchunks = 0;
    int max_group = 0;
    int grid_sweep = 0, grid_band = 0;
    bool mrt = false;  // some simulation of the lane uses the MRT collision
    // the correction launch applies the boundary rules too (boundary items, body
    // groups, and no band within three nodes of a non-periodic side)
    bool bnd_in_ib = false;
    hipGraphExec_t graph1 = nullptr, graphK = nullptr;
    hipGraphExec_t graphA = nullptr, graphB = nullptr;  // one step split: the sweep, the rest (run_interleaved)
    void drop() {
        for (hipGraphExec_t* g : {&graph1, &graphK, &graphA, &graphB}) {
            if (*g) (void)hipGraphExecDestroy(*g);
            *g = nullptr;
        }
    }
};

// Simulations whose largest body group has more markers than this run in the
// first lane when the batch uses two: their long correction kernels run while
// the other lane's lighter work does (between its two sweep launches when the
// lanes are interleaved).
constexpr int kHeavyGroupMarkers = 400;
// Fixed plans of at most this many band nodes are gathered and applied by
// their correction workgroup; larger ones by the band kernels over all CUs (a
// node's nine populations lie in nine cache lines, which one CU fetches at a
// fraction of the chip's rate: 5,000 nodes took 50 us each way in one
// workgroup against a few us spread over the chip), except in interleaved
// FP32 lanes, where the correction runs beside a sweep and takes every band.
constexpr int kFuseBandNodes = 1024;
// Two interleaved lanes are launched step by step from the host; below this
// many nodes the automatic choice replays each lane's graphs of several steps
// independently instead.
constexpr int64_t kInterleaveMinCells = 16 << 20;

struct lbm_batch {
    bool f64 = false;
    size_t budget = 0;
    int device = 0;
    hipStream_t stream = nullptr;   // the caller's (or an own) stream: lane 0
    bool own_stream = false;
    hipStream_t stream2 = nullptr;  // lane 1, owned
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_sweep0 = nullptr, ev_sweep1 = nullptr;  // lane 0's, lane 1's sweep of the current step is done
    std::vector<lbm_sim*> sims;
    std::vector<int> order;         // simulation table row -> index into sims
    DevBuf d_sims;
    size_t cap_sims = 0;
    DevBuf d_probe;                 // two flags of the hardware-queue check (ensure_lane_stream)
    int lanes_concurrent = -1;      // the second stream was seen running beside the batch stream (-1: not made)
    Lane lane[2];
    int lanes_req = 0;              // 0 automatic, 1 one lane, 2 two free-running, 3 two interleaved,
                                    // 4 two interleaved halves of equal node count (upload_tables)
    bool interleave = false;        // two lanes in use are interleaved step by step
    int nlanes = 1;                 // lanes in use
    int tiling = kTileDefault;
    int grid_bc = 0, grid_ib = 0;
    int graphK_steps = 8;
    size_t bytes = 0;
    std::string err;
    ~lbm_batch() {
        lane[0].drop();
        lane[1].drop();
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (ev_sweep0) (void)hipEventDestroy(ev_sweep0);
        if (ev_sweep1) (void)hipEventDestroy(ev_sweep1);
        if (stream2) (void)hipStreamDestroy(stream2);
    }
};

namespace {

lbm_status fail(lbm_sim* s, lbm_status st, const std::string& msg) {
    if (s) s->err = msg;
    return st;
}
lbm_status failb(lbm_batch* b, lbm_status st, const std::string& msg) {
    if (b) b->err = msg;
    return st;
}
lbm_status hipfail(lbm_sim* s, hipError_t e, const char* where) {
    return fail(s, e == hipErrorOutOfMemory ? LBM_ERR_NOMEM : LBM_ERR_DEVICE,
                fmt("%s: %s", where, hipGetErrorString(e)));
}

#define HIPS(s, call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hipfail(s, e_, #call); \
    } while (0)

int num_cus(int dev) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    return n;
}

bool bc_valid(const lbm_params* p) {
    const int nd = (p->bc_west == LBM_BC_DIRICHLET) + (p->bc_east == LBM_BC_DIRICHLET) +
                   (p->bc_south == LBM_BC_DIRICHLET) + (p->bc_north == LBM_BC_DIRICHLET);
    if (nd == 4) return p->nx >= 4 && p->ny >= 4;
    if (nd != 0) return false;
    auto ok = [](int v) { return v >= LBM_BC_PERIODIC && v <= LBM_BC_PRESSURE; };
    if (!ok(p->bc_west) || !ok(p->bc_east) || !ok(p->bc_south) || !ok(p->bc_north)) return false;
    if ((p->bc_west == LBM_BC_PERIODIC) != (p->bc_east == LBM_BC_PERIODIC)) return false;
    if ((p->bc_south == LBM_BC_PERIODIC) != (p->bc_north == LBM_BC_PERIODIC)) return false;
    if (p->bc_west == LBM_BC_FREESLIP || p->bc_west == LBM_BC_OUTFLOW || p->bc_west == LBM_BC_PRESSURE)
        return false;
    if (p->bc_east == LBM_BC_PRESSURE && p->nx < 5) return false;
    if (p->bc_east == LBM_BC_FREESLIP || p->bc_east == LBM_BC_VELOCITY) return false;
    if (p->bc_south == LBM_BC_VELOCITY || p->bc_south == LBM_BC_OUTFLOW || p->bc_south == LBM_BC_PRESSURE)
        return false;
    if (p->bc_north == LBM_BC_VELOCITY || p->bc_north == LBM_BC_OUTFLOW || p->bc_north == LBM_BC_PRESSURE)
        return false;
    return true;
}

// Boundary nodes the boundary kernel rebuilds every step: the whole perimeter
// of a prescribed-velocity box (2 nx + 2 (ny - 2) nodes, in the order of
// lbm_set_boundary_velocity), else the inlet column and the outlet column.
// Walls and free-slip sides need no kernel: the sweep applies their rules.
int boundary_count(const SimDev& h) {
    if (h.bc[SIDE_W] == BC_DIRICHLET) return 2 * h.nx + 2 * (h.ny - 2);
    int n = 0;
    if (h.bc[SIDE_W] == BC_VELOCITY) n += h.ny;
    if (h.bc[SIDE_E] == BC_OUTFLOW || h.bc[SIDE_E] == BC_PRESSURE) n += h.ny;
    return n;
}

// Sweep tiles of one simulation: (sim, x0, y0) for rectangular tilings;
// (sim, first block, row of that block) for block tilings (tx = 0), whose
// tiles are ty * rpt consecutive blocks of kBlk nodes in row-major order.
// The third field is the row the tile starts in either way.
void build_tiles(lbm_sim* s, int sim_index, int tiling, std::vector<int4>& out) {
    const Tiling& t = kTilings[tiling];
    if (t.tx == 0) {
        const int nbx = (s->p.nx + kBlk - 1) / kBlk, nb = nbx * s->p.ny, per = t.ty * t.rpt;
        for (int k0 = 0; k0 < nb; k0 += per) out.push_back(make_int4(sim_index, k0, k0 / nbx, 0));
        return;
    }
    const int th = t.ty * t.rpt;
    for (int y0 = 0; y0 < s->p.ny; y0 += th)
        for (int x0 = 0; x0 < s->p.nx; x0 += t.tx) out.push_back(make_int4(sim_index, x0, y0, 0));
}

// Chunks of 256 band nodes of one group for the band kernels: the groups
// whose correction workgroup does not gather and apply its band itself.
void build_chunks(const GroupDev& d, int group_index, std::vector<int2>& out) {
    if (d.in_kernel) return;
    for (int k = 0; k < d.nband; k += 256) out.push_back(make_int2(group_index, k));
}

void build_bc(lbm_sim* s, int sim_index, std::vector<int2>& out) {
    for (int k = 0; k < s->h.nperim; k += 256) out.push_back(make_int2(sim_index, k));
}

bool stencil_cell_host(const SimDev& S, double X, double Y, int kx, int ky, int& cell) {
    int x = (int)std::floor(X) - 1 + kx, y = (int)std::floor(Y) - 1 + ky;
    if (S.px) x = x < 0 ? x + S.nx : (x >= S.nx ? x - S.nx : x);
    if (S.py) y = y < 0 ? y + S.ny : (y >= S.ny ? y - S.ny : y);
    if (x < 0 || x >= S.nx || y < 0 || y >= S.ny) return false;
    cell = y * S.nx + x;
    return true;
}

// The domain a marker may occupy: on a non-periodic axis the lattice is
// closed half a spacing outside its first and last nodes (where half-way
// bounce-back places the wall, Fig. 2), so -1/2 <= X <= n - 1/2; on a
// periodic axis, one period, 0 <= X < n.  A free circle must fit whole
// (centre +- radius) on non-periodic axes, since its markers move on it.
bool markers_inside(const SimDev& h, const HostBody& B) {
    auto axis_ok = [](double v, double lo_pad, int n, bool periodic) {
        if (periodic) return v >= 0.0 && v < (double)n;
        return v - lo_pad >= -0.5 && v + lo_pad <= (double)n - 0.5;
    };
    if (B.kind == IB_FREE) {
        const double R = B.b.radius;
        return axis_ok(B.b.xc[0], h.px ? 0.0 : R, h.nx, h.px) && axis_ok(B.b.xc[1], h.py ? 0.0 : R, h.ny, h.py);
    }
    for (int l = 0; l < B.n; ++l)
        if (!axis_ok(B.X[l], 0.0, h.nx, h.px) || !axis_ok(B.Y[l], 0.0, h.ny, h.py)) return false;
    return true;
}

std::vector<int> body_cells(const lbm_sim* s, int b) {
    std::vector<int> c;
    const HostBody& B = s->body[b];
    for (int l = 0; l < B.n; ++l)
        for (int k = 0; k < 16; ++k) {
            int cell;
            if (stencil_cell_host(s->h, B.X[l], B.Y[l], k & 3, k >> 2, cell)) c.push_back(cell);
        }
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    return c;
}

template <typename V>
hipError_t upload(DevBuf& buf, const std::vector<V>& v, hipStream_t st) {
    hipError_t e = buf.alloc(std::max<size_t>(1, v.size()) * sizeof(V));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st);
}

// (Re)build bodies, markers and groups of a simulation after a marker change.
lbm_status rebuild_ib(lbm_sim* s) {
    hipStream_t st = s->stream;
    // markers of all bodies, concatenated in slot order
    std::vector<double> arr[5];
    std::vector<BodyDev> bd(LBM_MAX_BODIES);
    int m = 0, nbody = 0;
    bool any_free = false;
    for (int b = 0; b < LBM_MAX_BODIES; ++b) {
        BodyDev& d = bd[b];
        memset(&d, 0, sizeof d);
        const HostBody& B = s->body[b];
        if (!B.used) continue;
        ++nbody;
        d.used = 1;
        d.kind = B.kind;
        d.n = B.n;
        d.m0 = m;
        d.xc[0] = B.b.xc[0];
        d.xc[1] = B.b.xc[1];
        d.U[0] = B.b.U[0];
        d.U[1] = B.b.U[1];
        d.omega = B.b.omega;
        d.theta = B.b.theta;
        d.R = B.b.radius;
        d.rho_s = B.b.rho_s;
        d.Uprev[0] = d.U[0];
        d.Uprev[1] = d.U[1];
        d.omega_prev = d.omega;
        any_free |= B.kind == IB_FREE;
        for (int l = 0; l < B.n; ++l) {
            arr[0].push_back(B.X[l]);
            arr[1].push_back(B.Y[l]);
            arr[2].push_back(B.U[l]);
            arr[3].push_back(B.V[l]);
            arr[4].push_back(B.ds[l]);
        }
        m += B.n;
    }
    s->mcount = m;
    HIPS(s, s->bodies.alloc(sizeof(BodyDev) * LBM_MAX_BODIES));
    HIPS(s, hipMemcpyAsync(s->bodies.p, bd.data(), sizeof(BodyDev) * LBM_MAX_BODIES, hipMemcpyHostToDevice, st));
    HIPS(s, s->markers.alloc(sizeof(double) * 5 * std::max(1, m)));
    double* mk = static_cast<double*>(s->markers.p);
    for (int a = 0; a < 5; ++a)
        if (m) HIPS(s, hipMemcpyAsync(mk + (size_t)a * m, arr[a].data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    s->h.bodies = static_cast<BodyDev*>(s->bodies.p);
    s->h.mX = mk;
    s->h.mY = mk + m;
    s->h.mU = mk + 2 * (size_t)m;
    s->h.mV = mk + 3 * (size_t)m;
    s->h.mds = mk + 4 * (size_t)m;
    s->h.nbody = nbody;

    // groups: all bodies together when one is free, else by shared stencil nodes
    std::vector<std::vector<int>> groups;
    if (any_free) {
        std::vector<int> all;
        for (int b = 0; b < LBM_MAX_BODIES; ++b)
            if (s->body[b].used) all.push_back(b);
        groups.push_back(all);
    } else {
        std::vector<std::vector<int>> cells(LBM_MAX_BODIES);
        std::vector<int> parent(LBM_MAX_BODIES);
        std::iota(parent.begin(), parent.end(), 0);
        auto find = [&](int a) {
            while (parent[a] != a) a = parent[a] = parent[parent[a]];
            return a;
        };
        for (int b = 0; b < LBM_MAX_BODIES; ++b)
            if (s->body[b].used) cells[b] = body_cells(s, b);
        for (int a = 0; a < LBM_MAX_BODIES; ++a)
            for (int b = a + 1; b < LBM_MAX_BODIES; ++b) {
                if (!s->body[a].used || !s->body[b].used) continue;
                std::vector<int> both;
                std::set_intersection(cells[a].begin(), cells[a].end(), cells[b].begin(), cells[b].end(),
                                      std::back_inserter(both));
                if (!both.empty()) parent[find(a)] = find(b);
            }
        for (int b = 0; b < LBM_MAX_BODIES; ++b) {
            if (!s->body[b].used) continue;
            bool placed = false;
            for (auto& g : groups)
                if (find(g[0]) == find(b)) {
                    g.push_back(b);
                    placed = true;
                    break;
                }
            if (!placed) groups.push_back({b});
        }
    }
    for (Group* g : s->grp) delete g;
    s->grp.clear();
    const size_t tsz = s->f64 ? sizeof(double) : sizeof(float);
    s->band_near_edge = false;
    for (auto& members : groups) {
        Group* G = new (std::nothrow) Group();
        if (!G) return fail(s, LBM_ERR_NOMEM, "host allocation");
        s->grp.push_back(G);
        GroupDev& d = G->d;
        d.sim = 0;
        d.nbody = (int)members.size();
        int M = 0;
        for (int k = 0; k < d.nbody; ++k) {
            d.body[k] = members[k];
            M += s->body[members[k]].n;
        }
        d.M = M;
        d.dynamic = any_free ? 1 : 0;
        if (M > kMaxGroupMarkers) return fail(s, LBM_ERR_INVALID, "too many markers in one body group");
        if (d.dynamic && 16 * M > kMaxDynEntries)
            return fail(s, LBM_ERR_INVALID, "too many markers in a simulation with free bodies");
        d.cap_ent = 16 * M;
        int nband = 16 * M;
        std::vector<int> node_cell, node_run, ent, mnode(16 * (size_t)M, -1);
        if (!d.dynamic) {
            // same definition as the device build: entries sorted by cell, then marker
            std::vector<unsigned long long> keys;
            int g = 0;
            for (int b : members) {
                const HostBody& B = s->body[b];
                for (int l = 0; l < B.n; ++l, ++g)
                    for (int k = 0; k < 16; ++k) {
                        int cell;
                        if (stencil_cell_host(s->h, B.X[l], B.Y[l], k & 3, k >> 2, cell))
                            keys.push_back(((unsigned long long)(unsigned)cell << 32) | (unsigned)((g << 4) | k));
                    }
            }
            std::sort(keys.begin(), keys.end());
            for (size_t e = 0; e < keys.size(); ++e) {
                const int cell = (int)(keys[e] >> 32), low = (int)(keys[e] & 0xffffffffu);
                if (e == 0 || (keys[e - 1] >> 32) != (keys[e] >> 32)) {
                    node_cell.push_back(cell);
                    node_run.push_back((int)e);
                }
                ent.push_back(low);
                mnode[low] = (int)node_cell.size() - 1;
            }
            node_run.push_back((int)ent.size());
            nband = (int)node_cell.size();
            d.nband = nband;
            d.nent = (int)ent.size();
            const int nx = s->h.nx, ny = s->h.ny;
            for (int c : node_cell) {
                const int x = c % nx, y = c / nx;
                if ((!s->h.px && (x < 3 || x > nx - 4)) || (!s->h.py && (y < 3 || y > ny - 4))) s->band_near_edge = true;
            }
        } else {
            s->band_near_edge = true;
        }
        // colour classes: every stencil row four consecutive band nodes; two
        // markers conflict when their stencils share a band node; greedy
        // colouring in marker order
        std::vector<unsigned short> cord;
        std::vector<int> coff;
        if (!d.dynamic && M > 0 && M <= 0xFFFF && nband < 0xFFFF) {
            bool regular = true;
            for (int g = 0; g < M && regular; ++g)
                for (int ky = 0; ky < 4; ++ky) {
                    const int* m = &mnode[16 * (size_t)g + 4 * ky];
                    if (m[0] < 0 || m[1] != m[0] + 1 || m[2] != m[0] + 2 || m[3] != m[0] + 3) {
                        regular = false;
                        break;
                    }
                }
            if (regular) {
                std::vector<int> color(M, -1);
                int ncolor = 0;
                for (int g = 0; g < M && ncolor <= kMaxColors; ++g) {
                    unsigned long long used = 0;
                    for (int k = 0; k < 16; ++k) {
                        const int nd = mnode[16 * (size_t)g + k];
                        for (int e = node_run[nd]; e < node_run[nd + 1]; ++e) {
                            const int o = ent[e] >> 4;
                            if (o != g && color[o] >= 0) used |= 1ull << color[o];
                        }
                    }
                    int c = 0;
                    while (c < 64 && (used >> c & 1ull)) ++c;
                    color[g] = c;
                    ncolor = std::max(ncolor, c + 1);
                }
                if (ncolor <= kMaxColors) {
                    coff.assign(ncolor + 1, 0);
                    for (int g = 0; g < M; ++g) ++coff[color[g] + 1];
                    for (int c = 0; c < ncolor; ++c) coff[c + 1] += coff[c];
                    cord.assign(2 * (size_t)M, 0);  // marker at each position, then position of each marker
                    std::vector<int> fill(coff.begin(), coff.end() - 1);
                    for (int g = 0; g < M; ++g) {
                        const int pos = fill[color[g]]++;
                        cord[pos] = (unsigned short)g;
                        cord[M + g] = (unsigned short)pos;
                    }
                }
            }
        }
        d.ncolor = cord.empty() ? 0 : (int)coff.size() - 1;
        d.in_kernel = d.dynamic || nband <= kFuseBandNodes ? 1 : 0;
        d.cap_nodes = std::max(1, nband);
        HIPS(s, G->node_cell.alloc(sizeof(int) * d.cap_nodes));
        HIPS(s, G->node_run.alloc(sizeof(int) * (d.cap_nodes + 1)));
        HIPS(s, G->ent.alloc(sizeof(int) * std::max(1, d.cap_ent)));
        HIPS(s, G->mnode.alloc(sizeof(int) * std::max(1, 16 * M)));
        HIPS(s, G->flags.alloc(sizeof(int) * 4));
        HIPS(s, hipMemsetAsync(G->flags.p, 0, sizeof(int) * 4, st));
        HIPS(s, G->node4.alloc(tsz * 4 * d.cap_nodes));
        HIPS(s, G->ent_D.alloc(2 * tsz * std::max(1, d.cap_ent)));
        HIPS(s, G->m_phi.alloc(tsz * 8 * std::max(1, M)));
        HIPS(s, G->m_wtot.alloc(tsz * 5 * std::max(1, M)));
        HIPS(s, G->m_rows.alloc(sizeof(unsigned short) * 4 * std::max(1, M)));
        HIPS(s, G->m_red.alloc(sizeof(double) * 5 * std::max(1, M)));
        if (d.ncolor) {
            HIPS(s, G->cord.alloc(sizeof(unsigned short) * cord.size()));
            HIPS(s, G->coff.alloc(sizeof(int) * coff.size()));
        }
        d.node_cell = (int*)G->node_cell.p;
        d.node_run = (int*)G->node_run.p;
        d.ent = (int*)G->ent.p;
        d.mnode = (int*)G->mnode.p;
        d.flags = (int*)G->flags.p;
        d.node4 = G->node4.p;
        d.ent_D = G->ent_D.p;
        d.m_phi = G->m_phi.p;
        d.m_wtot = G->m_wtot.p;
        d.m_rows = (unsigned short*)G->m_rows.p;
        d.m_red = (double*)G->m_red.p;
        d.cord = (unsigned short*)G->cord.p;
        d.coff = (int*)G->coff.p;
        if (!d.dynamic) {
            HIPS(s, hipMemcpyAsync(d.node_cell, node_cell.data(), sizeof(int) * node_cell.size(), hipMemcpyHostToDevice, st));
            HIPS(s, hipMemcpyAsync(d.node_run, node_run.data(), sizeof(int) * node_run.size(), hipMemcpyHostToDevice, st));
            if (!ent.empty())
                HIPS(s, hipMemcpyAsync(d.ent, ent.data(), sizeof(int) * ent.size(), hipMemcpyHostToDevice, st));
            if (M) HIPS(s, hipMemcpyAsync(d.mnode, mnode.data(), sizeof(int) * mnode.size(), hipMemcpyHostToDevice, st));
            if (d.ncolor) {
                HIPS(s, hipMemcpyAsync(d.cord, cord.data(), sizeof(unsigned short) * cord.size(), hipMemcpyHostToDevice, st));
                HIPS(s, hipMemcpyAsync(d.coff, coff.data(), sizeof(int) * coff.size(), hipMemcpyHostToDevice, st));
            }
        }
    }
    std::vector<GroupDev> gd;
    s->max_group = 0;
    for (Group* g : s->grp) {
        gd.push_back(g->d);
        s->max_group = std::max(s->max_group, g->d.M);
    }
    HIPS(s, upload(s->groups, gd, st));
    s->h_chunks.clear();
    for (size_t gi = 0; gi < gd.size(); ++gi) build_chunks(gd[gi], (int)gi, s->h_chunks);
    HIPS(s, upload(s->chunks, s->h_chunks, st));
    HIPS(s, hipMemcpyAsync(s->desc.p, &s->h, sizeof(SimDev), hipMemcpyHostToDevice, st));
    HIPS(s, hipStreamSynchronize(st));
    return LBM_OK;
}

lbm_status sync_back(lbm_batch* b);

// A simulation inside a batch has its step state in the batch's device table.
lbm_status refresh(lbm_sim* s) {
    if (!s->batch) return LBM_OK;
    lbm_status rc = sync_back(s->batch);
    if (rc != LBM_OK) return fail(s, rc, "could not read the batch state");
    return LBM_OK;
}

lbm_status check_status(lbm_sim* s) {
    uint32_t st = 0;
    HIPS(s, hipMemcpyAsync(&st, s->status.p, sizeof st, hipMemcpyDeviceToHost, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    if (st & ST_UNSTABLE) return fail(s, LBM_ERR_UNSTABLE, "a density went non-positive or non-finite");
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_version(void) { return "lbmib-gfx950 0.1"; }

lbm_status lbm_create(const lbm_params* p, void* hip_stream, lbm_sim** out) {
    if (!out) return LBM_ERR_INVALID;
    *out = nullptr;
    if (!p || p->nx < 4 || p->ny < 4 || !(p->tau > 0.5) || p->ib_iters < 0 || p->ib_iters > 1000 ||
        !(p->rho0 > 0) || (p->precision != LBM_F64 && p->precision != LBM_F32_SHIFTED) || !bc_valid(p) ||
        (p->collision != LBM_BGK && p->collision != LBM_MRT) ||
        (p->delta != 0 && p->delta != 2 && p->delta != 3 && p->delta != 4) ||
        (int64_t)p->nx * p->ny > (int64_t)1 << 30)
        return LBM_ERR_INVALID;
    lbm_sim* s = new (std::nothrow) lbm_sim();
    if (!s) return LBM_ERR_NOMEM;
    s->p = *p;
    s->f64 = p->precision == LBM_F64;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return LBM_ERR_DEVICE;
    }
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) {
            delete s;
            return LBM_ERR_DEVICE;
        }
        s->own_stream = true;
    }
    const int esz = s->f64 ? 8 : 4;
    SimDev& h = s->h;
    memset(&h, 0, sizeof h);
    h.nblk = blocks_per_row(p->nx);
    h.rstride = (int64_t)h.nblk * Q * kBlk;
    h.nx = p->nx;
    h.ny = p->ny;
    h.bc[0] = p->bc_west;
    h.bc[1] = p->bc_east;
    h.bc[2] = p->bc_south;
    h.bc[3] = p->bc_north;
    h.px = p->bc_west == LBM_BC_PERIODIC;
    h.py = p->bc_south == LBM_BC_PERIODIC;
    h.omega = 1.0 / p->tau;
    h.rho0 = p->rho0;
    h.rho_base = s->f64 ? 0.0 : p->rho0;
    h.u_in[0] = p->u_in[0];
    h.u_in[1] = p->u_in[1];
    h.gravity[0] = p->gravity[0];
    h.gravity[1] = p->gravity[1];
    h.collision = p->collision;
    h.delta = p->delta == 0 ? 4 : p->delta;
    for (int k = 0; k < 9; ++k) h.mrt_s[k] = p->collision == LBM_MRT ? p->mrt_s[k] : 1.0 / p->tau;
    h.swapped = 0;
    h.active = 1;
    h.steps_left = -1;
    h.ib_iters = p->ib_iters;
    h.nperim = boundary_count(h);
    for (int side = 0; side < 4; ++side)
        if (h.bc[side] == BC_WALL || h.bc[side] == BC_FREESLIP) h.edges |= 1 << side;
    lbm_status rc = LBM_OK;
    auto bail = [&](lbm_status e) {
        lbm_destroy(s);
        return e;
    };
    if (s->pop.alloc((size_t)h.rstride * (p->ny + 2) * esz) != hipSuccess) return bail(LBM_ERR_NOMEM);
    if (s->desc.alloc(sizeof(SimDev)) != hipSuccess || s->status.alloc(sizeof(uint32_t)) != hipSuccess)
        return bail(LBM_ERR_NOMEM);
    if (hipMemsetAsync(s->pop.p, 0, s->pop.bytes, s->stream) != hipSuccess ||
        hipMemsetAsync(s->status.p, 0, sizeof(uint32_t), s->stream) != hipSuccess)
        return bail(LBM_ERR_DEVICE);
    h.pop = s->pop.p;
    h.status = (uint32_t*)s->status.p;
    if (p->bc_west == LBM_BC_DIRICHLET) {
        if (s->ubound.alloc(sizeof(double) * 2 * h.nperim) != hipSuccess) return bail(LBM_ERR_NOMEM);
        if (hipMemsetAsync(s->ubound.p, 0, s->ubound.bytes, s->stream) != hipSuccess) return bail(LBM_ERR_DEVICE);
        h.ubound = static_cast<const double*>(s->ubound.p);
    }
    rc = rebuild_ib(s);
    if (rc != LBM_OK) return bail(rc);
    build_tiles(s, 0, s->tiling, s->h_tiles);
    build_bc(s, 0, s->h_bc);
    if (upload(s->tiles, s->h_tiles, s->stream) != hipSuccess || upload(s->bcitems, s->h_bc, s->stream) != hipSuccess)
        return bail(LBM_ERR_NOMEM);
    if (launch_set_eq(s->f64, (const SimDev*)s->desc.p, p->nx, p->ny, 0, nullptr, nullptr, nullptr, p->rho0,
                      p->u_init[0], p->u_init[1], s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return bail(LBM_ERR_DEVICE);
    *out = s;
    return LBM_OK;
}

void lbm_destroy(lbm_sim* s) {
    if (!s) return;
    if (s->batch) lbm_batch_retire(s->batch, s);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    bool own = s->own_stream;
    hipStream_t st = s->stream;
    delete s;
    if (own && st) (void)hipStreamDestroy(st);
}

const char* lbm_last_error(const lbm_sim* s) { return s ? s->err.c_str() : "null handle"; }

lbm_status ib_set_markers(lbm_sim* s, int32_t id, int32_t n, const double* xy, const double* uv,
                          const double* ds, const ib_body* body) {
    if (!s) return LBM_ERR_INVALID;
    if (s->batch) return fail(s, LBM_ERR_STATE, "markers cannot change while the simulation is in a batch");
    if (id < 0 || id >= LBM_MAX_BODIES || n < 0) return fail(s, LBM_ERR_INVALID, "bad body id or count");
    HostBody old = s->body[id];
    HostBody& B = s->body[id];
    if (n == 0) {
        B = HostBody();
    } else {
        if (!body) return fail(s, LBM_ERR_INVALID, "body descriptor required");
        HostBody nb;
        nb.used = true;
        nb.kind = body->kind;
        nb.n = n;
        nb.b = *body;
        nb.X.resize(n);
        nb.Y.resize(n);
        nb.U.resize(n);
        nb.V.resize(n);
        nb.ds.resize(n);
        if (body->kind == IB_FREE) {
            if (xy || uv || ds || !(body->radius > 0) || !(body->rho_s > 0))
                return fail(s, LBM_ERR_INVALID, "free bodies take radius and density, not marker arrays");
            for (int l = 0; l < n; ++l) {
                const double a = 2.0 * M_PI * l / n + body->theta;
                nb.X[l] = body->xc[0] + body->radius * std::cos(a);
                nb.Y[l] = body->xc[1] + body->radius * std::sin(a);
                nb.U[l] = body->U[0] - body->omega * (nb.Y[l] - body->xc[1]);
                nb.V[l] = body->U[1] + body->omega * (nb.X[l] - body->xc[0]);
                nb.ds[l] = 2.0 * M_PI * body->radius / n;
            }
        } else if (body->kind == IB_FIXED) {
            if (!xy) return fail(s, LBM_ERR_INVALID, "fixed bodies need marker positions");
            for (int l = 0; l < n; ++l) {
                nb.X[l] = xy[2 * l];
                nb.Y[l] = xy[2 * l + 1];
                if (!std::isfinite(nb.X[l]) || !std::isfinite(nb.Y[l]))
                    return fail(s, LBM_ERR_INVALID, "non-finite marker position");
            }
            for (int l = 0; l < n; ++l) {
                if (uv) {
                    nb.U[l] = uv[2 * l];
                    nb.V[l] = uv[2 * l + 1];
                } else {
                    nb.U[l] = body->U[0] - body->omega * (nb.Y[l] - body->xc[1]);
                    nb.V[l] = body->U[1] + body->omega * (nb.X[l] - body->xc[0]);
                }
                if (ds) {
                    nb.ds[l] = ds[l];
                } else {
                    const int a = (l + n - 1) % n, c = (l + 1) % n;
                    nb.ds[l] = 0.5 * (std::hypot(nb.X[l] - nb.X[a], nb.Y[l] - nb.Y[a]) +
                                      std::hypot(nb.X[c] - nb.X[l], nb.Y[c] - nb.Y[l]));
                }
            }
        } else {
            return fail(s, LBM_ERR_INVALID, "unknown body kind");
        }
        if (!markers_inside(s->h, nb))
            return fail(s, LBM_ERR_INVALID, "a marker lies outside the lattice (beyond a non-periodic side, "
                                            "or outside one period of a periodic axis)");
        B = nb;
    }
    lbm_status rc = rebuild_ib(s);
    if (rc != LBM_OK) {
        s->body[id] = old;
        std::string msg = s->err;
        (void)rebuild_ib(s);
        s->err = msg;
    }
    return rc;
}

lbm_status lbm_set_boundary_velocity(lbm_sim* s, const double* ub) {
    if (!s || !ub) return LBM_ERR_INVALID;
    if (!s->ubound.p) return fail(s, LBM_ERR_INVALID, "not a prescribed-velocity box");
    if (s->batch) return fail(s, LBM_ERR_STATE, "boundary velocities cannot change while in a batch");
    HIPS(s, hipMemcpyAsync(s->ubound.p, ub, s->ubound.bytes, hipMemcpyHostToDevice, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status ib_set_marker_velocities(lbm_sim* s, int32_t id, const double* uv) {
    if (!s || !uv || id < 0 || id >= LBM_MAX_BODIES) return LBM_ERR_INVALID;
    HostBody& B = s->body[id];
    if (!B.used || B.kind != IB_FIXED) return fail(s, LBM_ERR_INVALID, "no such fixed body");
    if (s->batch) return fail(s, LBM_ERR_STATE, "markers cannot change while the simulation is in a batch");
    int m0 = 0;
    for (int b = 0; b < id; ++b)
        if (s->body[b].used) m0 += s->body[b].n;
    for (int l = 0; l < B.n; ++l) {
        B.U[l] = uv[2 * l];
        B.V[l] = uv[2 * l + 1];
    }
    HIPS(s, hipMemcpyAsync(s->h.mU + m0, B.U.data(), sizeof(double) * B.n, hipMemcpyHostToDevice, s->stream));
    HIPS(s, hipMemcpyAsync(s->h.mV + m0, B.V.data(), sizeof(double) * B.n, hipMemcpyHostToDevice, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_step(lbm_sim* s, int32_t nsteps) {
    if (!s || nsteps < 0) return LBM_ERR_INVALID;
    if (s->batch) return fail(s, LBM_ERR_STATE, "simulation is stepped by its batch");
    const SimDev* d = (const SimDev*)s->desc.p;
    const int ntiles = (int)s->h_tiles.size(), nbc = (int)s->h_bc.size(), ng = (int)s->grp.size();
    const int nch = (int)s->h_chunks.size();
    const GroupDev* gdev = (const GroupDev*)s->groups.p;
    const int2* ch = (const int2*)s->chunks.p;
    for (int t = 0; t < nsteps; ++t) {
        const int parity = s->h.swapped;
        HIPS(s, launch_sweep(s->f64, s->h.collision != 0, s->tiling, d, (const int4*)s->tiles.p, nullptr, ntiles, ntiles, parity, s->stream));
        if (nbc) HIPS(s, launch_boundary(s->f64, d, (const int2*)s->bcitems.p, nullptr, nbc, nbc, parity, s->stream));
        if (ng) {
            HIPS(s, launch_band(s->f64, false, d, gdev, ch, nullptr, nch, nch, parity, s->stream));
            HIPS(s, launch_ib(s->f64, s->max_group, d, (GroupDev*)s->groups.p, nullptr, ng, ng, parity, s->stream));
            HIPS(s, launch_band(s->f64, true, d, gdev, ch, nullptr, nch, nch, parity, s->stream));
        }
        s->h.swapped ^= 1;
        s->h.steps_done += 1;
        ++s->steps;
    }
    return LBM_OK;
}

lbm_status lbm_sync(lbm_sim* s) {
    if (!s) return LBM_ERR_INVALID;
    HIPS(s, hipStreamSynchronize(s->stream));
    return check_status(s);
}

int64_t lbm_step_count(lbm_sim* s) {
    if (!s) return -1;
    if (refresh(s) != LBM_OK) return -1;
    return s->steps;
}

lbm_status ib_forces(lbm_sim* s, int32_t id, double F[2], double* T, double diag[2], ib_body* state_out) {
    if (!s || id < 0 || id >= LBM_MAX_BODIES) return LBM_ERR_INVALID;
    {
        lbm_status rc_ = refresh(s);
        if (rc_ != LBM_OK) return rc_;
    }
    if (!s->body[id].used) return fail(s, LBM_ERR_INVALID, "no such body");
    BodyDev b;
    HIPS(s, hipMemcpyAsync(&b, (BodyDev*)s->bodies.p + id, sizeof b, hipMemcpyDeviceToHost, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    if (F) {
        F[0] = b.F[0];
        F[1] = b.F[1];
    }
    if (T) *T = b.T;
    if (diag) {
        diag[0] = b.resid;
        diag[1] = b.maxslip;
    }
    if (state_out) {
        *state_out = s->body[id].b;
        state_out->xc[0] = b.xc[0];
        state_out->xc[1] = b.xc[1];
        state_out->U[0] = b.U[0];
        state_out->U[1] = b.U[1];
        state_out->omega = b.omega;
        state_out->theta = b.theta;
    }
    return check_status(s);
}

lbm_status lbm_fields_device(lbm_sim* s, void* rho, void* ux, void* uy) {
    if (!s) return LBM_ERR_INVALID;
    {
        lbm_status rc_ = refresh(s);
        if (rc_ != LBM_OK) return rc_;
    }
    HIPS(s, launch_fields(s->f64, (const SimDev*)s->desc.p, s->p.nx, s->p.ny, s->h.swapped, (double*)rho,
                          (double*)ux, (double*)uy, s->stream));
    return LBM_OK;
}

lbm_status lbm_fields(lbm_sim* s, double* rho, double* ux, double* uy) {
    if (!s) return LBM_ERR_INVALID;
    {
        lbm_status rc_ = refresh(s);
        if (rc_ != LBM_OK) return rc_;
    }
    const size_t n = (size_t)s->p.nx * s->p.ny;
    DevBuf tmp;
    HIPS(s, tmp.alloc(3 * n * sizeof(double)));
    double* d = (double*)tmp.p;
    HIPS(s, launch_fields(s->f64, (const SimDev*)s->desc.p, s->p.nx, s->p.ny, s->h.swapped, d, d + n, d + 2 * n,
                          s->stream));
    if (rho) HIPS(s, hipMemcpyAsync(rho, d, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (ux) HIPS(s, hipMemcpyAsync(ux, d + n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (uy) HIPS(s, hipMemcpyAsync(uy, d + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    return check_status(s);
}

lbm_status lbm_fields_noalloc(lbm_sim* s, double* rho, double* ux, double* uy) {
    if (!s) return LBM_ERR_INVALID;
    {
        lbm_status rc_ = refresh(s);
        if (rc_ != LBM_OK) return rc_;
    }
    double* stage = nullptr;
    HIPS(s, static_scratch(&stage));
    const int nx = s->p.nx, ny = s->p.ny;
    const size_t per_row = 3 * (size_t)nx;
    if (per_row > kStaticScratchDoubles)
        return fail(s, LBM_ERR_INVALID, fmt("rows of %d nodes exceed the static staging buffer (at most %zu nodes per row)",
                                            nx, kStaticScratchDoubles / 3));
    const int rows = (int)std::min<size_t>((size_t)ny, kStaticScratchDoubles / per_row);
    // rows [y0, y0 + r) at a time: fields into the staging array, then to the
    // caller's arrays; the copies finish before the next chunk overwrites it
    for (int y0 = 0; y0 < ny; y0 += rows) {
        const int r = std::min(rows, ny - y0);
        const size_t n = (size_t)r * nx, off = (size_t)y0 * nx;
        HIPS(s, launch_fields_rows(s->f64, (const SimDev*)s->desc.p, nx, y0, r, s->h.swapped, stage, stage + n,
                                   stage + 2 * n, s->stream));
        if (rho) HIPS(s, hipMemcpyAsync(rho + off, stage, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        if (ux) HIPS(s, hipMemcpyAsync(ux + off, stage + n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        if (uy) HIPS(s, hipMemcpyAsync(uy + off, stage + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPS(s, hipStreamSynchronize(s->stream));
    }
    return check_status(s);
}

lbm_status lbm_get_populations(lbm_sim* s, double* f) {
    if (!s || !f) return LBM_ERR_INVALID;
    {
        lbm_status rc_ = refresh(s);
        if (rc_ != LBM_OK) return rc_;
    }
    const size_t n = (size_t)s->p.nx * s->p.ny * 9;
    DevBuf tmp;
    HIPS(s, tmp.alloc(n * sizeof(double)));
    HIPS(s, launch_get_pop(s->f64, (const SimDev*)s->desc.p, s->p.nx, s->p.ny, s->h.swapped, (double*)tmp.p,
                           s->stream));
    HIPS(s, hipMemcpyAsync(f, tmp.p, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_sim* s, const double* f) {
    if (!s || !f) return LBM_ERR_INVALID;
    if (s->batch) return fail(s, LBM_ERR_STATE, "simulation is in a batch");
    const size_t n = (size_t)s->p.nx * s->p.ny * 9;
    DevBuf tmp;
    HIPS(s, tmp.alloc(n * sizeof(double)));
    HIPS(s, hipMemcpyAsync(tmp.p, f, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPS(s, launch_set_pop(s->f64, (const SimDev*)s->desc.p, s->p.nx, s->p.ny, s->h.swapped, (const double*)tmp.p,
                           s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_set_fields(lbm_sim* s, const double* rho, const double* ux, const double* uy) {
    if (!s || !rho || !ux || !uy) return LBM_ERR_INVALID;
    if (s->batch) return fail(s, LBM_ERR_STATE, "simulation is in a batch");
    const size_t n = (size_t)s->p.nx * s->p.ny;
    DevBuf tmp;
    HIPS(s, tmp.alloc(3 * n * sizeof(double)));
    double* d = (double*)tmp.p;
    HIPS(s, hipMemcpyAsync(d, rho, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPS(s, hipMemcpyAsync(d + n, ux, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPS(s, hipMemcpyAsync(d + 2 * n, uy, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPS(s, launch_set_eq(s->f64, (const SimDev*)s->desc.p, s->p.nx, s->p.ny, s->h.swapped, d, d + n, d + 2 * n, 0,
                          0, 0, s->stream));
    HIPS(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

size_t lbm_device_bytes(const lbm_sim* s) {
    if (!s) return 0;
    size_t b = s->pop.bytes + s->desc.bytes + s->status.bytes + s->bodies.bytes + s->markers.bytes + s->tiles.bytes +
               s->bcitems.bytes + s->groups.bytes + s->ubound.bytes + s->chunks.bytes;
    for (const Group* g : s->grp)
        b += g->node_cell.bytes + g->node_run.bytes + g->ent.bytes + g->mnode.bytes + g->flags.bytes +
             g->node4.bytes + g->ent_D.bytes + g->m_phi.bytes +
             g->m_wtot.bytes + g->m_rows.bytes + g->m_red.bytes + g->cord.bytes + g->coff.bytes;
    return b;
}

// Mirrors the allocations of lbm_create, rebuild_ib and the per-simulation
// tables above, taking every plan at its largest size: a group of M markers
// has at most 16 M band nodes and stencil entries, and the groups partition
// the bodies, so per-group constants count once per body.
size_t lbm_device_bytes_bound(const lbm_params* p, int32_t nbodies, const int32_t* markers) {
    if (!p || p->nx < 1 || p->ny < 1 || nbodies < 0 || nbodies > LBM_MAX_BODIES || (nbodies > 0 && !markers))
        return 0;
    const size_t tsz = p->precision == LBM_F64 ? sizeof(double) : sizeof(float);
    SimDev h{};
    h.nx = p->nx;
    h.ny = p->ny;
    h.bc[SIDE_W] = p->bc_west;
    h.bc[SIDE_E] = p->bc_east;
    h.bc[SIDE_S] = p->bc_south;
    h.bc[SIDE_N] = p->bc_north;
    const size_t nperim = (size_t)boundary_count(h);
    size_t b = (size_t)blocks_per_row(p->nx) * Q * kBlk * (size_t)(p->ny + 2) * tsz;  // populations
    b += sizeof(SimDev) + sizeof(uint32_t);
    if (p->bc_west == LBM_BC_DIRICHLET) b += sizeof(double) * 2 * nperim;
    const Tiling& t = kTilings[kTileDefault];
    size_t ntiles;
    if (t.tx == 0) {
        const size_t nb = (size_t)((p->nx + kBlk - 1) / kBlk) * p->ny, per = (size_t)t.ty * t.rpt;
        ntiles = (nb + per - 1) / per;
    } else {
        const size_t th = (size_t)t.ty * t.rpt;
        ntiles = ((p->ny + th - 1) / th) * ((p->nx + t.tx - 1) / t.tx);
    }
    b += sizeof(int4) * std::max<size_t>(1, ntiles);
    b += sizeof(int2) * std::max<size_t>(1, (nperim + 255) / 256);
    size_t M = 0, nb = 0;
    for (int k = 0; k < nbodies; ++k) {
        if (markers[k] < 0) return 0;
        if (markers[k] > 0) {
            M += (size_t)markers[k];
            ++nb;
        }
    }
    b += sizeof(BodyDev) * LBM_MAX_BODIES + sizeof(double) * 5 * std::max<size_t>(1, M);
    b += sizeof(GroupDev) * std::max<size_t>(1, nb);
    b += sizeof(int2) * (16 * M / 256 + nb + 1);  // band chunks
    // per group of Mg markers, with cn = max(1, band nodes) <= 16 Mg + 1
    const size_t per_marker = sizeof(int) * 16 * 2          // node_cell, node_run
                              + sizeof(int) * 16 * 2        // ent, mnode
                              + tsz * 4 * 16                // node4
                              + 2 * tsz * 16                // ent_D
                              + tsz * (8 + 5)               // m_phi, m_wtot
                              + sizeof(unsigned short) * 4  // m_rows
                              + sizeof(double) * 5          // m_red
                              + sizeof(unsigned short) * 2; // cord
    const size_t per_group = sizeof(int) * 3 + sizeof(int) * 2 + sizeof(int) * 4 + tsz * 4 + 2 * tsz + tsz * 13 +
                             sizeof(unsigned short) * 4 + sizeof(double) * 5 + sizeof(int) * (kMaxColors + 1);
    b += per_marker * M + per_group * nb;
    return b;
}

int32_t lbm_tiling_count(void) { return kNumTilings; }

lbm_status lbm_tiling_info(int32_t k, int32_t* tx, int32_t* ty, int32_t* rpt) {
    if (k < 0 || k >= kNumTilings) return LBM_ERR_INVALID;
    if (tx) *tx = kTilings[k].tx;
    if (ty) *ty = kTilings[k].ty;
    if (rpt) *rpt = kTilings[k].rpt;
    return LBM_OK;
}

}  // extern "C"

// ================================================================ batches

namespace {

lbm_status hipfailb(lbm_batch* b, hipError_t e, const char* where) {
    return failb(b, e == hipErrorOutOfMemory ? LBM_ERR_NOMEM : LBM_ERR_DEVICE,
                 fmt("%s: %s", where, hipGetErrorString(e)));
}

#define HIPB(b, call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hipfailb(b, e_, #call); \
    } while (0)

void drop_graphs(lbm_batch* b) {
    b->lane[0].drop();
    b->lane[1].drop();
}

// Copy the per-simulation step state (AA state, counters) of the device table
// back into the simulations' host descriptors.
lbm_status sync_back(lbm_batch* b) {
    HIPB(b, hipStreamSynchronize(b->stream));
    if (b->sims.empty()) return LBM_OK;
    std::vector<SimDev> h(b->sims.size());
    HIPB(b, hipMemcpy(h.data(), b->d_sims.p, sizeof(SimDev) * h.size(), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < h.size(); ++k) {
        lbm_sim* s = b->sims[b->order[k]];
        s->h.swapped = h[k].swapped;
        s->h.steps_done = h[k].steps_done;
        s->h.steps_left = h[k].steps_left;
        s->h.active = h[k].active;
        s->steps = h[k].steps_done;
    }
    return LBM_OK;
}

template <typename V>
hipError_t ensure_cap(DevBuf& buf, size_t& cap, size_t need, bool& grew) {
    if (need <= cap && buf.p) return hipSuccess;
    size_t c = std::max<size_t>(need + need / 2, 16);
    hipError_t e = buf.alloc(c * sizeof(V));
    if (e != hipSuccess) return e;
    cap = c;
    grew = true;
    return hipSuccess;
}

// Rebuild and upload the batch's work tables from the admitted simulations'
// host descriptors (call sync_back first when simulations are in flight).
// Unless one lane is requested, the simulations whose largest body group
// exceeds kHeavyGroupMarkers form lane 0 when that leaves both lanes non-empty
// and lane 0 with at most half of the nodes; otherwise one lane holds
// everything.  Lanes = 4 splits them into two lanes of about equal node count
// instead.
lbm_status upload_tables(lbm_batch* b) {
    const int n = (int)b->sims.size();
    std::vector<int> heavy, light;
    int64_t heavy_cells = 0, cells = 0;
    for (int k = 0; k < n; ++k) {
        const lbm_sim* s = b->sims[k];
        const int64_t c = (int64_t)s->p.nx * s->p.ny;
        cells += c;
        if (s->max_group > kHeavyGroupMarkers) {
            heavy.push_back(k);
            heavy_cells += c;
        } else {
            light.push_back(k);
        }
    }
    // lanes 4: halves of equal node count (largest first, each to the lane
    // with fewer nodes so far), interleaved, so that one half's correction
    // runs under the other half's sweep
    const bool halves = b->lanes_req == 4 && n >= 2;
    const bool by_weight = !halves && b->lanes_req != 1 && b->lanes_req != 4 && !heavy.empty() && !light.empty() &&
                           2 * heavy_cells <= cells;
    const bool two = by_weight || halves;
    const int nl = two ? 2 : 1;
    const bool il = two && (b->lanes_req >= 3 || (b->lanes_req == 0 && cells >= kInterleaveMinCells));
    if (nl != b->nlanes || il != b->interleave) drop_graphs(b);
    b->nlanes = nl;
    b->interleave = il;
    b->order.clear();
    int lane0_sims = n;  // simulations of lane 0 (the first ones in b->order)
    if (by_weight) {
        b->order = heavy;
        b->order.insert(b->order.end(), light.begin(), light.end());
        lane0_sims = (int)heavy.size();
    } else if (halves) {
        std::vector<int> idx(n);
        for (int k = 0; k < n; ++k) idx[k] = k;
        auto cells_of = [&](int k) { return (int64_t)b->sims[k]->p.nx * b->sims[k]->p.ny; };
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return cells_of(a) > cells_of(c); });
        std::vector<int> half[2];
        int64_t sum[2] = {0, 0};
        for (int k : idx) {
            const int l = sum[1] < sum[0] ? 1 : 0;
            half[l].push_back(k);
            sum[l] += cells_of(k);
        }
        for (int l = 0; l < 2; ++l) std::sort(half[l].begin(), half[l].end());  // admission order within a lane
        b->order = half[0];
        b->order.insert(b->order.end(), half[1].begin(), half[1].end());
        lane0_sims = (int)half[0].size();
    } else {
        for (int k = 0; k < n; ++k) b->order.push_back(k);
    }
    std::vector<SimDev> sims;
    for (int r = 0; r < n; ++r) sims.push_back(b->sims[b->order[r]]->h);
    bool grew_sims = false;
    HIPB(b, ensure_cap<SimDev>(b->d_sims, b->cap_sims, sims.size(), grew_sims));
    if (grew_sims) drop_graphs(b);
    if (!sims.empty())
        HIPB(b, hipMemcpyAsync(b->d_sims.p, sims.data(), sizeof(SimDev) * sims.size(), hipMemcpyHostToDevice, b->stream));
    const int lane_begin[3] = {0, lane0_sims, n};
    for (int l = 0; l < 2; ++l) {
        Lane& L = b->lane[l];
        const int r0 = l < nl ? lane_begin[l] : n, r1 = l < nl ? lane_begin[l + 1] : n;
        std::vector<int4> tiles;
        std::vector<int2> bc;
        std::vector<GroupDev> groups;
        // row bands of tiles dealt round-robin to the eight XCDs
        std::vector<int4> per_xcd[8];
        int band = 0;
        for (int r = r0; r < r1; ++r) {
            lbm_sim* s = b->sims[b->order[r]];
            std::vector<int4> mine;
            build_tiles(s, r, b->tiling, mine);
            for (size_t i = 0; i < mine.size(); ++i) {
                if (i > 0 && mine[i].z != mine[i - 1].z) ++band;
                per_xcd[band & 7].push_back(mine[i]);
            }
            ++band;
            build_bc(s, r, bc);
            for (Group* g : s->grp) {
                GroupDev d = g->d;
                d.sim = r;
                // interleaved FP32 lanes: every band is gathered and applied by
                // its correction workgroup, which runs beside the other lane's
                // sweep (the band kernels would need the whole chip between the
                // sweeps; the results are the same)
                if (il && !b->f64) d.in_kernel = 1;
                groups.push_back(d);
            }
        }
        // largest groups first: the persistent correction kernel starts the long ones early
        std::stable_sort(groups.begin(), groups.end(), [](const GroupDev& a, const GroupDev& c) { return a.M > c.M; });
        std::vector<int2> chunks;
        for (size_t gi = 0; gi < groups.size(); ++gi) build_chunks(groups[gi], (int)gi, chunks);
        const int max_group = groups.empty() ? 0 : groups.front().M;
        bool changed = ib_variant(b->f64, max_group, il) != ib_variant(b->f64, L.max_group, il);
        L.max_group = max_group;
        bool mrt = false, near_edge = false;
        for (int r = r0; r < r1; ++r) {
            mrt = mrt || b->sims[b->order[r]]->h.collision != 0;
            near_edge = near_edge || b->sims[b->order[r]]->band_near_edge;
        }
        changed = changed || mrt != L.mrt;
        L.mrt = mrt;
        const bool bnd_in_ib = !bc.empty() && !groups.empty() && !near_edge;
        changed = changed || bnd_in_ib != L.bnd_in_ib;
        L.bnd_in_ib = bnd_in_ib;
        BatchHeader h{};
        h.nsims = r1 - r0;
        h.nbc = (int)bc.size();
        h.ngroups = (int)groups.size();
        h.nchunks = (int)chunks.size();
        std::vector<int4> tl;
        for (int x = 0; x < 8; ++x) {
            h.xcd_start[x] = (int)tl.size();
            tl.insert(tl.end(), per_xcd[x].begin(), per_xcd[x].end());
        }
        h.xcd_start[8] = (int)tl.size();
        h.ntiles = (int)tl.size();
        // One workgroup per tile (workgroup b runs on XCD b mod 8 and takes that
        // XCD's tile b / 8): with a persistent grid the tiles of late-starting
        // workgroups made the tail of every sweep.  Extra workgroups exit at once,
        // so the grid only grows (with headroom) and captured graphs stay valid
        // while tiles come and go.
        int per_xcd_max = 1;
        for (int x = 0; x < 8; ++x) per_xcd_max = std::max(per_xcd_max, h.xcd_start[x + 1] - h.xcd_start[x]);
        if (8 * per_xcd_max > L.grid_sweep) {
            L.grid_sweep = 8 * (per_xcd_max + per_xcd_max / 4);
            changed = true;
        }
        // band kernels: one workgroup per chunk, grown the same way
        if (h.nchunks > L.grid_band) {
            L.grid_band = h.nchunks + h.nchunks / 4 + 8;
            changed = true;
        }
        // a kind of kernel with no work in the lane is left out of its graphs
        changed = changed || (h.nbc > 0) != (L.nbc > 0) || (h.nchunks > 0) != (L.nchunks > 0) ||
                  (h.ngroups > 0) != (L.ngroups > 0);
        bool grew = false;
        HIPB(b, ensure_cap<int4>(L.d_tiles, L.cap_tiles, tl.size(), grew));
        HIPB(b, ensure_cap<int2>(L.d_bc, L.cap_bc, bc.size(), grew));
        HIPB(b, ensure_cap<GroupDev>(L.d_groups, L.cap_groups, groups.size(), grew));
        HIPB(b, ensure_cap<int2>(L.d_chunks, L.cap_chunks, chunks.size(), grew));
        if (!L.d_hdr.p) {
            HIPB(b, L.d_hdr.alloc(sizeof(BatchHeader)));
            grew = true;
        }
        if (grew || changed || L.sim0 != r0) L.drop();
        L.sim0 = r0;
        if (!tl.empty()) HIPB(b, hipMemcpyAsync(L.d_tiles.p, tl.data(), sizeof(int4) * tl.size(), hipMemcpyHostToDevice, b->stream));
        if (!bc.empty()) HIPB(b, hipMemcpyAsync(L.d_bc.p, bc.data(), sizeof(int2) * bc.size(), hipMemcpyHostToDevice, b->stream));
        if (!groups.empty())
            HIPB(b, hipMemcpyAsync(L.d_groups.p, groups.data(), sizeof(GroupDev) * groups.size(), hipMemcpyHostToDevice, b->stream));
        if (!chunks.empty())
            HIPB(b, hipMemcpyAsync(L.d_chunks.p, chunks.data(), sizeof(int2) * chunks.size(), hipMemcpyHostToDevice, b->stream));
        HIPB(b, hipMemcpyAsync(L.d_hdr.p, &h, sizeof h, hipMemcpyHostToDevice, b->stream));
        HIPB(b, hipStreamSynchronize(b->stream));
        L.nsims = h.nsims;
        L.ntiles = h.ntiles;
        L.nbc = h.nbc;
        L.ngroups = h.ngroups;
        L.nchunks = h.nchunks;
    }
    return LBM_OK;
}

// The kernels of one step of lane l, one kernel kind k (0 sweep, 1 boundary,
// 2 band gather, 3 correction sweeps, 4 band apply, 5 bookkeeping) on `st`.
hipError_t launch_kind(lbm_batch* b, int l, int k, hipStream_t st) {
    const Lane& L = b->lane[l];
    SimDev* sims = (SimDev*)b->d_sims.p;
    const BatchHeader* hdr = (const BatchHeader*)L.d_hdr.p;
    // kinds with no work in the lane are not launched (upload_tables drops
    // the captured graphs when that changes); the boundary rules ride on the
    // correction launch when they cannot touch a band
    if ((k == 1 && (L.nbc == 0 || L.bnd_in_ib)) || ((k == 2 || k == 4) && L.nchunks == 0) ||
        (k == 3 && L.ngroups == 0))
        return hipSuccess;
    switch (k) {
        case 0: return launch_sweep(b->f64, L.mrt, b->tiling, sims, (const int4*)L.d_tiles.p, hdr, 0, L.grid_sweep, -1, st);
        case 1: return launch_boundary(b->f64, sims, (const int2*)L.d_bc.p, hdr, 0, b->grid_bc, -1, st);
        case 2:
            return launch_band(b->f64, false, sims, (const GroupDev*)L.d_groups.p, (const int2*)L.d_chunks.p, hdr, 0,
                               L.grid_band, -1, st);
        case 3:
            return launch_ib(b->f64, L.max_group, sims, (GroupDev*)L.d_groups.p, hdr, 0, b->grid_ib, -1, st,
                             b->interleave, L.bnd_in_ib ? (const int2*)L.d_bc.p : nullptr);
        case 4:
            return launch_band(b->f64, true, sims, (const GroupDev*)L.d_groups.p, (const int2*)L.d_chunks.p, hdr, 0,
                               L.grid_band, -1, st);
        default: return launch_advance(sims + L.sim0, hdr, 0, st);
    }
}

hipError_t enqueue_steps(lbm_batch* b, int l, int n, hipStream_t st) {
    for (int t = 0; t < n; ++t)
        for (int k = 0; k < 6; ++k) {
            hipError_t e = launch_kind(b, l, k, st);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

template <typename F>
hipError_t capture_fn(hipStream_t st, F&& enqueue, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e2 = enqueue();
    e = hipStreamEndCapture(st, &g);
    if (e2 != hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

hipError_t capture(lbm_batch* b, int l, int n, hipStream_t st, hipGraphExec_t* out) {
    return capture_fn(st, [&]() { return enqueue_steps(b, l, n, st); }, out);
}

// Lane 1 runs on the batch's second stream, ordered after everything already
// enqueued on the batch stream; the batch stream waits for it at the end.  The
// second stream must reach the GPU through another hardware queue than the
// batch stream (else the lanes run one after the other): candidates are
// created until one runs concurrently with the batch stream, the others are
// destroyed afterwards (kept until then, so that the next candidate lands
// elsewhere); if none does, the last one serves (same results, no overlap).
constexpr int kLaneStreamTries = 6;

lbm_status ensure_lane_stream(lbm_batch* b) {
    if (b->stream2) return LBM_OK;
    if (!b->d_probe.p) HIPB(b, b->d_probe.alloc(2 * sizeof(int)));
    std::vector<hipStream_t> rejected;
    hipStream_t pick = nullptr;
    bool concurrent = false;
    hipError_t err = hipSuccess;
    for (int k = 0; k < kLaneStreamTries && !concurrent; ++k) {
        hipStream_t c = nullptr;
        err = hipStreamCreateWithFlags(&c, hipStreamNonBlocking);
        if (err != hipSuccess) break;
        err = streams_run_concurrently(b->stream, c, (int*)b->d_probe.p, &concurrent);
        if (err != hipSuccess) {
            rejected.push_back(c);
            break;
        }
        if (concurrent)
            pick = c;
        else
            rejected.push_back(c);
    }
    if (err == hipSuccess && !pick) {
        pick = rejected.back();
        rejected.pop_back();
    }
    for (hipStream_t r : rejected) (void)hipStreamDestroy(r);
    HIPB(b, err);
    b->stream2 = pick;
    b->lanes_concurrent = concurrent ? 1 : 0;
    HIPB(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    HIPB(b, hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    HIPB(b, hipEventCreateWithFlags(&b->ev_sweep0, hipEventDisableTiming));
    HIPB(b, hipEventCreateWithFlags(&b->ev_sweep1, hipEventDisableTiming));
    return LBM_OK;
}

// Two lanes, interleaved step by step with their sweeps in turn: lane 1's
// sweep of step t waits for lane 0's sweep of step t, and lane 0's sweep of
// step t + 1 for lane 1's sweep of step t, so each lane's boundary rules and
// correction run while the other lane's sweep streams (a lean correction
// workgroup finds room on a CU beside sweep waves; a 768-thread one waits for
// a whole CU).  Each lane replays two graphs per step, its sweep and the rest
// of its step; the events that order the lanes are recorded and waited on
// outside any capture.
lbm_status run_interleaved(lbm_batch* b, int n) {
    hipStream_t st[2] = {b->stream, b->stream2};
    for (int l = 0; l < 2; ++l) {
        Lane& L = b->lane[l];
        if (!L.graphA) HIPB(b, capture_fn(st[l], [&]() { return launch_kind(b, l, 0, st[l]); }, &L.graphA));
        if (!L.graphB)
            HIPB(b, capture_fn(st[l], [&]() {
                for (int k = 1; k < 6; ++k) {
                    hipError_t e = launch_kind(b, l, k, st[l]);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            }, &L.graphB));
    }
    HIPB(b, hipEventRecord(b->ev_fork, st[0]));
    HIPB(b, hipStreamWaitEvent(st[1], b->ev_fork, 0));
    for (int t = 0; t < n; ++t) {
        if (t > 0) HIPB(b, hipStreamWaitEvent(st[0], b->ev_sweep1, 0));
        HIPB(b, hipGraphLaunch(b->lane[0].graphA, st[0]));
        HIPB(b, hipEventRecord(b->ev_sweep0, st[0]));
        HIPB(b, hipGraphLaunch(b->lane[0].graphB, st[0]));
        HIPB(b, hipStreamWaitEvent(st[1], b->ev_sweep0, 0));
        HIPB(b, hipGraphLaunch(b->lane[1].graphA, st[1]));
        HIPB(b, hipEventRecord(b->ev_sweep1, st[1]));
        HIPB(b, hipGraphLaunch(b->lane[1].graphB, st[1]));
    }
    HIPB(b, hipEventRecord(b->ev_join, st[1]));
    HIPB(b, hipStreamWaitEvent(st[0], b->ev_join, 0));
    return LBM_OK;
}

// n steps of every lane: each lane replays its graphs of 8 and 1 steps on its
// own stream, or two lanes are interleaved step by step (run_interleaved).
lbm_status run_steps(lbm_batch* b, int n) {
    hipStream_t st[2] = {b->stream, nullptr};
    if (b->nlanes == 2) {
        lbm_status rc = ensure_lane_stream(b);
        if (rc != LBM_OK) return rc;
        if (b->interleave) return run_interleaved(b, n);
        st[1] = b->stream2;
        HIPB(b, hipEventRecord(b->ev_fork, st[0]));
        HIPB(b, hipStreamWaitEvent(st[1], b->ev_fork, 0));
    }
    for (int l = 0; l < b->nlanes; ++l) {
        Lane& L = b->lane[l];
        if (!L.graph1) HIPB(b, capture(b, l, 1, st[l], &L.graph1));
        if (!L.graphK) HIPB(b, capture(b, l, b->graphK_steps, st[l], &L.graphK));
        int left = n;
        for (; left >= b->graphK_steps; left -= b->graphK_steps) HIPB(b, hipGraphLaunch(L.graphK, st[l]));
        for (; left > 0; --left) HIPB(b, hipGraphLaunch(L.graph1, st[l]));
    }
    if (b->nlanes == 2) {
        HIPB(b, hipEventRecord(b->ev_join, st[1]));
        HIPB(b, hipStreamWaitEvent(st[0], b->ev_join, 0));
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(int32_t precision, size_t budget, void* hip_stream, lbm_batch** out) {
    if (!out || (precision != LBM_F64 && precision != LBM_F32_SHIFTED)) return LBM_ERR_INVALID;
    *out = nullptr;
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ERR_NOMEM;
    b->f64 = precision == LBM_F64;
    b->budget = budget;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return LBM_ERR_DEVICE;
    }
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) {
            delete b;
            return LBM_ERR_DEVICE;
        }
        b->own_stream = true;
    }
    const int ncu = num_cus(b->device);
    b->grid_bc = ncu * 8;
    b->grid_ib = ncu * 2;
    if (upload_tables(b) != LBM_OK) {
        lbm_batch_destroy(b);
        return LBM_ERR_NOMEM;
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    (void)sync_back(b);
    for (lbm_sim* s : b->sims) {
        s->batch = nullptr;
        s->h.active = 1;
        s->h.steps_left = -1;
        (void)hipMemcpy(s->desc.p, &s->h, sizeof(SimDev), hipMemcpyHostToDevice);
    }
    b->sims.clear();
    drop_graphs(b);
    bool own = b->own_stream;
    hipStream_t st = b->stream;
    delete b;
    if (own && st) (void)hipStreamDestroy(st);
}

lbm_status lbm_batch_admit(lbm_batch* b, lbm_sim* s, int64_t steps) {
    if (!b || !s) return LBM_ERR_INVALID;
    if (s->batch) return failb(b, LBM_ERR_INVALID, "simulation already in a batch");
    if (s->f64 != b->f64) return failb(b, LBM_ERR_INVALID, "precision differs from the batch");
    const size_t need = lbm_device_bytes(s);
    if (b->budget && b->bytes + need > b->budget) return failb(b, LBM_ERR_NOMEM, "HBM budget exhausted");
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    HIPB(b, hipStreamSynchronize(s->stream));
    s->h.active = steps == 0 ? 0 : 1;
    s->h.steps_left = steps > 0 ? steps : -1;
    b->sims.push_back(s);
    s->batch = b;
    b->bytes += need;
    rc = upload_tables(b);
    if (rc != LBM_OK) {
        b->sims.pop_back();
        s->batch = nullptr;
        b->bytes -= need;
        s->h.active = 1;
        s->h.steps_left = -1;
    }
    return rc;
}

lbm_status lbm_batch_retire(lbm_batch* b, lbm_sim* s) {
    if (!b || !s || s->batch != b) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    auto it = std::find(b->sims.begin(), b->sims.end(), s);
    b->sims.erase(it);
    b->bytes -= std::min(b->bytes, lbm_device_bytes(s));
    s->batch = nullptr;
    s->h.active = 1;
    s->h.steps_left = -1;
    HIPB(b, hipMemcpy(s->desc.p, &s->h, sizeof(SimDev), hipMemcpyHostToDevice));
    return upload_tables(b);
}

lbm_status lbm_batch_step(lbm_batch* b, int32_t nsteps) {
    if (!b || nsteps < 0) return LBM_ERR_INVALID;
    return run_steps(b, nsteps);
}

lbm_status lbm_batch_sync(lbm_batch* b) {
    if (!b) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    for (lbm_sim* s : b->sims) {
        uint32_t st = 0;
        HIPB(b, hipMemcpy(&st, s->status.p, sizeof st, hipMemcpyDeviceToHost));
        if (st & ST_UNSTABLE) return failb(b, LBM_ERR_UNSTABLE, "a simulation in the batch went unstable");
    }
    return LBM_OK;
}

lbm_status lbm_batch_remaining(lbm_batch* b, lbm_sim* s, int64_t* remaining) {
    if (!b || !s || s->batch != b || !remaining) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    *remaining = s->h.active ? (s->h.steps_left < 0 ? -1 : s->h.steps_left) : 0;
    return LBM_OK;
}

size_t lbm_batch_bytes(const lbm_batch* b) { return b ? b->bytes : 0; }

lbm_status lbm_batch_set_tiling(lbm_batch* b, int32_t tiling) {
    if (!b || tiling < 0 || tiling >= kNumTilings) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    b->tiling = tiling;
    drop_graphs(b);
    return upload_tables(b);
}

int32_t lbm_batch_get_tiling(const lbm_batch* b) { return b ? b->tiling : -1; }

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t trials, int32_t* chosen) {
    if (!b || trials <= 0) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    if (b->sims.empty()) {
        if (chosen) *chosen = b->tiling;
        return LBM_OK;
    }
    // save the state every candidate will advance
    struct Saved {
        DevBuf pop, bodies, markers;
        SimDev h;
    };
    std::vector<Saved> saved(b->sims.size());
    for (size_t k = 0; k < b->sims.size(); ++k) {
        lbm_sim* s = b->sims[k];
        saved[k].h = s->h;
        HIPB(b, saved[k].pop.alloc(s->pop.bytes));
        HIPB(b, saved[k].bodies.alloc(s->bodies.bytes));
        HIPB(b, saved[k].markers.alloc(s->markers.bytes));
        HIPB(b, hipMemcpyAsync(saved[k].pop.p, s->pop.p, s->pop.bytes, hipMemcpyDeviceToDevice, b->stream));
        HIPB(b, hipMemcpyAsync(saved[k].bodies.p, s->bodies.p, s->bodies.bytes, hipMemcpyDeviceToDevice, b->stream));
        HIPB(b, hipMemcpyAsync(saved[k].markers.p, s->markers.p, s->markers.bytes, hipMemcpyDeviceToDevice, b->stream));
    }
    HIPB(b, hipStreamSynchronize(b->stream));
    hipEvent_t e0, e1;
    HIPB(b, hipEventCreate(&e0));
    HIPB(b, hipEventCreate(&e1));
    // one candidate: tables, a warm-up step, then `trials` timed steps replayed
    // from freshly captured graphs; the state is restored afterwards
    auto trial = [&](float& ms) -> lbm_status {
        drop_graphs(b);
        lbm_status r = upload_tables(b);
        if (r != LBM_OK) return r;
        r = run_steps(b, 1);
        if (r != LBM_OK) return r;
        HIPB(b, hipEventRecord(e0, b->stream));
        r = run_steps(b, trials);
        if (r != LBM_OK) return r;
        HIPB(b, hipEventRecord(e1, b->stream));
        HIPB(b, hipEventSynchronize(e1));
        HIPB(b, hipEventElapsedTime(&ms, e0, e1));
        for (size_t q = 0; q < b->sims.size(); ++q) {
            lbm_sim* s = b->sims[q];
            s->h = saved[q].h;
            HIPB(b, hipMemcpyAsync(s->pop.p, saved[q].pop.p, s->pop.bytes, hipMemcpyDeviceToDevice, b->stream));
            HIPB(b, hipMemcpyAsync(s->bodies.p, saved[q].bodies.p, s->bodies.bytes, hipMemcpyDeviceToDevice, b->stream));
            HIPB(b, hipMemcpyAsync(s->markers.p, saved[q].markers.p, s->markers.bytes, hipMemcpyDeviceToDevice, b->stream));
            HIPB(b, hipMemsetAsync(s->status.p, 0, sizeof(uint32_t), b->stream));
        }
        HIPB(b, hipStreamSynchronize(b->stream));
        return LBM_OK;
    };
    // every tiling under each lane schedule: the requested one; with an
    // automatic request also two interleaved halves; and one lane (when there
    // are two simulations or more).  The fastest pair stays (ties go to the
    // earlier one): the best tiling differs between schedules.
    const int req = b->lanes_req;
    std::vector<int> cand{req};
    if (req != 1 && b->sims.size() >= 2) {
        if (req == 0) cand.push_back(4);
        cand.push_back(1);
    }
    int best = b->tiling, best_lanes = req;
    float best_ms = 1e30f;
    for (int c : cand) {
        b->lanes_req = c;
        for (int k = 0; k < kNumTilings && rc == LBM_OK; ++k) {
            b->tiling = k;
            float ms = 0.f;
            rc = trial(ms);
            if (rc == LBM_OK && ms < best_ms) {
                best_ms = ms;
                best = k;
                best_lanes = c;
            }
        }
        if (rc != LBM_OK) break;
    }
    b->tiling = best;
    b->lanes_req = rc == LBM_OK ? best_lanes : req;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graphs(b);
    lbm_status rc2 = upload_tables(b);
    if (rc == LBM_OK) rc = rc2;
    if (chosen) *chosen = best;
    return rc;
}

lbm_status lbm_batch_set_lanes(lbm_batch* b, int32_t lanes) {
    if (!b || lanes < 0 || lanes > 4) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    b->lanes_req = lanes;
    drop_graphs(b);
    return upload_tables(b);
}

int32_t lbm_batch_get_lanes(const lbm_batch* b) { return b ? b->nlanes : -1; }

int32_t lbm_batch_get_lane_mode(const lbm_batch* b) { return b ? b->lanes_req : -1; }

int32_t lbm_batch_lanes_concurrent(const lbm_batch* b) { return b ? b->lanes_concurrent : -1; }

lbm_status lbm_batch_profile(lbm_batch* b, int32_t nsteps, double ms[4], int64_t* cells) {
    if (!b || nsteps < 0 || !ms) return LBM_ERR_INVALID;
    lbm_status rc = sync_back(b);
    if (rc != LBM_OK) return rc;
    int64_t c = 0;
    for (lbm_sim* s : b->sims)
        if (s->h.active) c += (int64_t)s->p.nx * s->p.ny;
    if (cells) *cells = c;
    for (int k = 0; k < 4; ++k) ms[k] = 0.0;
    // every kernel kind of every lane in turn on the batch stream, events
    // around each kind: sweep, boundary, correction (band gather, sweeps,
    // band apply), bookkeeping
    static const int cat_of[6] = {0, 1, 2, 2, 2, 3};
    hipEvent_t ev[7];
    for (int k = 0; k < 7; ++k) HIPB(b, hipEventCreate(&ev[k]));
    for (int t = 0; t < nsteps; ++t) {
        HIPB(b, hipEventRecord(ev[0], b->stream));
        for (int k = 0; k < 6; ++k) {
            for (int l = 0; l < b->nlanes; ++l) HIPB(b, launch_kind(b, l, k, b->stream));
            HIPB(b, hipEventRecord(ev[k + 1], b->stream));
        }
        HIPB(b, hipEventSynchronize(ev[6]));
        for (int k = 0; k < 6; ++k) {
            float m = 0.f;
            HIPB(b, hipEventElapsedTime(&m, ev[k], ev[k + 1]));
            ms[cat_of[k]] += m;
        }
    }
    for (int k = 0; k < 7; ++k) (void)hipEventDestroy(ev[k]);
    return LBM_OK;
}


}  // extern "C"

// Host engine and C-ABI of the SPFD library: geometry and brick layout,
// multigrid hierarchy, flexible preconditioned CG driver, E-field.
//
// Method (paper, Sec. II Eqs. (1), (3); Sec. III): Eq. (3) is solved by CG
// preconditioned with a multigrid cycle; the paper used a closed-source
// algebraic multigrid inside FGMRES with an unstated configuration.  Here the
// hierarchy is a structured aggregation multigrid built for the voxel grid:
//   * aggregates are 2x2x2 blocks of nodes; with the piecewise-constant
//     prolongation P the Galerkin operator P^T A P of a 7-point graph
//     Laplacian is again a 7-point graph Laplacian whose edge conductance is
//     the sum of the four fine conductances crossing the aggregate interface;
//   * smoothing is a Chebyshev polynomial in D^-1 A on [2/ratio, 2]; the grid
//     graph is bipartite, so the largest eigenvalue of D^-1 A is exactly 2;
//   * the coarsest level (<= coarsest_max unknowns) is solved with a dense
//     FP64 pseudo-inverse;
//   * the outer iteration is flexible CG in FP64 (alpha, beta, residual norms
//     and the final gauge in FP64); in mixed precision the whole cycle runs in
//     FP32.  All scalars stay on the device; the host only polls a stop flag.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "kernels.h"
#include "spfd.h"

using namespace spfd;

namespace {

struct Level {
    int N[3] = {0, 0, 0};        // nodes
    int G[3] = {0, 0, 0};        // bricks
    int nb = 0;
    std::vector<int> slot_of;    // dense brick grid -> slot (host)
    std::vector<int4> coord;     // slot -> brick coordinates (host)
    int *d_slot_of = nullptr;
    int *d_nbr = nullptr;
    int4 *d_coord = nullptr;
    int *d_parent_slot = nullptr;  // slot of the coarse brick that holds this brick (levels < last)
    uint8_t *d_tiles = nullptr;    // finest level, label form
    double *d_w64 = nullptr;
    float *d_w32 = nullptr;
    uint16_t *d_w16 = nullptr;     // first coarse level of an FP32 cycle: FP16 weights / w16s
    float w16s = 0.0f;
    // cycle buffers (type of the cycle)
    void *x = nullptr, *x2 = nullptr, *d = nullptr, *b = nullptr;
    long long dofs = 0;
    // unstructured (ELL) level: rows = split aggregates, K neighbours per row
    bool ell = false;
    int nrow = 0, K = 0;
    int *d_col = nullptr;
    double *d_val64 = nullptr;
    float *d_val32 = nullptr;
    int4 *d_pos = nullptr;          // grid position of each row at this level
    int *d_mptr = nullptr;          // members of each row in the finer level (CSR)
    int *d_mem = nullptr;
    int *d_memb = nullptr;          // the same as a direct table of 8 per row (null: an aggregate has more)
    int *d_agg = nullptr;           // this level's unknown -> row of the next (split) level, -1 if none
    unsigned long long *d_cmask = nullptr;  // node columns with unknowns, per brick (structured levels)
    double *d_dinv64 = nullptr;             // inverse diagonal (0 where it vanishes), FP64 and FP32
    float *d_dinv32 = nullptr;
    int seg = 0;                            // column segment (nodes per lane) of an FP32 cycle on this level:
                                            // 4 or 8 when tuned at build, 0 = by the brick-count threshold
    Topo topo() const { return Topo{nb, d_nbr, d_cmask}; }
    long long nodes() const { return ell ? (long long)nrow : (long long)nb * BS; }
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // second stream of the build (default priority): the connected components, then the column masks and
    // inverse diagonals, run there beside the coarsening and the coarsest inverse; joined before the build
    // returns
    hipStream_t side = nullptr;
    hipEvent_t ev_side[2] = {nullptr, nullptr};   // [0] main -> side (inputs ready), [1] side -> main (work done)
    std::string err;
    // geometry
    int state = 0;  // 0 created, 1 geometry, 2 sigma, 3 built, 4 sources
    Grid g{};
    double h[3] = {0, 0, 0};
    double geo4[3] = {0, 0, 0};
    uint8_t *d_labels = nullptr;
    double *d_sigvox = nullptr;
    bool voxel_mode = false;
    // several voxel models packed along z into one handle (spfd_set_geometry_many); np = 0: one model
    int np = 0;
    ModelBoxes mbox{};
    Grid mgrid[MAX_MODELS];
    long long mnodes_off[MAX_MODELS + 1] = {};   // offsets of the models' dense node arrays in psi
    int mfirst[MAX_MODELS] = {}, mcount[MAX_MODELS] = {};   // the models' finest-level bricks (after build)
    int2 *d_mrange = nullptr;                               // the same on the device (first, count)
    double *d_mtables = nullptr;                            // [MAX_MODELS][MAX_LABELS] conductivity tables
    int nlab = 0;
    double table[MAX_LABELS];
    double *d_table64 = nullptr;
    float *d_table32 = nullptr;
    // hierarchy
    spfd_amg_options opt{};
    std::vector<Level> lv;
    int ncomp = 0;
    int *d_comp = nullptr;
    int *d_counts = nullptr;
    double *d_means = nullptr;
    double *d_cpart = nullptr;   // partials of the component means (comp_mean_parts of the finest level)
    int ncoarse = 0;
    int *d_cdof_node = nullptr;
    int *d_node_cdof = nullptr;
    int *d_cadj = nullptr;
    double *d_Ainv = nullptr;
    int *d_cwork = nullptr;
    std::vector<double> cheb_c1, cheb_c2;
    double cheb_c0 = 0.0;
    // outer CG state
    int nrhs = 0;
    double *d_bs = nullptr;   // right sides [nrhs][n0]
    std::vector<int> has_source;
    double *d_x = nullptr, *d_r = nullptr, *d_q = nullptr;
    // the search directions of the current window of CG steps (a right side's p_k in the slot given by its
    // Scal::hcount, in the cycle's precision; slots phist_stride elements apart) and their step sizes
    // [nrhs][phist_len]; x is updated from them every phist_len steps and at the end of a pass
    uint8_t *d_phist = nullptr;
    double *d_ahist = nullptr;
    int phist_len = 2;
    long long phist_stride = 0;
    void *d_z = nullptr;
    float *d_r32 = nullptr;
    Scal *d_scal = nullptr;
    Scal *h_scal = nullptr;   // pinned, one per right side plus one for the adjoint solve
    Scal *h_ring = nullptr;   // pinned, 2 x (nrhs + 1): scalars of the last two enqueued CG steps
    Scal *h_ring_dev = nullptr;   // device address of h_ring (written by the last kernel of a CG step)
    int h_cap = 0;                // right sides h_scal and h_ring hold (plus one each)
    Scal *d_nostop = nullptr;     // zeroed scalars (never stopped) for cycles run outside a CG step
    Scal *step_mirror = nullptr;  // where the CG step being enqueued leaves its scalars
    hipEvent_t ev_it[2] = {nullptr, nullptr};
    // adjoint solve
    double *d_adj_b = nullptr;
    double *d_adj_c = nullptr;
    double *d_adj_lam = nullptr;
    double *d_adj_labpart = nullptr;
    double *d_adj_labout = nullptr;
    Scal *d_adj_scal = nullptr;
    // flexible GMRES: basis V [(m+1)][n0], preconditioned vectors Z [m][n0], least-squares state, partials
    double *d_fgV = nullptr;
    void *d_fgZ = nullptr;
    FGState *d_fgst = nullptr;
    double *d_fgpart = nullptr;
    int fg_m = 0;
    // quantile selection
    uint8_t *d_sel_work = nullptr;
    double *d_sel_out = nullptr;
    double *d_part = nullptr;
    int pstride = 0;          // partial sums per right side
    int *d_again = nullptr;   // per right side: restart from the true residual
    int nbat = 0;             // right sides the solve buffers hold
    int nbat_vec = 0;         // vectors of each kind the solve buffers hold (1 for packed models)
    std::vector<std::pair<int, int>> seg_cache;   // per level: bricks and the tuned segment (4 or 8)
    int *d_ints = nullptr;    // small scratch ints
    int *h_ints = nullptr;    // pinned
    uint8_t *h_stage = nullptr;   // pinned staging for the host-built tables of the hierarchy
    size_t stage_cap = 0;
    // the library's own stream (all work) and the caller's stream it follows
    hipStream_t user_stream = nullptr;
    hipEvent_t ev_user = nullptr;
    // captured CG iterations (one per slot of the host ring), replayed with hipGraphLaunch
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        const Scal *mirror = nullptr;
        long long launch[SPFD_K_COUNT] = {};
        double bytes[SPFD_K_COUNT] = {};
    };
    StepGraph sg[2];
    int sg_nb = -1, sg_max_iter = -1, sg_flexible = -1;
    bool cg_flexible = false;   // beta of the CG: flexible (-alpha z.q / (r.z)_old) or standard (r.z / (r.z)_old)
    const Scal *sg_sc = nullptr;
    StepGraph *capturing = nullptr;
    int step_ctx = 0;   // 0: outside the CG loop, 1: in an untimed CG step, 2: in the sampled step
    bool r32_ready = false;   // d_r32 holds the FP32 copy of the residual the next CG start reads
    bool bscale0 = false;     // the running cycle's finest-level right side is held as D^-1 b (OpArgs::bscale)
    // per-class launch timing (tracing aid); cold: a flush of d_flush before every timed launch
    unsigned tmask = 0;
    bool tcold = false;
    void *d_flush = nullptr;
    std::vector<void *> flush_allocs;
    std::vector<hipEvent_t> tev[SPFD_K_COUNT];
    size_t tused[SPFD_K_COUNT] = {};
    long long tlaunch[SPFD_K_COUNT] = {};
    double tbytes[SPFD_K_COUNT] = {};
    long long ttimed[SPFD_K_COUNT] = {};    // launches with events, and their bytes
    double ttbytes[SPFD_K_COUNT] = {};
    // bookkeeping: live allocations per owner, and released buffers kept for
    // reuse (a rebuild with the same geometry allocates nothing)
    std::vector<void *> geo_allocs, hier_allocs, rhs_allocs, src_allocs;
    std::vector<std::pair<size_t, void *>> pool;
    std::vector<std::pair<void *, size_t>> sizes;
    size_t bytes = 0;
    // device memory of the handle: the caller's allocator if given, else hipMalloc / hipFree
    spfd_allocator alloc{};
};

struct HipFail {
    hipError_t e;
    const char *what;
};

#define HIPCHK(...)                                                  \
    do {                                                             \
        hipError_t e_ = (__VA_ARGS__);                               \
        if (e_ != hipSuccess) throw HipFail{e_, #__VA_ARGS__};       \
    } while (0)

void drop_graphs(Ctx *c);

// method / restart of the solve options (nrhs: right sides solved together)
const char *check_method(spfd_solve_options &so, int nrhs)
{
    if (so.method != SPFD_CG && so.method != SPFD_FGMRES) return "unknown method (SPFD_CG or SPFD_FGMRES)";
    if (so.method == SPFD_FGMRES) {
        if (so.restart == 0) so.restart = 30;
        if (so.restart < 1 || so.restart > FG_MAXM) return "restart must be in 1..32";
        if (nrhs != 1) return "FGMRES solves one right side per handle";
    }
    return nullptr;
}

}  // namespace

LaunchEvents &spfd::next_launch_events()
{
    static thread_local LaunchEvents ev;
    return ev;
}

namespace {

// order the library's stream after the work the caller has queued on its stream
void enter(Ctx *c)
{
    HIPCHK(hipEventRecord(c->ev_user, c->user_stream));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_user, 0));
}

size_t size_of(Ctx *c, void *p)
{
    for (auto &q : c->sizes)
        if (q.first == p) return q.second;
    return 0;
}

// one device buffer from the caller's allocator or hipMalloc, and its release
hipError_t raw_alloc(Ctx *c, void **p, size_t bytes)
{
    if (c->alloc.alloc) {
        *p = c->alloc.alloc(bytes, c->alloc.user);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

void raw_free(Ctx *c, void *p)
{
    if (c->alloc.alloc)
        c->alloc.free(p, c->alloc.user);
    else
        (void)hipFree(p);
}

template <typename T>
T *dalloc(Ctx *c, std::vector<void *> &owner, size_t count)
{
    size_t bytes = count * sizeof(T);
    bytes = bytes == 0 ? 256 : (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    for (size_t i = 0; i < c->pool.size(); ++i)
        if (c->pool[i].first == bytes) {
            p = c->pool[i].second;
            c->pool.erase(c->pool.begin() + i);
            break;
        }
    if (!p) {
        hipError_t e = raw_alloc(c, &p, bytes);
        if (e != hipSuccess) {
            // give the cached buffers back and try once more
            for (auto &q : c->pool) {
                raw_free(c, q.second);
                for (size_t i = 0; i < c->sizes.size(); ++i)
                    if (c->sizes[i].first == q.second) {
                        c->sizes.erase(c->sizes.begin() + i);
                        break;
                    }
            }
            c->pool.clear();
            e = raw_alloc(c, &p, bytes);
            if (e != hipSuccess) throw HipFail{e, "device allocation"};
        }
        c->sizes.push_back({p, bytes});
    }
    owner.push_back(p);
    c->bytes += bytes;
    return (T *)p;
}

// release an owner's buffers into the reuse pool
void free_all(Ctx *c, std::vector<void *> &owner)
{
    for (void *p : owner) {
        const size_t b = size_of(c, p);
        c->bytes -= b;
        c->pool.push_back({b, p});
    }
    owner.clear();
}

// return every buffer to the device
void release_device(Ctx *c)
{
    free_all(c, c->flush_allocs);
    c->d_flush = nullptr;
    free_all(c, c->src_allocs);
    free_all(c, c->rhs_allocs);
    free_all(c, c->hier_allocs);
    free_all(c, c->geo_allocs);
    for (auto &q : c->pool) raw_free(c, q.second);
    c->pool.clear();
    c->sizes.clear();
    c->bytes = 0;
}

spfd_status fail(Ctx *c, spfd_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

// Brackets one launch of kernel class `cls` with HIP events when timing is on
// for that class, and adds the launch's algorithmic bytes to the class counter.
constexpr size_t FLUSH_BYTES = (size_t)1 << 30;   // four times the Infinity Cache

struct TScope {
    Ctx *c;
    int cls;
    bool on;
    TScope(Ctx *c_, int cls_, double bytes)
        : c(c_), cls(cls_), on(((c_->tmask >> cls_) & 1u) && !c_->capturing && c_->step_ctx != 1)
    {
        if (c->capturing) {
            // counted once per replay of the graph being captured
            c->capturing->launch[cls] += 1;
            c->capturing->bytes[cls] += bytes;
            return;
        }
        c->tlaunch[cls] += 1;
        c->tbytes[cls] += bytes;
        if (on) {
            // cold timing: the caches are flushed first (outside the timed interval)
            if (c->tcold && c->d_flush) (void)launch_flush(c->d_flush, FLUSH_BYTES, c->stream);
            // the launch inside the scope records both events itself
            hipEvent_t e0 = event(), e1 = event();
            if (!e0 || !e1) {
                on = false;
                return;
            }
            c->tused[cls] += 2;
            c->ttimed[cls] += 1;
            c->ttbytes[cls] += bytes;
            next_launch_events() = LaunchEvents{e0, e1};
            this->bytes = bytes;
        }
    }
    ~TScope()
    {
        if (on && next_launch_events().start) {
            // nothing was launched in the scope: drop the sample
            next_launch_events() = LaunchEvents{};
            c->tused[cls] -= 2;
            c->ttimed[cls] -= 1;
            c->ttbytes[cls] -= bytes;
        }
    }
    double bytes = 0.0;
    hipEvent_t event()
    {
        std::vector<hipEvent_t> &v = c->tev[cls];
        while (v.size() < c->tused[cls] + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            v.push_back(e);
        }
        return v[c->tused[cls] + (next_pending++)];
    }
    int next_pending = 0;
};

// packed voxel models start at node layers that are multiples of this, one empty layer apart at least
constexpr int MODEL_ALIGN = 64;

// ------------------------------------------------------------ brick topology on the host
// Pinned staging of at least `bytes` (copies from pageable memory go through a
// slow bounce buffer).  Call only while nothing in the stream uses the previous area.
uint8_t *stage(Ctx *c, size_t bytes)
{
    if (bytes > c->stage_cap) {
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->h_stage) (void)hipHostFree(c->h_stage);
        c->h_stage = nullptr;
        c->stage_cap = 0;
        const size_t cap = std::max<size_t>(bytes, (size_t)4 << 20);
        HIPCHK(hipHostMalloc((void **)&c->h_stage, cap, hipHostMallocDefault));
        c->stage_cap = cap;
    }
    return c->h_stage;
}

void build_topology(Ctx *c, Level &L, const std::vector<uint8_t> &flags, std::vector<void *> &owner)
{
    const int G0 = L.G[0], G1 = L.G[1], G2 = L.G[2];
    L.slot_of.assign((size_t)G0 * G1 * G2, -1);
    L.coord.clear();
    // slots in brick-grid order (x fastest): neighbours along x are adjacent slots
    for (int bz = 0; bz < G2; ++bz)
        for (int by = 0; by < G1; ++by)
            for (int bx = 0; bx < G0; ++bx) {
                const size_t id = bx + (size_t)G0 * (by + (size_t)G1 * bz);
                if (flags[id]) {
                    L.slot_of[id] = (int)L.coord.size();
                    L.coord.push_back(make_int4(bx, by, bz, 0));
                }
            }
    L.nb = (int)L.coord.size();
    std::vector<int> nbr((size_t)L.nb * 6 + 6, -1);
    auto look = [&](int x, int y, int z) -> int {
        if (x < 0 || y < 0 || z < 0 || x >= G0 || y >= G1 || z >= G2) return -1;
        return L.slot_of[x + (size_t)G0 * (y + (size_t)G1 * z)];
    };
    for (int s = 0; s < L.nb; ++s) {
        const int4 q = L.coord[s];
        nbr[s * 6 + NMX] = look(q.x - 1, q.y, q.z);
        nbr[s * 6 + NPX] = look(q.x + 1, q.y, q.z);
        nbr[s * 6 + NMY] = look(q.x, q.y - 1, q.z);
        nbr[s * 6 + NPY] = look(q.x, q.y + 1, q.z);
        nbr[s * 6 + NMZ] = look(q.x, q.y, q.z - 1);
        nbr[s * 6 + NPZ] = look(q.x, q.y, q.z + 1);
    }
    L.d_slot_of = dalloc<int>(c, owner, L.slot_of.size());
    L.d_nbr = dalloc<int>(c, owner, nbr.size());
    L.d_coord = dalloc<int4>(c, owner, L.coord.size() + 1);
    // the three tables through one pinned staging area
    const size_t b0 = L.slot_of.size() * sizeof(int), b1 = nbr.size() * sizeof(int),
                 b2 = L.coord.size() * sizeof(int4);
    const size_t o1 = (b0 + 255) & ~(size_t)255, o2 = o1 + ((b1 + 255) & ~(size_t)255);
    uint8_t *st = stage(c, o2 + b2);
    memcpy(st, L.slot_of.data(), b0);
    memcpy(st + o1, nbr.data(), b1);
    if (b2) memcpy(st + o2, L.coord.data(), b2);
    HIPCHK(hipMemcpyAsync(L.d_slot_of, st, b0, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(L.d_nbr, st + o1, b1, hipMemcpyHostToDevice, c->stream));
    if (L.nb) HIPCHK(hipMemcpyAsync(L.d_coord, st + o2, b2, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
}

__global__ void k_count_dofs(const double *w, long long stride, Topo topo, int *count)
{
    __shared__ int nb[6];
    __shared__ int cnt;
    const int b = blockIdx.x, t = threadIdx.x;
    if (t < 6) nb[t] = topo.nbr[b * 6 + t];
    if (t == 0) cnt = 0;
    __syncthreads();
    int tx, ty, tz;
    brick_xyz(t, tx, ty, tz);
    double W[6];
    long long I[6];
    nbr_index((long long)b * BS, t, tx, ty, tz, nb, I);
    stored_weights(w, stride, (long long)b * BS, t, I, W);
    if (diag_of(W) > 0.0) atomicAdd(&cnt, 1);
    __syncthreads();
    if (t == 0 && cnt) atomicAdd(count, cnt);
}

// rows of an ELL level with a positive diagonal (the sum of the row's stored entries, in the order the
// enumeration of the coarsest level uses), counted by many workgroups
__global__ __launch_bounds__(256) void k_count_ell_dofs(int n, int K, const int *__restrict__ col,
                                                        const double *__restrict__ val, int *count)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double d = 0.0;
        for (int k = 0; k < K; ++k)
            if (col[(long long)k * n + i] >= 0) d += val[(long long)k * n + i];
        if (d > 0.0) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(count, cnt);
}

long long count_dofs(Ctx *c, const Level &L)
{
    HIPCHK(hipMemsetAsync(c->d_ints, 0, sizeof(int), c->stream));
    if (L.nb > 0) hipLaunchKernelGGL(k_count_dofs, dim3(L.nb), dim3(NT), 0, c->stream, L.d_w64, L.nodes(), L.topo(), c->d_ints);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_ints, c->d_ints, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return c->h_ints[0];
}

template <typename T>
OpArgs<T> level_op(Ctx *c, int l);

template <>
OpArgs<double> level_op<double>(Ctx *c, int l)
{
    OpArgs<double> op{};
    const Level &L = c->lv[l];
    op.stride = L.nodes();
    op.short_below = c->opt.short_segment_bricks;
    if (l == 0 && !c->voxel_mode) {
        op.w = nullptr;
        op.tiles = L.d_tiles;
        op.table = c->d_table64;
        op.nlab = c->nlab;
        for (int d = 0; d < 3; ++d) op.geo4[d] = c->geo4[d];
    } else {
        op.w = L.d_w64;
    }
    return op;
}

template <>
OpArgs<float> level_op<float>(Ctx *c, int l)
{
    OpArgs<float> op{};
    const Level &L = c->lv[l];
    op.stride = L.nodes();
    op.short_below = L.seg == 4 ? 0x7fffffff : L.seg == 8 ? 0 : c->opt.short_segment_bricks;
    if (l == 0 && !c->voxel_mode) {
        op.w = nullptr;
        op.tiles = L.d_tiles;
        op.table = c->d_table32;
        op.nlab = c->nlab;
        for (int d = 0; d < 3; ++d) op.geo4[d] = (float)c->geo4[d];
        op.bscale = c->bscale0 ? 1 : 0;
    } else {
        op.w = L.d_w32;
        if (l == 1 && L.d_w16) {
            op.wh = L.d_w16;
            op.whs = L.w16s;
        }
    }
    return op;
}

// ------------------------------------------------------------ the multigrid cycle
// algorithmic bytes per unknown of the operator: 1 label byte on the finest
// level in label form, otherwise the three stored weights of the node
template <typename T>
double op_bytes(Ctx *c, int l)
{
    if (l == 0 && !c->voxel_mode) return 1.0;
    if (sizeof(T) == sizeof(float) && l == 1 && c->lv[1].d_w16) return 3.0 * sizeof(uint16_t);
    return 3.0 * sizeof(T);
}

// The FP32 copy of the outer residual that an FP32 cycle reads is held as D^-1 r where the finest level is
// in label form and the cycle has more than one level: its first two smoothing steps then read no inverse
// diagonal (the kernels form D r where they need r).  Written so by the solve start and the residual update
// of the standard-beta CG.
bool r32_scaled(const Ctx *c)
{
    return c->opt.precision == SPFD_MIXED && !c->voxel_mode && c->lv.size() > 1 && c->lv[0].d_dinv32 != nullptr;
}

template <typename T>
const T *ell_val(const Level &L);
template <>
const double *ell_val<double>(const Level &L) { return L.d_val64; }
template <>
const float *ell_val<float>(const Level &L) { return L.d_val32; }

Batch level_batch(Ctx *c, int l, int n)
{
    Batch bt;
    bt.n = n;
    bt.vs = c->lv[l].nodes();
    bt.vsc = l + 1 < (int)c->lv.size() ? c->lv[l + 1].nodes() : 0;
    bt.ps = c->pstride;
    return bt;
}

template <typename T, typename TB>
void cheb_first(Ctx *c, int l, const TB *b, T *x, const Scal *sc, int nb)
{
    Level &L = c->lv[l];
    const Batch bt = level_batch(c, l, nb);
    if (L.ell) {
        TScope ts(c, SPFD_K_COARSE, nb * (double)L.nrow * (2.0 * sizeof(T) + L.K * (4.0 + sizeof(T))));
        HIPCHK(launch_ell_cheb_first<T>(L.nrow, L.K, L.d_col, ell_val<T>(L), (const T *)b, x, (T)c->cheb_c0, sc, bt,
                                        c->stream));
        return;
    }
    const double by = nb * (double)L.dofs * (sizeof(TB) + op_bytes<T>(c, l) + sizeof(T));
    TScope ts(c, l == 0 ? SPFD_K_SMOOTH0_FIRST : SPFD_K_COARSE, by);
    HIPCHK(launch_cheb_first<T, TB>(level_op<T>(c, l), L.topo(), b, x, (T)c->cheb_c0, sc, bt, c->stream));
}

// with_prolong: the step first adds coarse_scale * P x_c of the structured
// level l+1 to xin (the prolongation fused into the first post-smoothing step)
template <typename T>
const T *dinv_of(const Level &L);
template <>
const double *dinv_of<double>(const Level &L) { return L.d_dinv64; }
template <>
const float *dinv_of<float>(const Level &L) { return L.d_dinv32; }

// CG dot products formed by the last finest-level smoothing step: z.b with
// the cycle's right side b (the residual, or its FP32 copy in an FP32 cycle)
// and z.q
struct CycleDots {
    const double *q = nullptr;
    double *part = nullptr;
};

// dmode (structured levels): where the step takes the previous update from (CHEB_D_*); the ELL levels
// always use din / dout
template <typename T, typename TB>
void cheb_step(Ctx *c, int l, const TB *b, const T *xin, T *xout, const T *din, T *dout, T c1, T c2, const Scal *sc,
               int nb, bool with_prolong = false, const CycleDots *dots = nullptr, int dmode = CHEB_D_AUTO)
{
    Level &L = c->lv[l];
    const Batch bt = level_batch(c, l, nb);
    if (L.ell) {
        TScope ts(c, SPFD_K_COARSE, nb * (double)L.nrow * (4.0 * sizeof(T) + L.K * (4.0 + sizeof(T))));
        const bool pro = with_prolong && c->lv[l + 1].ell;
        HIPCHK(launch_ell_cheb_step<T>(L.nrow, L.K, L.d_col, ell_val<T>(L), (const T *)b, xin, xout, din, dout, c1, c2,
                                       sc, bt, c->stream, pro ? L.d_agg : nullptr,
                                       pro ? (const T *)c->lv[l + 1].x : nullptr, (T)c->opt.coarse_scale));
        return;
    }
    const bool prev = dmode == CHEB_D_PREV || dmode == CHEB_D_PREV_PRO;
    double per = sizeof(TB) + op_bytes<T>(c, l) + sizeof(T) * (2 + (din || prev ? 1 : 0) + (dout ? 1 : 0));
    if (with_prolong || dmode == CHEB_D_PREV_PRO) per += sizeof(T) / 8.0;
    if (dots && dots->q) per += 8.0;
    const int cls = l == 0 ? (with_prolong ? SPFD_K_PROLONG0 : dots ? SPFD_K_DOTS : SPFD_K_SMOOTH0) : SPFD_K_COARSE;
    TScope ts(c, cls, nb * (double)L.dofs * per);
    const T *xc = nullptr;
    if (with_prolong || dmode == CHEB_D_PREV_PRO) xc = (const T *)c->lv[l + 1].x;
    HIPCHK(launch_cheb_step<T, TB>(level_op<T>(c, l), L.topo(), b, xin, xout, din, dout, c1, c2, sc, bt, c->stream, xc,
                                   L.d_parent_slot, L.d_coord, (T)c->opt.coarse_scale, dots ? dots->q : nullptr,
                                   dots ? dots->part : nullptr, dmode));
}

// Chebyshev degree of level l (any degree keeps the buffer parity of the
// cycle: a level does 2m-1 buffer swaps)
int level_degree(const Ctx *c, int l)
{
    return l == 1 ? c->opt.level1_degree : c->opt.smooth_degree;
}

template <typename T, typename TB>
void smooth_pre(Ctx *c, int l, const TB *b, T *&cur, T *&other, const Scal *sc, int nb, bool first_done)
{
    // first_done: the restriction that produced b already stored the first step in cur
    const int m = level_degree(c, l);
    T *d = (T *)c->lv[l].d;
    int k0 = 1;
    if (!first_done && l == 0 && m >= 2) {
        // the first two steps in one pass on the finest level (x1 formed where read: one kernel and one
        // write and read of x1 less; 53 -> 45 us per cycle on the body phantom)
        Level &L = c->lv[0];
        // b, the operator, the inverse diagonal (none with a scaled b) and the output
        TScope ts(c, SPFD_K_SMOOTH0, nb * (double)L.dofs * (sizeof(TB) + op_bytes<T>(c, 0) +
                                                            (c->bscale0 ? 1.0 : 2.0) * sizeof(T)) +
                                         nb * (double)L.dofs * (m > 2 ? sizeof(T) : 0.0));
        HIPCHK(launch_cheb_first2<T, TB>(level_op<T>(c, 0), L.topo(), b, dinv_of<T>(L), other, m > 2 ? d : nullptr,
                                         (T)c->cheb_c0, (T)c->cheb_c1[1], (T)c->cheb_c2[1], sc, level_batch(c, 0, nb),
                                         c->stream));
        T *t = cur; cur = other; other = t;
        k0 = 2;
    } else if (!first_done) {
        cheb_first<T, TB>(c, l, b, cur, sc, nb);
    }
    // On the structured levels no step stores its update d: the buffer a step writes holds the iterate
    // before its input (ping-pong), from which the step forms d itself.  The first two finest steps in one
    // pass never store x1, so they store d for the third step (degree > 2).
    const bool ell = c->lv[l].ell;
    for (int k = k0; k < m; ++k) {
        if (ell) {
            cheb_step<T, TB>(c, l, b, cur, other, k == 1 ? nullptr : d, k < m - 1 ? d : nullptr, (T)c->cheb_c1[k],
                             (T)c->cheb_c2[k], sc, nb);
        } else {
            const int dm = k == 1 ? CHEB_D_FROM_X : (k0 == 2 && k == 2 ? CHEB_D_STORED : CHEB_D_PREV);
            cheb_step<T, TB>(c, l, b, cur, other, dm == CHEB_D_STORED ? d : nullptr, nullptr, (T)c->cheb_c1[k],
                             (T)c->cheb_c2[k], sc, nb, false, nullptr, dm);
        }
        T *t = cur; cur = other; other = t;
    }
}

template <typename T, typename TB>
void smooth_post(Ctx *c, int l, const TB *b, T *&cur, T *&other, const Scal *sc, int nb, bool with_prolong,
                 const CycleDots *dots = nullptr)
{
    const int m = level_degree(c, l);
    T *d = (T *)c->lv[l].d;
    const bool ell = c->lv[l].ell;
    for (int k = 0; k < m; ++k) {
        const T c1 = k == 0 ? T(0) : (T)c->cheb_c1[k];
        const T c2 = k == 0 ? (T)c->cheb_c0 : (T)c->cheb_c2[k];
        if (ell) {
            cheb_step<T, TB>(c, l, b, cur, other, k == 0 ? nullptr : d, k < m - 1 ? d : nullptr, c1, c2, sc, nb,
                             with_prolong && k == 0, k == m - 1 ? dots : nullptr);
        } else {
            // the first step needs no d (c1 = 0); the second finds the pre-smoothed iterate in its output
            // buffer, without the coarse-grid correction if the first step applied it on the fly
            const int dm = k == 0 ? CHEB_D_FROM_X : (k == 1 && with_prolong ? CHEB_D_PREV_PRO : CHEB_D_PREV);
            cheb_step<T, TB>(c, l, b, cur, other, nullptr, nullptr, c1, c2, sc, nb, with_prolong && k == 0,
                             k == m - 1 ? dots : nullptr, dm);
        }
        T *t = cur; cur = other; other = t;
    }
}

template <typename T>
const T *stored_w(const Level &L);
template <>
const double *stored_w<double>(const Level &L) { return L.d_w64; }
template <>
const float *stored_w<float>(const Level &L) { return L.d_w32; }

template <typename T, typename TB>
void restrict_level(Ctx *c, int l, const TB *b, const T *x, const Scal *sc, int nb, bool fuse_first)
{
    // fuse_first: also the first Chebyshev step of level l+1 into its x2 (where its smoothing starts)
    Level &L = c->lv[l];
    Level &C = c->lv[l + 1];
    const Batch bt = level_batch(c, l, nb);
    T *xc = fuse_first ? (T *)C.x2 : nullptr;
    const T *dc = fuse_first ? dinv_of<T>(C) : nullptr;
    const T c0 = (T)c->cheb_c0;
    const double fb = fuse_first ? nb * (double)C.dofs * 2.0 * sizeof(T) : 0.0;
    if (C.ell) {
        FineLevelT<T> f{};
        if (L.ell) {
            f.n = L.nrow;
            f.K = L.K;
            f.col = L.d_col;
            f.val = ell_val<T>(L);
        } else {
            f.w = stored_w<T>(L);
            f.stride = L.nodes();
            f.nbr = L.d_nbr;
        }
        TScope ts(c, SPFD_K_COARSE, nb * ((double)L.dofs * 3.0 * sizeof(T) + (double)C.nrow * 8.0) + fb);
        HIPCHK(launch_restrict_members<T>(f, L.nodes(), (const T *)b, x, C.nrow, C.d_mptr, C.d_mem,
                                          (T *)C.b, sc, bt, c->stream, xc, dc, c0, C.d_memb));
        return;
    }
    const double by = nb * ((double)L.dofs * (sizeof(TB) + op_bytes<T>(c, l) + sizeof(T)) + (double)C.dofs * sizeof(T));
    TScope ts(c, l == 0 ? SPFD_K_RESTRICT0 : SPFD_K_COARSE, by + fb);
    HIPCHK(launch_resid_restrict<T, TB>(level_op<T>(c, l), L.topo(), b, x, (T *)C.b, L.d_parent_slot, L.d_coord, sc, bt,
                                        c->stream, xc, dc, c0));
}

template <typename T>
void prolong_level(Ctx *c, int l, T *x, const Scal *sc, int nb)
{
    Level &L = c->lv[l];
    Level &C = c->lv[l + 1];
    const Batch bt = level_batch(c, l, nb);
    if (C.ell) {
        TScope ts(c, SPFD_K_COARSE, nb * (double)L.nodes() * (2.0 * sizeof(T) + 4.0));
        HIPCHK(launch_prolong_agg<T>(L.nodes(), L.d_agg, x, (const T *)C.x, (T)c->opt.coarse_scale, sc, bt, c->stream));
        return;
    }
    const double by = nb * ((double)L.dofs * 2.0 * sizeof(T) + (double)C.dofs * sizeof(T));
    TScope ts(c, l == 0 ? SPFD_K_PROLONG0 : SPFD_K_COARSE, by);
    HIPCHK(launch_prolong<T>(L.topo(), x, (const T *)C.x, L.d_parent_slot, L.d_coord, (T)c->opt.coarse_scale, sc, bt,
                             c->stream));
}

template <typename T, typename TB>
void coarse_solve(Ctx *c, const TB *b, T *x, const Scal *sc, int nb)
{
    const double n = (double)c->ncoarse;
    const Batch bt = level_batch(c, (int)c->lv.size() - 1, nb);
    TScope ts(c, SPFD_K_COARSE, n * n * 8.0 + nb * n * (sizeof(TB) + sizeof(T)));
    HIPCHK(launch_coarse_apply<T, TB>(b, x, c->d_Ainv, c->d_cdof_node, c->ncoarse, sc, bt, c->stream));
}

// z = B r for a batch of nb right sides: one V-cycle (T = arithmetic of the
// cycle); r is the outer residual (FP64, or its FP32 copy for an FP32 cycle)
// dots (optional): the finest post-smoothing step also writes the partials of
// z.r and z.q (cheb_dot_parts<T> per right side); returns false when the
// cycle has no smoothing step to carry them (single level)
// bs: r is the scaled FP32 copy D^-1 r (r32_scaled)
template <typename T, typename TR>
bool vcycle(Ctx *c, const TR *r, T *z, const Scal *sc, int nb, const CycleDots *dots = nullptr, bool bs = false)
{
    const int nl = (int)c->lv.size();
    std::vector<T *> res(nl, nullptr);
    if (bs && !(sizeof(T) == sizeof(float) && sizeof(TR) == sizeof(float) && r32_scaled(c)))
        throw HipFail{hipErrorInvalidValue, "scaled right side outside an FP32 cycle in label form"};
    struct ScaleScope {
        Ctx *c;
        ScaleScope(Ctx *c_, bool v) : c(c_) { c->bscale0 = v; }
        ~ScaleScope() { c->bscale0 = false; }
    } scs(c, bs);
    // the stencil kernels read a stop flag per launch row: a cycle outside a CG step never stops
    if (!sc) {
        if (!c->d_nostop || nb > c->nbat) throw HipFail{hipErrorInvalidValue, "cycle without scalars"};
        sc = c->d_nostop;
    }
    if (nl == 1) {
        coarse_solve<T, TR>(c, r, z, sc, nb);  // single level: the dense solve is exact
        return false;
    }
    // downward: pre-smooth, restrict the residual.  The smoother ping-pongs
    // between two buffers; starting in x2 makes the (2m-1) swaps of a level end
    // in the level's output buffer (z on the finest level, x below).
    for (int l = 0; l < nl - 1; ++l) {
        Level &L = c->lv[l];
        T *cur = (T *)L.x2;
        T *other = l == 0 ? z : (T *)L.x;
        // the restriction stores the next level's first Chebyshev step unless that level is the coarsest
        const bool fuse = l + 2 < nl;
        if (l == 0) {
            smooth_pre<T, TR>(c, l, r, cur, other, sc, nb, false);
            restrict_level<T, TR>(c, l, r, cur, sc, nb, fuse);
        } else {
            smooth_pre<T, T>(c, l, (const T *)L.b, cur, other, sc, nb, true);
            restrict_level<T, T>(c, l, (const T *)L.b, cur, sc, nb, fuse);
        }
        res[l] = cur;
    }
    {
        Level &C = c->lv[nl - 1];
        coarse_solve<T, T>(c, (const T *)C.b, (T *)C.x, sc, nb);
    }
    // upward: prolongate and correct, post-smooth
    for (int l = nl - 2; l >= 0; --l) {
        Level &L = c->lv[l];
        T *cur = res[l];
        T *other = (cur == (T *)L.x2) ? (l == 0 ? z : (T *)L.x) : (T *)L.x2;
        // between two structured or two ELL levels the prolongation rides on the first post-smoothing step
        const bool fused = L.ell == c->lv[l + 1].ell;
        if (!fused) prolong_level<T>(c, l, cur, sc, nb);
        if (l == 0)
            smooth_post<T, TR>(c, l, r, cur, other, sc, nb, fused, dots);
        else
            smooth_post<T, T>(c, l, (const T *)L.b, cur, other, sc, nb, fused);
        T *want = l == 0 ? z : (T *)L.x;
        if (cur != want)
            HIPCHK(hipMemcpyAsync(want, cur, nb * L.nodes() * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    }
    return dots != nullptr;
}

// Partial sums of the CG kernels per launch row: packed models write one row per model, of the model's
// own count (bricks, or groups of the CG step), and the finisher sums just those.
enum { ROWS_BRICKS = 1, ROWS_CG_GROUPS = 2, ROWS_RU_GROUPS = 3 };

void finish(Ctx *c, int n, int mode, Scal *sc, int max_iter, int nb = 1, Scal *mirror = nullptr, int rows = 0)
{
    TScope ts(c, SPFD_K_FINISH, nb * (double)n * 8.0 * (mode == FIN_BETA ? 2 : 1));
    FinRows fr{};
    if (c->np && rows) {
        fr.used = 1;
        for (int m = 0; m < c->np; ++m)
            fr.n[m] = rows == ROWS_BRICKS      ? c->mcount[m]
                      : rows == ROWS_RU_GROUPS ? rupdate_parts(c->mcount[m])
                                               : cg_step_parts(c->mcount[m]);
    }
    HIPCHK(launch_finish(c->d_part, n, mode, sc, max_iter, c->stream, nullptr, nullptr, 0, nb, c->pstride, mirror,
                         fr.used ? &fr : nullptr));
}

// The finest level as the CG kernels see it: all bricks, or one launch row per packed model (its bricks,
// its scalars, its partial sums; the vectors are shared, so no per-row offset)
Topo cg_topo(Ctx *c)
{
    Topo t = c->lv[0].topo();
    if (c->np) {
        t.np = c->np;
        t.prange = c->d_mrange;
        for (int m = 0; m < c->np; ++m) t.pmax = std::max(t.pmax, c->mcount[m]);
    }
    return t;
}

Batch cg_batch(Ctx *c, int nb)
{
    Batch bt = level_batch(c, 0, nb);
    if (c->np) bt.vs = bt.vsc = 0;
    return bt;
}

void set_defaults(spfd_amg_options &o)
{
    if (o.precision != SPFD_MIXED) o.precision = SPFD_FP64;
    if (o.smooth_degree <= 0) o.smooth_degree = 2;
    if (o.smooth_degree > 4) o.smooth_degree = 4;
    if (o.coarsest_max <= 0) o.coarsest_max = 1024;
    if (o.coarsest_max > 1024) o.coarsest_max = 1024;
    if (!(o.cheby_ratio > 1.0)) o.cheby_ratio = 8.0;
    if (!(o.coarse_scale > 0.0)) o.coarse_scale = 1.9;
    if (o.split_level <= 0) o.split_level = 2;
    if (o.level1_degree <= 0) o.level1_degree = 4;
    if (o.level1_degree > 8) o.level1_degree = 8;
    // 0: tuned per level at build (the threshold below stands until then); < 0: 8-node segments everywhere
    if (o.short_segment_bricks == 0) o.short_segment_bricks = 8192;
    if (o.short_segment_bricks < 0) o.short_segment_bricks = 0;
}

// Step k of a smoothing pass is d_k = c1[k] d_{k-1} + c2[k] D^-1 (b - A x),
// x += d_k (the first, from x = 0: x = c0 D^-1 b).  Chebyshev on [lmax/ratio,
// lmax] of D^-1 A with lmax = 2 (the largest eigenvalue of D^-1 A for a
// weighted graph Laplacian on a bipartite grid graph); l1-Jacobi is
// c1 = 0, c2 = c0 = 1/2, since the l1 norm of every row is twice its diagonal.
void chebyshev_coefficients(Ctx *c)
{
    c->cheb_c1.assign(8, 0.0);
    c->cheb_c2.assign(8, 0.0);
    if (c->opt.smoother == SPFD_SMOOTH_CHEBYSHEV4) {
        // Chebyshev polynomial of the fourth kind in D^-1 A on [0, lmax] (no lower bound): the error
        // polynomial p_m satisfies max |p_m(l)| sqrt(l / lmax) = 1 / (2m + 1) on [0, lmax]
        const double rho = 2.0;
        c->cheb_c0 = 4.0 / (3.0 * rho);
        for (int k = 1; k < 8; ++k) {
            c->cheb_c1[k] = (2.0 * k - 1.0) / (2.0 * k + 3.0);
            c->cheb_c2[k] = (8.0 * k + 4.0) / ((2.0 * k + 3.0) * rho);
        }
        return;
    }
    if (c->opt.smoother == SPFD_SMOOTH_L1_JACOBI) {
        c->cheb_c0 = 0.5;
        for (int k = 1; k < 8; ++k) c->cheb_c2[k] = 0.5;
        return;
    }
    const double lmax = 2.0, lmin = lmax / c->opt.cheby_ratio;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma1 = theta / delta;
    c->cheb_c0 = 1.0 / theta;
    double rho_prev = 1.0 / sigma1;
    for (int k = 1; k < 8; ++k) {
        const double rho = 1.0 / (2.0 * sigma1 - rho_prev);
        c->cheb_c1[k] = rho * rho_prev;
        c->cheb_c2[k] = 2.0 * rho / delta;
        rho_prev = rho;
    }
}

// The column segment of every structured level with stored weights in an FP32
// cycle (4 or 8 nodes per lane): both variants of one Chebyshev step are timed
// on the level's own buffers (best of three after a warm-up each) and the
// faster one is kept for every kernel of that level.  Both compute each node
// the same way, so the choice changes the speed only, never a result.
void tune_segments(Ctx *c)
{
    if (c->opt.precision != SPFD_MIXED) return;
    // levels to tune: structured, stored weights, smoothed; a level of the same brick count as at the
    // last tuning of this handle keeps its choice (a rebuild with new conductivities, same geometry)
    std::vector<int> todo;
    for (size_t l = 0; l + 1 < c->lv.size(); ++l) {
        Level &L = c->lv[l];
        L.seg = 0;
        if (L.ell || (l == 0 && !c->voxel_mode) || L.nb <= 0) continue;
        if (l < c->seg_cache.size() && c->seg_cache[l].first == L.nb) {
            L.seg = c->seg_cache[l].second;
            continue;
        }
        todo.push_back((int)l);
    }
    if (todo.empty()) return;
    constexpr int REPS = 3;   // per variant, after one warm-up launch; variants alternate
    std::vector<hipEvent_t> ev(todo.size() * 2 * (REPS + 1) * 2, nullptr);
    for (hipEvent_t &e : ev) HIPCHK(hipEventCreate(&e));
    size_t k = 0;
    for (int l : todo) {
        Level &L = c->lv[l];
        for (int rep = 0; rep <= REPS; ++rep)
            for (int v = 0; v < 2; ++v) {
                L.seg = v == 0 ? 4 : 8;
                HIPCHK(hipEventRecord(ev[k++], c->stream));
                HIPCHK(launch_cheb_step<float, float>(level_op<float>(c, l), L.topo(), (const float *)L.b,
                                                      (const float *)L.x, (float *)L.x2, (const float *)L.d, nullptr,
                                                      0.5f, 0.5f, c->d_nostop, level_batch(c, l, 1), c->stream));
                HIPCHK(hipEventRecord(ev[k++], c->stream));
            }
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    k = 0;
    for (int l : todo) {
        float best[2] = {1e30f, 1e30f};
        for (int rep = 0; rep <= REPS; ++rep)
            for (int v = 0; v < 2; ++v) {
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
                k += 2;
                if (rep > 0 && ms < best[v]) best[v] = ms;
            }
        Level &L = c->lv[l];
        L.seg = best[0] <= best[1] ? 4 : 8;
        if (c->seg_cache.size() <= (size_t)l) c->seg_cache.resize(l + 1, {-1, 0});
        c->seg_cache[l] = {L.nb, L.seg};
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    // the tuning steps wrote x2 (zeros, from zero inputs); cleared again all the same
    for (int l : todo) {
        Level &L = c->lv[l];
        HIPCHK(hipMemsetAsync(L.x2, 0, (size_t)L.nodes() * c->nbat_vec * sizeof(float), c->stream));
    }
}

// Zeroes up to ZL_MAX device ranges in one launch (one grid row per range),
// in place of one hipMemsetAsync per buffer: each memset call costs as much
// host time as a kernel launch.  Ranges start 16-byte aligned (every buffer
// here is a whole allocation) and hold whole 4-byte words.
constexpr int ZL_MAX = 32;
struct ZeroList {
    int n = 0;
    void *ptr[ZL_MAX];
    unsigned long long bytes[ZL_MAX];
};

__global__ __launch_bounds__(256) void k_zero_list(ZeroList zl)
{
    uint8_t *p = (uint8_t *)zl.ptr[blockIdx.y];
    const unsigned long long nb = zl.bytes[blockIdx.y];
    const unsigned long long n16 = nb / 16, t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (unsigned long long i = t; i < n16; i += (unsigned long long)gridDim.x * blockDim.x)
        ((uint4 *)p)[i] = make_uint4(0u, 0u, 0u, 0u);
    const unsigned long long tail = n16 * 16 + 4 * t;   // the last (< 16) bytes, one word per thread
    if (tail < nb) *(unsigned *)(p + tail) = 0u;
}

// queue zeroing of [p, p + bytes): into the list, or by memset when the list is full or the range does not
// fit the kernel's alignment
void zero_add(Ctx *c, ZeroList &zl, void *p, size_t bytes)
{
    if (!p || bytes == 0) return;
    if (zl.n == ZL_MAX || ((uintptr_t)p & 15) || (bytes & 3)) {
        HIPCHK(hipMemsetAsync(p, 0, bytes, c->stream));
        return;
    }
    zl.ptr[zl.n] = p;
    zl.bytes[zl.n] = bytes;
    ++zl.n;
}

void zero_flush(Ctx *c, ZeroList &zl)
{
    if (zl.n == 0) return;
    unsigned long long mx = 0;
    for (int i = 0; i < zl.n; ++i) mx = std::max(mx, zl.bytes[i]);
    const unsigned long long need = (mx / 16 + 255) / 256;
    const unsigned gx = (unsigned)std::max<unsigned long long>(1, std::min<unsigned long long>(need, 1024));
    hipLaunchKernelGGL(k_zero_list, dim3(gx, (unsigned)zl.n), dim3(256), 0, c->stream, zl);
    HIPCHK(hipGetLastError());
    zl.n = 0;
}

// Zeroes the node columns without unknowns (clear bits of each brick's column
// mask) of nv consecutive vectors of the finest level's layout, one wave per
// brick.  No kernel writes those slots, but the stencils of neighbouring
// columns read them (with conductance 0), so they must hold finite values.
template <typename T>
__global__ __launch_bounds__(256) void k_zero_empty_cols(const unsigned long long *__restrict__ cmask, int nb,
                                                         long long nodes, int nv, T *__restrict__ v)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= nb || ((cmask[b] >> lane) & 1ull)) return;
    T *p = v + (long long)b * BS + lane;
    for (int y = 0; y < nv; ++y, p += nodes)
#pragma unroll
        for (int z = 0; z < BD; ++z) p[64 * z] = T(0);
}

// solve buffers for nb right sides: cycle vectors of every level, the outer
// CG vectors and the partial sums
void alloc_cycle_buffers(Ctx *c, int nb)
{
    drop_graphs(c);
    free_all(c, c->rhs_allocs);
    c->d_fgV = nullptr;
    c->d_fgZ = nullptr;
    c->d_fgst = nullptr;
    c->d_fgpart = nullptr;
    c->fg_m = 0;
    const bool mixed = c->opt.precision == SPFD_MIXED;
    const size_t w = mixed ? sizeof(float) : sizeof(double);
    const int nvec = c->np ? 1 : nb;   // packed models share one vector of each kind
    c->nbat_vec = nvec;
    ZeroList zl;
    for (size_t l = 0; l < c->lv.size(); ++l) {
        Level &L = c->lv[l];
        const size_t n = (size_t)L.nodes() * nvec;
        L.x = dalloc<uint8_t>(c, c->rhs_allocs, n * w);
        L.x2 = dalloc<uint8_t>(c, c->rhs_allocs, n * w);
        L.d = dalloc<uint8_t>(c, c->rhs_allocs, n * w);
        L.b = dalloc<uint8_t>(c, c->rhs_allocs, n * w);
        zero_add(c, zl, L.x, n * w);
        zero_add(c, zl, L.x2, n * w);
        zero_add(c, zl, L.d, n * w);
        zero_add(c, zl, L.b, n * w);
    }
    const size_t n0 = (size_t)c->lv[0].nodes() * nvec;
    c->d_x = dalloc<double>(c, c->rhs_allocs, n0);
    c->d_r = dalloc<double>(c, c->rhs_allocs, n0);
    c->d_q = dalloc<double>(c, c->rhs_allocs, n0);
    // window of search directions (cg_window, or by default up to MAX_PHIST steps within about 16 GiB, at
    // least two), an even count (the step graphs alternate the two slots of the host ring); a 1e-8 solve
    // of the 8.9 M-unknown body takes 21 steps, so x is updated once at its end
    {
        const size_t per = n0 * w;
        size_t h = per ? ((size_t)16 << 30) / per : (size_t)MAX_PHIST;
        if (c->opt.cg_window > 0) h = (size_t)c->opt.cg_window;
        h = std::max<size_t>(2, std::min<size_t>(MAX_PHIST, h)) & ~(size_t)1;
        c->phist_len = (int)h;
        c->phist_stride = (long long)n0;
        c->d_phist = dalloc<uint8_t>(c, c->rhs_allocs, h * per);
        // every step writes all nodes of the columns with unknowns of its slot before a later step reads
        // them, so only the other columns are cleared; packed models stop one by one (a stopped model's
        // bricks keep whatever the allocation held, and a neighbouring model's stencil may read them):
        // all of it
        const Level &L0 = c->lv[0];
        if (c->np || !L0.d_cmask) {
            zero_add(c, zl, c->d_phist, h * per);
        } else if (L0.nb > 0) {
            const dim3 grid((unsigned)((L0.nb + 3) / 4));
            const int nv = (int)(h * nvec);
            if (mixed)
                hipLaunchKernelGGL(k_zero_empty_cols<float>, grid, dim3(256), 0, c->stream, L0.d_cmask, L0.nb,
                                   L0.nodes(), nv, (float *)c->d_phist);
            else
                hipLaunchKernelGGL(k_zero_empty_cols<double>, grid, dim3(256), 0, c->stream, L0.d_cmask, L0.nb,
                                   L0.nodes(), nv, (double *)c->d_phist);
            HIPCHK(hipGetLastError());
        }
        c->d_ahist = dalloc<double>(c, c->rhs_allocs, (size_t)nb * h);
        zero_add(c, zl, c->d_ahist, (size_t)nb * h * sizeof(double));
    }
    c->d_z = dalloc<uint8_t>(c, c->rhs_allocs, n0 * w);
    c->d_r32 = mixed ? dalloc<float>(c, c->rhs_allocs, n0) : nullptr;
    // every vector starts at zero: slots of node columns without unknowns are never written and must
    // read as (finite) zeros, since stencils multiply them by conductance 0
    zero_add(c, zl, c->d_x, n0 * sizeof(double));
    zero_add(c, zl, c->d_r, n0 * sizeof(double));
    zero_add(c, zl, c->d_z, n0 * w);
    zero_add(c, zl, c->d_r32, n0 * sizeof(float));
    zero_add(c, zl, c->d_q, n0 * sizeof(double));
    c->pstride = 2 * c->lv[0].nb + 64;
    c->d_part = dalloc<double>(c, c->rhs_allocs, (size_t)c->pstride * nb);
    zero_add(c, zl, c->d_part, (size_t)c->pstride * nb * sizeof(double));
    c->d_nostop = dalloc<Scal>(c, c->rhs_allocs, nb);
    zero_add(c, zl, c->d_nostop, (size_t)nb * sizeof(Scal));
    zero_flush(c, zl);
    c->nbat = nb;
}

// Coarse level whose unknowns are the connected pieces of the 2x2x2
// aggregates of F (F structured or ELL), with its ELL Galerkin operator.
Level split_level(Ctx *c, Level &F)
{
    Level C;
    C.ell = true;
    const long long nf = F.nodes();
    int *parent = dalloc<int>(c, c->hier_allocs, nf);
    int *flag = dalloc<int>(c, c->hier_allocs, nf);
    int *idx = dalloc<int>(c, c->hier_allocs, nf);
    int *tmp = dalloc<int>(c, c->hier_allocs, nf / 2048 + 2);
    if (F.ell)
        HIPCHK(launch_pieces_ell(F.nrow, F.K, F.d_col, F.d_val64, F.d_pos, parent, c->stream));
    else
        HIPCHK(launch_pieces_brick(F.d_w64, F.nodes(), F.topo(), F.d_coord, parent, c->stream));
    HIPCHK(launch_pieces_finish(parent, nf, flag, c->stream));
    HIPCHK(scan_exclusive_ints(flag, nf, idx, tmp, c->d_ints, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_ints, c->d_ints, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int nc = c->h_ints[0];
    C.nrow = nc;
    C.d_pos = dalloc<int4>(c, c->hier_allocs, nc + 1);
    if (F.ell)
        HIPCHK(launch_piece_pos_ell(F.nrow, parent, idx, F.d_pos, C.d_pos, c->stream));
    else
        HIPCHK(launch_piece_pos_brick(parent, idx, F.topo(), F.d_coord, C.d_pos, c->stream));
    // fine -> coarse map and member lists
    F.d_agg = dalloc<int>(c, c->hier_allocs, nf);
    int *count = dalloc<int>(c, c->hier_allocs, nc + 1);
    HIPCHK(hipMemsetAsync(count, 0, (nc + 1) * sizeof(int), c->stream));
    HIPCHK(launch_pieces_assign(parent, idx, nf, F.d_agg, count, c->stream));
    C.d_mptr = dalloc<int>(c, c->hier_allocs, nc + 1);
    int *tmp2 = dalloc<int>(c, c->hier_allocs, nc / 2048 + 2);
    HIPCHK(scan_exclusive_ints(count, nc + 1, C.d_mptr, tmp2, c->d_ints + 1, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_ints + 1, c->d_ints + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int nmem = c->h_ints[1];
    C.d_mem = dalloc<int>(c, c->hier_allocs, nmem + 1);
    HIPCHK(hipMemsetAsync(count, 0, (nc + 1) * sizeof(int), c->stream));
    HIPCHK(launch_members(F.d_agg, nf, nc, C.d_mptr, count, C.d_mem, c->stream));
    C.d_memb = dalloc<int>(c, c->hier_allocs, (size_t)nc * 8 + 1);
    HIPCHK(hipMemsetAsync(c->d_ints + 4, 0, sizeof(int), c->stream));
    HIPCHK(launch_members8(nc, C.d_mptr, C.d_mem, C.d_memb, c->d_ints + 4, c->stream));
    // Galerkin rows: lengths, then the ELL arrays
    FineLevelArgs fa{};
    if (F.ell) {
        fa.n = F.nrow;
        fa.K = F.K;
        fa.col = F.d_col;
        fa.val = F.d_val64;
    } else {
        fa.w = F.d_w64;
        fa.stride = F.nodes();
        fa.nbr = F.d_nbr;
    }
    int *len = dalloc<int>(c, c->hier_allocs, nc + 1);
    HIPCHK(hipMemsetAsync(c->d_ints + 2, 0, 2 * sizeof(int), c->stream));
    HIPCHK(launch_galerkin_ell(fa, F.d_agg, nc, C.d_mptr, C.d_mem, 0, len, 0, nullptr, nullptr, nullptr, c->d_ints + 2,
                               c->d_ints + 3, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_ints + 2, c->d_ints + 2, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->h_ints[2]) throw HipFail{hipErrorInvalidValue, "split aggregate with too many coarse neighbours"};
    if (c->h_ints[4]) C.d_memb = nullptr;   // an aggregate of more than 8 members: the CSR restriction
    // rows of up to 8 entries are stored with 8 (padding: column -1, value 0), the width of the fixed-width
    // cycle kernels of the ELL levels
    C.K = std::max(c->h_ints[3], 8);
    C.d_col = dalloc<int>(c, c->hier_allocs, (size_t)C.K * nc + 1);
    C.d_val64 = dalloc<double>(c, c->hier_allocs, (size_t)C.K * nc + 1);
    C.d_val32 = dalloc<float>(c, c->hier_allocs, (size_t)C.K * nc + 1);
    HIPCHK(launch_galerkin_ell(fa, F.d_agg, nc, C.d_mptr, C.d_mem, 1, len, C.K, C.d_col, C.d_val64, C.d_val32,
                               c->d_ints + 2, c->d_ints + 3, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    // unknowns of the new level: rows with a conducting connection (their number only)
    HIPCHK(hipMemsetAsync(c->d_ints, 0, sizeof(int), c->stream));
    if (C.nrow > 0)
        hipLaunchKernelGGL(k_count_ell_dofs, dim3((unsigned)((C.nrow + 255) / 256)), dim3(256), 0, c->stream, C.nrow,
                           C.K, C.d_col, C.d_val64, c->d_ints);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_ints, c->d_ints, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    C.dofs = c->h_ints[0];
    return C;
}

spfd_status do_build(Ctx *c)
{
    drop_graphs(c);
    HIPCHK(hipStreamSynchronize(c->side));   // an earlier build that failed may have left its components running
    free_all(c, c->hier_allocs);
    c->d_adj_b = c->d_adj_c = c->d_adj_lam = c->d_adj_labpart = c->d_adj_labout = nullptr;
    c->d_adj_scal = nullptr;
    free_all(c, c->rhs_allocs);
    free_all(c, c->src_allocs);
    c->lv.clear();
    c->has_source.clear();
    c->nrhs = 0;
    Grid &g = c->g;
    // 1. bricks of the finest level + input validation
    const size_t nbg = (size_t)g.Gx * g.Gy * g.Gz;
    uint8_t *d_flags = dalloc<uint8_t>(c, c->hier_allocs, nbg);
    HIPCHK(hipMemsetAsync(d_flags, 0, nbg, c->stream));
    HIPCHK(hipMemsetAsync(c->d_ints, 0, 4 * sizeof(int), c->stream));
    HIPCHK(launch_brick_flags(c->d_labels, c->d_table64, c->nlab, c->voxel_mode ? c->d_sigvox : nullptr, g, d_flags,
                              c->d_ints, c->stream));
    uint8_t *hflags = stage(c, nbg);
    HIPCHK(hipMemcpyAsync(hflags, d_flags, nbg, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_ints, c->d_ints, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<uint8_t> flags(hflags, hflags + nbg);
    if (c->h_ints[0] == 1) return fail(c, SPFD_INVALID_ARG, "a voxel label is not covered by the sigma table");
    if (c->h_ints[0] == 2) return fail(c, SPFD_INVALID_ARG, "per-voxel sigma must be finite and >= 0");
    c->lv.emplace_back();
    Level &L0 = c->lv[0];
    L0.N[0] = g.Nx; L0.N[1] = g.Ny; L0.N[2] = g.Nz;
    L0.G[0] = g.Gx; L0.G[1] = g.Gy; L0.G[2] = g.Gz;
    build_topology(c, L0, flags, c->hier_allocs);
    if (L0.nb == 0) return fail(c, SPFD_INVALID_ARG, "no conducting voxel");
    if ((long long)L0.nb * BS > 0x7fffffffLL) return fail(c, SPFD_INVALID_ARG, "grid too large");
    // 2. finest-level conductances (stored FP64 for setup; label tiles for the solve)
    L0.d_w64 = dalloc<double>(c, c->hier_allocs, (size_t)3 * L0.nodes());
    L0.d_w32 = dalloc<float>(c, c->hier_allocs, (size_t)3 * L0.nodes());
    HIPCHK(launch_weights0(c->d_labels, c->d_table64, c->voxel_mode ? c->d_sigvox : nullptr, g, c->geo4, L0.d_coord,
                           L0.nb, L0.d_w64, L0.d_w32, c->stream));
    if (!c->voxel_mode) {
        L0.d_tiles = dalloc<uint8_t>(c, c->hier_allocs, (size_t)L0.nb * TILE_BYTES);
        HIPCHK(launch_label_tiles(c->d_labels, g, L0.d_coord, L0.nb, L0.d_tiles, c->stream));
    }
    // 3. connected components of the conductor (the gauge of Eq. (3)): on the side stream, beside the
    //    coarsening, which needs only the number of unknowns (the nodes with a positive diagonal, counted
    //    here); joined at the end of the build
    int *d_ncomp = dalloc<int>(c, c->hier_allocs, 1);
    {
        const long long n = L0.nodes();
        int *parent = dalloc<int>(c, c->hier_allocs, n);
        int *flag = dalloc<int>(c, c->hier_allocs, n);
        int *idx = dalloc<int>(c, c->hier_allocs, n);
        int *tmp = dalloc<int>(c, c->hier_allocs, n / 2048 + 2);
        c->d_comp = dalloc<int>(c, c->hier_allocs, n);
        HIPCHK(hipEventRecord(c->ev_side[0], c->stream));
        HIPCHK(hipStreamWaitEvent(c->side, c->ev_side[0], 0));
        HIPCHK(launch_components(L0.d_w64, n, L0.topo(), parent, flag, idx, tmp, c->d_comp, nullptr, d_ncomp, c->side));
        L0.dofs = count_dofs(c, L0);
    }
    // 4. coarsening: 2x2x2 aggregation until the level is small enough; from
    //    level split_level on, aggregates are split into their connected pieces
    while (c->lv.back().dofs > c->opt.coarsest_max && c->lv.size() < 20) {
        const int l = (int)c->lv.size() - 1;
        Level &F = c->lv[l];
        const bool split = !c->opt.no_split && (l >= c->opt.split_level || F.ell);
        if (!F.ell && F.N[0] == 1 && F.N[1] == 1 && F.N[2] == 1) break;
        if (split) {
            Level C = split_level(c, F);
            c->lv.push_back(std::move(C));
            continue;
        }
        Level C;
        for (int d = 0; d < 3; ++d) {
            C.N[d] = (F.N[d] + 1) / 2;
            C.G[d] = (C.N[d] + 7) / 8;
        }
        std::vector<uint8_t> cflags((size_t)C.G[0] * C.G[1] * C.G[2], 0);
        for (int s = 0; s < F.nb; ++s) {
            const int4 q = F.coord[s];
            cflags[(q.x >> 1) + (size_t)C.G[0] * ((q.y >> 1) + (size_t)C.G[1] * (q.z >> 1))] = 1;
        }
        build_topology(c, C, cflags, c->hier_allocs);
        std::vector<int> ps(F.nb);
        for (int s = 0; s < F.nb; ++s) {
            const int4 q = F.coord[s];
            ps[s] = C.slot_of[(q.x >> 1) + (size_t)C.G[0] * ((q.y >> 1) + (size_t)C.G[1] * (q.z >> 1))];
        }
        F.d_parent_slot = dalloc<int>(c, c->hier_allocs, F.nb);
        {
            uint8_t *st = stage(c, ps.size() * sizeof(int));  // (the stream is idle: topology just synced)
            memcpy(st, ps.data(), ps.size() * sizeof(int));
            HIPCHK(hipMemcpyAsync(F.d_parent_slot, st, ps.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        }
        C.d_w64 = dalloc<double>(c, c->hier_allocs, (size_t)3 * C.nodes());
        C.d_w32 = dalloc<float>(c, c->hier_allocs, (size_t)3 * C.nodes());
        HIPCHK(launch_galerkin(F.d_w64, F.nodes(), F.d_slot_of, F.G[0], F.G[1], F.G[2], F.N[0], F.N[1], F.N[2], C.d_coord,
                               C.nb, C.d_w64, C.d_w32, C.nodes(), c->stream));
        // the first coarse level of an FP32 cycle is bandwidth-bound and smoothed hardest: its smoothing
        // and restriction read FP16 weights scaled so the largest is 2^15 (relative rounding 2^-11;
        // the Galerkin operators below it come from the FP64 weights).  If the smallest nonzero
        // weight would then fall below FP16's normal range (2^-14), the FP32 weights are kept.
        if (c->opt.precision == SPFD_MIXED && c->lv.size() == 1 && !c->opt.level1_fp32) {
            unsigned *dm = dalloc<unsigned>(c, c->hier_allocs, 2);
            const unsigned init[2] = {0u, 0x7f800000u};
            memcpy(c->h_ints, init, sizeof(init));
            HIPCHK(hipMemcpyAsync(dm, c->h_ints, sizeof(init), hipMemcpyHostToDevice, c->stream));
            HIPCHK(launch_wmax(C.d_w32, 3LL * C.nodes(), dm, c->stream));
            HIPCHK(hipMemcpyAsync(c->h_ints, dm, sizeof(init), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            float mw, mp;
            memcpy(&mw, &c->h_ints[0], sizeof(float));
            memcpy(&mp, &c->h_ints[1], sizeof(float));
            if (mw > 0.0f && (double)mp / mw * 32768.0 >= 0x1p-14) {
                C.w16s = mw / 32768.0f;
                C.d_w16 = dalloc<uint16_t>(c, c->hier_allocs, (size_t)3 * C.nodes());
                HIPCHK(launch_w16(C.d_w32, 3LL * C.nodes(), 1.0f / C.w16s, C.d_w16, c->stream));
            }
        }
        HIPCHK(hipStreamSynchronize(c->stream));
        c->lv.push_back(std::move(C));
        c->lv.back().dofs = count_dofs(c, c->lv.back());
    }
    // column masks of the structured levels (the stencil kernels skip columns without unknowns) and
    // the inverse diagonals (first Chebyshev steps folded into neighbouring kernels): on the side stream,
    // after the components, beside the coarsest inverse; joined with them
    HIPCHK(hipEventRecord(c->ev_side[0], c->stream));
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_side[0], 0));
    for (Level &L : c->lv) {
        L.d_dinv64 = dalloc<double>(c, c->hier_allocs, L.nodes());
        L.d_dinv32 = dalloc<float>(c, c->hier_allocs, L.nodes());
        if (L.ell) {
            HIPCHK(launch_dinv_ell(L.nrow, L.K, L.d_col, L.d_val64, L.d_dinv64, L.d_dinv32, c->side));
        } else if (L.nb > 0) {
            L.d_cmask = dalloc<unsigned long long>(c, c->hier_allocs, L.nb);
            HIPCHK(launch_col_masks(L.d_w64, L.nodes(), L.topo(), L.d_cmask, c->side));
            HIPCHK(launch_dinv_struct(L.d_w64, L.nodes(), Topo{L.nb, L.d_nbr}, L.d_dinv64, L.d_dinv32, c->side));
        }
    }
    HIPCHK(hipEventRecord(c->ev_side[1], c->side));
    // 5. coarsest level: dense pseudo-inverse
    {
        Level &C = c->lv.back();
        const int maxd = 1024;
        c->d_node_cdof = dalloc<int>(c, c->hier_allocs, C.nodes());
        c->d_cdof_node = dalloc<int>(c, c->hier_allocs, maxd);
        c->d_cadj = dalloc<int>(c, c->hier_allocs, (size_t)maxd * 6);
        if (C.ell)
            HIPCHK(launch_coarse_enum_ell(C.nrow, C.K, C.d_col, C.d_val64, c->d_node_cdof, c->d_cdof_node, c->d_ints,
                                          maxd, c->stream));
        else
            HIPCHK(launch_coarse_setup(C.d_w64, C.nodes(), C.topo(), c->d_node_cdof, c->d_cdof_node, c->d_cadj,
                                       c->d_ints, maxd, c->stream));
        HIPCHK(hipMemcpyAsync(c->h_ints, c->d_ints, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        c->ncoarse = c->h_ints[0];
        if (c->ncoarse > maxd)
            return fail(c, SPFD_INVALID_ARG, "coarsest level too large (grid cannot be coarsened further)");
        c->d_Ainv = dalloc<double>(c, c->hier_allocs, (size_t)c->ncoarse * c->ncoarse + 1);
        c->d_cwork = dalloc<int>(c, c->hier_allocs, coarse_factor_work_ints(maxd));
        if (C.ell)
            HIPCHK(launch_coarse_dense_ell(C.nrow, C.K, C.d_col, C.d_val64, c->d_node_cdof, c->d_cdof_node, c->ncoarse,
                                           c->d_Ainv, c->stream));
        else
            HIPCHK(launch_coarse_assemble_brick(C.d_w64, C.nodes(), C.topo(), c->d_cdof_node, c->d_cadj, c->ncoarse,
                                                c->d_Ainv, c->stream));
        double *dwork = dalloc<double>(c, c->hier_allocs, dense_inverse_work_doubles(c->ncoarse));
        HIPCHK(launch_coarse_factor(c->ncoarse, c->d_Ainv, c->d_cwork, dwork, c->stream));
    }
    // join the side stream (components, masks, inverse diagonals); the component count sizes the gauge's
    // buffers
    {
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_side[1], 0));
        HIPCHK(hipMemcpyAsync(c->h_ints, d_ncomp, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        c->ncomp = c->h_ints[0];
        const Level &F0 = c->lv[0];   // (the coarsening above may have moved the level vector)
        const long long n = F0.nodes();
        c->d_counts = dalloc<int>(c, c->hier_allocs, c->ncomp + 1);
        c->d_means = dalloc<double>(c, c->hier_allocs, c->ncomp + 1);
        c->d_cpart = dalloc<double>(c, c->hier_allocs, comp_mean_parts(F0.nb));
        HIPCHK(hipMemsetAsync(c->d_counts, 0, (c->ncomp + 1) * sizeof(int), c->stream));
        HIPCHK(launch_comp_counts(c->d_comp, n, c->d_counts, c->stream));
    }
    chebyshev_coefficients(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    return SPFD_OK;
}

// Packed models: each model's finest-level bricks form one contiguous slot range (slots follow the
// brick grid with z slowest, and the models sit in disjoint brick layers).  Checked, not assumed.
spfd_status model_ranges(Ctx *c)
{
    const Level &L0 = c->lv[0];
    int m = 0;
    for (int k = 0; k < c->np; ++k) c->mfirst[k] = c->mcount[k] = 0;
    for (int b = 0; b < L0.nb; ++b) {
        const int z0 = L0.coord[b].z * BD;   // first node layer of the brick
        while (m < c->np && z0 > c->mbox.zoff[m] + c->mbox.nz[m]) ++m;
        if (m == c->np || z0 + BD - 1 < c->mbox.zoff[m])
            return fail(c, SPFD_HIP_ERROR, "a brick lies outside every model's layers");
        if (c->mcount[m] == 0) c->mfirst[m] = b;
        if (c->mfirst[m] + c->mcount[m] != b) return fail(c, SPFD_HIP_ERROR, "a model's bricks are not contiguous");
        c->mcount[m] += 1;
    }
    for (int k = 0; k < c->np; ++k)
        if (c->mcount[k] == 0) return fail(c, SPFD_INVALID_ARG, "a voxel model has no conducting voxel");
    int2 rg[MAX_MODELS];
    for (int k = 0; k < c->np; ++k) rg[k] = make_int2(c->mfirst[k], c->mcount[k]);
    c->d_mrange = dalloc<int2>(c, c->hier_allocs, MAX_MODELS);
    HIPCHK(hipMemcpyAsync(c->d_mrange, rg, c->np * sizeof(int2), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SPFD_OK;
}

spfd_status do_set_num_rhs(Ctx *c, int nrhs)
{
    free_all(c, c->src_allocs);
    // packed models: one right side per model, in one shared vector
    if (c->np) nrhs = c->np;
    const size_t n0 = (size_t)c->lv[0].nodes();
    c->d_bs = dalloc<double>(c, c->src_allocs, n0 * (c->np ? 1 : nrhs));
    HIPCHK(hipMemsetAsync(c->d_bs, 0, n0 * (c->np ? 1 : nrhs) * sizeof(double), c->stream));
    c->has_source.assign(nrhs, 0);
    c->d_scal = dalloc<Scal>(c, c->src_allocs, nrhs);
    c->d_again = dalloc<int>(c, c->src_allocs, nrhs + 1);
    HIPCHK(hipMemsetAsync(c->d_scal, 0, nrhs * sizeof(Scal), c->stream));
    drop_graphs(c);
    // pinned host scalars: kept while they hold enough right sides (a pinned allocation costs ~50-100 us of
    // host time, every rebuild passes here), cleared once the stream is idle (no step writes the ring)
    if (c->h_scal && c->h_ring && c->h_cap >= nrhs) {
        HIPCHK(hipStreamSynchronize(c->stream));
        memset(c->h_scal, 0, sizeof(Scal) * (c->h_cap + 1));
        memset(c->h_ring, 0, sizeof(Scal) * 2 * (c->h_cap + 1));
    } else {
        if (c->h_scal) (void)hipHostFree(c->h_scal);
        c->h_scal = nullptr;
        if (c->h_ring) (void)hipHostFree(c->h_ring);
        c->h_ring = nullptr;
        c->h_cap = 0;
        HIPCHK(hipHostMalloc((void **)&c->h_scal, sizeof(Scal) * (nrhs + 1), hipHostMallocDefault));
        // coherent: the step's last kernel stores the scalars here, the host reads them after an event
        HIPCHK(hipHostMalloc((void **)&c->h_ring, sizeof(Scal) * 2 * (nrhs + 1),
                             hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer((void **)&c->h_ring_dev, c->h_ring, 0));
        c->h_cap = nrhs;
    }
    c->nrhs = nrhs;
    alloc_cycle_buffers(c, nrhs);
    HIPCHK(hipStreamSynchronize(c->stream));
    return SPFD_OK;
}

// The flexible CG of a batch, split into phases so that a driver can advance
// several handles in lockstep: begin (z0 = B r0, r0.z0), step (one iteration),
// end (the deferred x update).
// With packed models the cycle runs once over all of them (it is block-diagonal: no aggregate, brick or
// component spans two models) with no stop flag, and the dot products follow per model.
template <typename T>
void pcg_begin(Ctx *c, Scal *sc, int nb)
{
    Level &L0 = c->lv[0];
    const Topo topo = cg_topo(c);
    const Batch bt = cg_batch(c, nb);
    T *z = (T *)c->d_z;
    const double n0 = (double)L0.dofs * (c->np ? 1 : nb);
    CycleDots dots{nullptr, c->d_part};   // r.z only
    // an FP32 cycle starts from the FP32 copy of r when the start wrote one (as every later cycle does)
    const bool r32 = sizeof(T) == sizeof(float) && c->r32_ready;
    c->r32_ready = false;
    // (the start pass writes the scaled copy where r32_scaled holds)
    const bool bs = r32 && r32_scaled(c);
    if (c->np) {
        if (r32)
            vcycle<T, float>(c, c->d_r32, z, nullptr, 1, nullptr, bs);
        else
            vcycle<T, double>(c, c->d_r, z, nullptr, 1, nullptr);
    } else if (r32 ? vcycle<T, float>(c, c->d_r32, z, sc, nb, &dots, bs)
                   : vcycle<T, double>(c, c->d_r, z, sc, nb, &dots)) {
        finish(c, cheb_dot_parts<T>(topo.nb), FIN_BETA0, sc, 0, nb);
        return;
    }
    {
        TScope ts(c, SPFD_K_DOTS, n0 * (sizeof(T) + 8.0));
        HIPCHK(launch_dots<T>(topo, z, c->d_r, c->d_q, c->d_part, sc, 1, bt, c->stream));
    }
    finish(c, topo_count(topo), FIN_BETA0, sc, 0, nb, nullptr, ROWS_BRICKS);
}

// CG step `it`: for it >= 1 first z = B r (the cycle, which also forms z.r and, for the flexible beta,
// z.q) and beta; then p = z + beta p, the deferred x update and q = A p, alpha, and the residual update
// with its norm, which decides the stop.  The step ends at the stop decision, so the step that converges
// leaves no cycle behind it (step 0's cycle and beta are formed by pcg_begin).
template <typename T>
void pcg_step(Ctx *c, Scal *sc, int nb, int it, int max_iter)
{
    Level &L0 = c->lv[0];
    const Topo topo = cg_topo(c);
    const int nmax = topo_count(topo);
    const OpArgs<double> op = level_op<double>(c, 0);
    const Batch bt = cg_batch(c, nb);
    T *z = (T *)c->d_z;
    const double n0 = (double)L0.dofs * (c->np ? 1 : nb);
    const double wz = sizeof(T);
    // an FP32 cycle reads an FP32 copy of the residual, written by the update kernel
    float *r32 = sizeof(T) == sizeof(float) ? c->d_r32 : nullptr;
    // p_k in the window slot Scal::hcount (= it % nh: x is updated and the window emptied every nh steps),
    // in the cycle's precision
    const int nh = c->phist_len;
    T *ph = (T *)c->d_phist;
    if (it > 0) {
        const bool flex = c->cg_flexible;
        const int bmode = flex ? FIN_BETA : FIN_BETA_STD;
        CycleDots dots{flex ? c->d_q : nullptr, c->d_part};
        // the residual update of the standard beta writes the scaled copy where r32_scaled holds
        const bool bs = r32 && !flex && r32_scaled(c);
        bool fused = false;
        if (c->np) {
            if (r32)
                vcycle<T, float>(c, r32, z, nullptr, 1, nullptr, bs);
            else
                vcycle<T, double>(c, c->d_r, z, nullptr, 1, nullptr);
        } else {
            fused = r32 ? vcycle<T, float>(c, r32, z, sc, nb, &dots, bs)
                        : vcycle<T, double>(c, c->d_r, z, sc, nb, &dots);
        }
        if (fused) {
            finish(c, cheb_dot_parts<T>(topo.nb), bmode, sc, 0, nb);
        } else {
            {
                TScope ts(c, SPFD_K_DOTS, n0 * (wz + (flex ? 16.0 : 8.0)));
                HIPCHK(launch_dots<T>(topo, z, c->d_r, c->d_q, c->d_part, sc, flex ? 0 : 1, bt, c->stream));
            }
            finish(c, nmax, bmode, sc, 0, nb, nullptr, ROWS_BRICKS);
        }
    }
    // p_k = z_k + beta p_{k-1}, q_k = A p_k.  Only the flexible beta reads q_k later (z.q); with the
    // standard beta the residual update forms A p_k again from p_k instead.  x is updated at the end of
    // the window (x_flush).
    const bool keep_q = c->cg_flexible;
    {
        // z, p_{k-1}, p_k in the cycle's precision; q in FP64
        TScope ts(c, SPFD_K_SPMV, n0 * (wz + (it ? 2.0 * wz : wz) + (keep_q ? 8.0 : 0.0) + op_bytes<double>(c, 0)));
        HIPCHK(launch_cg_step<T>(op, topo, z, ph, c->phist_stride, nh, keep_q ? c->d_q : nullptr, c->d_part, sc,
                                 it == 0, bt, c->stream));
    }
    finish(c, cg_step_parts(nmax), FIN_ALPHA, sc, 0, nb, nullptr, ROWS_CG_GROUPS);
    if (keep_q) {
        {
            TScope ts(c, SPFD_K_UPDATE, n0 * (24.0 + (r32 ? 4.0 : 0.0)));
            HIPCHK(launch_rupdate(topo, c->d_r, c->d_q, c->d_part, sc, bt, r32, c->stream, c->d_ahist, nh));
        }
        finish(c, nmax, FIN_RR, sc, max_iter, nb, c->step_mirror, ROWS_BRICKS);
    } else {
        {
            // r (read and written), p_k and the operator; the FP32 copy of r
            TScope ts(c, SPFD_K_UPDATE, n0 * (16.0 + wz + op_bytes<double>(c, 0) + (r32 ? 4.0 : 0.0)));
            HIPCHK(launch_col_rupdate<T>(op, topo, ph, c->phist_stride, nh, c->d_r, r32, c->d_part, sc, bt, c->stream,
                                         r32 && r32_scaled(c), c->d_ahist));
        }
        finish(c, rupdate_parts(nmax), FIN_RR, sc, max_iter, nb, c->step_mirror, ROWS_RU_GROUPS);
    }
}

// x += sum alpha_j p_j over the steps of the window taken and not yet added; full: then an empty window
// (steps: how many directions are added, for the byte count)
void x_flush(Ctx *c, Scal *sc, int nb, int steps, bool full = true)
{
    Level &L0 = c->lv[0];
    const double wp = c->opt.precision == SPFD_MIXED ? 4.0 : 8.0;
    TScope ts(c, SPFD_K_PUPDATE, (double)L0.dofs * (c->np ? 1 : nb) * (16.0 + steps * wp));
    if (c->opt.precision == SPFD_MIXED)
        HIPCHK(launch_x_flush<float>(cg_topo(c), c->d_x, (const float *)c->d_phist, c->phist_stride, c->d_ahist,
                                     c->phist_len, sc, cg_batch(c, nb), c->stream, full ? 1 : 0));
    else
        HIPCHK(launch_x_flush<double>(cg_topo(c), c->d_x, (const double *)c->d_phist, c->phist_stride, c->d_ahist,
                                      c->phist_len, sc, cg_batch(c, nb), c->stream, full ? 1 : 0));
}

void pcg_end(Ctx *c, Scal *sc, int nb, int steps)
{
    // the search directions of the last, partial window
    x_flush(c, sc, nb, steps % c->phist_len);
}

void pcg_begin_any(Ctx *c, Scal *sc, int nb)
{
    if (c->opt.precision == SPFD_MIXED)
        pcg_begin<float>(c, sc, nb);
    else
        pcg_begin<double>(c, sc, nb);
}

void pcg_step_any(Ctx *c, Scal *sc, int nb, int it, int max_iter)
{
    if (c->opt.precision == SPFD_MIXED)
        pcg_step<float>(c, sc, nb, it, max_iter);
    else
        pcg_step<double>(c, sc, nb, it, max_iter);
}

void drop_graphs(Ctx *c)
{
    for (auto &g : c->sg) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = Ctx::StepGraph{};
    }
    c->sg_nb = -1;
    c->sg_sc = nullptr;
    c->sg_max_iter = -1;
}

// Enqueue CG step `it`; its last kernel also stores the scalars into hsc (a
// slot of the pinned ring).  Steps after the first have fixed kernel
// arguments per buffer parity, so they are captured once into a HIP graph and
// replayed: one host call instead of some fifty launches, which keeps the
// short coarse-level kernels back to back.  The first step, eager solves and
// the step sampled by the launch timing run eagerly.  The graphs hold no
// memset nodes.
void pcg_step_enqueue(Ctx *c, Scal *sc, Scal *hsc, int nb, int it, int max_iter, bool eager)
{
    if (!c->h_ring || hsc < c->h_ring || hsc + nb > c->h_ring + 2 * (c->nrhs + 1))
        throw HipFail{hipErrorInvalidValue, "CG step scalars outside the pinned ring"};
    Scal *mirror = c->h_ring_dev + (hsc - c->h_ring);
    struct MirrorScope {
        Ctx *c;
        MirrorScope(Ctx *c_, Scal *m) : c(c_) { c->step_mirror = m; }
        ~MirrorScope() { c->step_mirror = nullptr; }
    } ms(c, mirror);
    const bool timed_sample = c->tmask != 0 && it == 1;
    // a full window of search directions updates x before the next step overwrites its first slot
    const bool flush = (it + 1) % c->phist_len == 0;
    if (eager || it == 0 || timed_sample) {
        c->step_ctx = timed_sample ? 2 : 1;
        pcg_step_any(c, sc, nb, it, max_iter);
        c->step_ctx = 0;
        if (flush) x_flush(c, sc, nb, c->phist_len);
        return;
    }
    if (c->sg_nb != nb || c->sg_sc != sc || c->sg_max_iter != max_iter || c->sg_flexible != (int)c->cg_flexible) {
        drop_graphs(c);
        c->sg_nb = nb;
        c->sg_sc = sc;
        c->sg_max_iter = max_iter;
        c->sg_flexible = (int)c->cg_flexible;
    }
    Ctx::StepGraph &g = c->sg[it & 1];
    if (g.exec && g.mirror != mirror) {
        (void)hipGraphExecDestroy(g.exec);
        g = Ctx::StepGraph{};
    }
    if (!g.exec) {
        g = Ctx::StepGraph{};
        g.mirror = mirror;
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        c->capturing = &g;
        try {
            pcg_step_any(c, sc, nb, it, max_iter);
        } catch (...) {
            c->capturing = nullptr;
            (void)hipStreamEndCapture(c->stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        c->capturing = nullptr;
        HIPCHK(hipStreamEndCapture(c->stream, &graph));
        const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(e);
    }
    HIPCHK(hipGraphLaunch(g.exec, c->stream));
    for (int k = 0; k < SPFD_K_COUNT; ++k) {
        c->tlaunch[k] += g.launch[k];
        c->tbytes[k] += g.bytes[k];
    }
    if (flush) x_flush(c, sc, nb, c->phist_len);
}

// Host loop of the CG iterations, one step ahead: step it+1 is enqueued before
// the host waits for the scalars of step it, so the GPU never idles on the
// host's poll.  When step it converged, an already enqueued step it+1 finds
// the stop flag and writes nothing, but its kernels still launch and load.
// So when the residual history predicts that step it is the last one (the
// ratio of the last two ||r||^2 carried one step further reaches the
// tolerance within a margin), step it+1 is held back until step it is seen:
// a wrong guess costs the host's round trip, a right one saves a whole step.
constexpr double HOLD_MARGIN = 4.0;

void pcg_iterations(Ctx *c, Scal *sc, int nb, const spfd_solve_options &so)
{
    Scal *ring[2] = {c->h_ring, c->h_ring + nb};
    const bool eager = so.eager != 0;
    c->cg_flexible = so.flexible != 0;
    c->step_ctx = 1;
    pcg_begin_any(c, sc, nb);
    c->step_ctx = 0;
    auto enqueue = [&](int k) {
        pcg_step_enqueue(c, sc, ring[k & 1], nb, k, so.max_iter, eager);
        HIPCHK(hipEventRecord(c->ev_it[k & 1], c->stream));
    };
    // ||r||^2 after the last two steps seen by the host (< 0: not seen yet)
    std::vector<double> rr1(nb, -1.0), rr2(nb, -1.0), tol2(nb, 0.0);
    std::vector<int> seen_done(nb, 0);
    int seen_iters = 0;
    auto likely_last = [&]() {
        if (seen_iters + 1 >= so.max_iter) return true;
        for (int i = 0; i < nb; ++i) {
            if (seen_done[i]) continue;
            if (!(rr1[i] > 0.0 && rr2[i] > 0.0)) return false;
            const double next = rr1[i] * (rr1[i] / rr2[i]);
            if (!(next <= HOLD_MARGIN * tol2[i])) return false;
        }
        return true;
    };
    enqueue(0);
    int queued = 0;
    for (int it = 0; it <= so.max_iter; ++it) {
        if (queued < it) {
            enqueue(it);
            queued = it;
        }
        if (it + 1 <= so.max_iter && !likely_last()) {
            enqueue(it + 1);
            queued = it + 1;
        } else if (queued == it) {
            // step it+1 is held back: the GPU would idle during the host's poll, so x takes the directions
            // kept so far now (the window goes on: they are only marked as added)
            x_flush(c, sc, nb, (it + 1) % c->phist_len, false);
        }
        HIPCHK(hipEventSynchronize(c->ev_it[it & 1]));
        const Scal *hs = ring[it & 1];
        bool all = true;
        for (int i = 0; i < nb; ++i) {
            all = all && hs[i].done;
            seen_done[i] = hs[i].done;
            rr2[i] = rr1[i];
            rr1[i] = hs[i].rr;
            tol2[i] = hs[i].tol2;
            seen_iters = std::max(seen_iters, hs[i].iters);
        }
        if (all) break;
    }
    pcg_end(c, sc, nb, queued + 1);
}

void resid_b(Ctx *c, const double *b, long long bvs, Scal *sc, double *r, int mode, int nb);

// Flexible GMRES (one right side): from x and its residual r in c->d_r, cycles
// of up to m columns with the same multigrid cycle as the CG, each column
// z_j = B v_j, w = A z_j, two classical Gram-Schmidt passes, Givens rotation;
// x += Z y at the end of a cycle, restart from the true residual b - A x.
template <typename T>
void fgmres_iterations(Ctx *c, const double *b, long long bvs, Scal *sc, const spfd_solve_options &so)
{
    Level &L0 = c->lv[0];
    const long long n0 = L0.nodes();
    const int m = so.restart;
    const bool mixed = sizeof(T) == sizeof(float);
    if (c->fg_m < m) {
        c->d_fgV = dalloc<double>(c, c->rhs_allocs, (size_t)(m + 1) * n0);
        c->d_fgZ = dalloc<uint8_t>(c, c->rhs_allocs, (size_t)m * n0 * sizeof(T));
        if (!c->d_fgst) c->d_fgst = (FGState *)dalloc<uint8_t>(c, c->rhs_allocs, sizeof(FGState));
        if (!c->d_fgpart) c->d_fgpart = dalloc<double>(c, c->rhs_allocs, (size_t)FG_MAXM * FG_PARTS);
        HIPCHK(hipMemsetAsync(c->d_fgV, 0, (size_t)(m + 1) * n0 * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(c->d_fgZ, 0, (size_t)m * n0 * sizeof(T), c->stream));
        c->fg_m = m;
    }
    double *V = c->d_fgV;
    T *Z = (T *)c->d_fgZ;
    FGState *st = c->d_fgst;
    double *part = c->d_fgpart;
    double *w = c->d_q;
    float *v32 = mixed ? c->d_r32 : nullptr;
    const int ng = fg_parts(n0);
    const OpArgs<double> op = level_op<double>(c, 0);
    const Topo topo = L0.topo();
    const Batch bt = level_batch(c, 0, 1);
    const double nd = (double)L0.dofs;
    Scal *hs = c->h_ring;
    auto poll = [&]() {
        HIPCHK(hipMemcpyAsync(hs, sc, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return hs->done != 0;
    };
    // ||r||^2 and the stop test of the start
    {
        TScope ts(c, SPFD_K_DOTS, nd * 8.0);
        HIPCHK(launch_mdot(c->d_r, n0, c->d_r, n0, 1, part, sc, c->stream));
    }
    HIPCHK(launch_finish(part, ng, FIN_RESID0, sc, 0, c->stream, nullptr, nullptr, 0, 1, 0));
    HIPCHK(launch_fg_start(st, sc, c->stream));
    {
        TScope ts(c, SPFD_K_UPDATE, nd * (16.0 + (mixed ? 4.0 : 0.0)));
        HIPCHK(launch_fg_scale(c->d_r, V, v32, n0, st, sc, c->stream));
    }
    if (poll()) return;
    // Columns run one ahead of the host's check, as the CG steps do: column j+1
    // is enqueued before the host reads the stop test of column j (a column
    // after the last one finds the stop flag and stores nothing), unless the
    // residual estimates predict that column j ends the solve, or j ends the cycle.
    Scal *ring[2] = {c->h_ring, c->h_ring + 1};
    auto enqueue_column = [&](int j) {
        T *zj = Z + (long long)j * n0;
        if (mixed)
            vcycle<T, float>(c, v32, zj, sc, 1);
        else
            vcycle<T, double>(c, V + (long long)j * n0, zj, sc, 1);
        {
            TScope ts(c, SPFD_K_SPMV, nd * (sizeof(T) + 8.0 + op_bytes<double>(c, 0)));
            HIPCHK(launch_spmv<T>(op, topo, zj, w, sc, bt, c->stream));
        }
        const int nv = j + 1;
        {
            TScope ts(c, SPFD_K_DOTS, nd * 8.0 * (nv + 1));
            HIPCHK(launch_mdot(V, n0, w, n0, nv, part, sc, c->stream));
        }
        HIPCHK(launch_msum(part, ng, nv, st->h1, sc, c->stream));
        {
            TScope ts(c, SPFD_K_DOTS, nd * 8.0 * (nv + 2));
            HIPCHK(launch_mupdate(V, n0, w, n0, nv, st->h1, 0, part, sc, c->stream));
        }
        HIPCHK(launch_msum(part, ng, nv, st->h2, sc, c->stream));
        {
            TScope ts(c, SPFD_K_DOTS, nd * 8.0 * (nv + 2));
            HIPCHK(launch_mupdate(V, n0, w, n0, nv, st->h2, 1, part, sc, c->stream));
        }
        HIPCHK(launch_msum(part, ng, 1, &st->hnext, sc, c->stream));
        HIPCHK(launch_fg_column(st, sc, j, so.max_iter, c->stream));
        {
            TScope ts(c, SPFD_K_UPDATE, nd * (16.0 + (mixed ? 4.0 : 0.0)));
            HIPCHK(launch_fg_scale(w, V + (long long)nv * n0, v32, n0, st, sc, c->stream));
        }
        HIPCHK(hipMemcpyAsync(ring[j & 1], sc, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipEventRecord(c->ev_it[j & 1], c->stream));
    };
    double rr1 = -1.0, rr2 = -1.0;  // residual estimates of the last two columns seen
    int j = 0, queued = -1;
    for (;;) {
        if (queued < j) {
            enqueue_column(j);
            queued = j;
        }
        const bool likely_last = rr1 > 0.0 && rr2 > 0.0 && rr1 * (rr1 / rr2) <= HOLD_MARGIN * ring[0]->tol2;
        if (j + 1 < m && !likely_last) {
            enqueue_column(j + 1);
            queued = j + 1;
        }
        HIPCHK(hipEventSynchronize(c->ev_it[j & 1]));
        const bool done = ring[j & 1]->done != 0;
        rr2 = rr1;
        rr1 = ring[j & 1]->rr;
        const int k = j + 1;
        if (!done && k < m) {
            j = k;
            continue;
        }
        // end of a cycle or of the solve: x += Z y over the k columns formed
        HIPCHK(launch_fg_ysolve(st, k, c->stream));
        {
            TScope ts(c, SPFD_K_UPDATE, nd * (16.0 + k * (double)sizeof(T)));
            HIPCHK(launch_fg_xupdate<T>(c->d_x, Z, n0, n0, k, st, c->stream));
        }
        if (done) return;
        // restart from the true residual
        resid_b(c, b, bvs, sc, c->d_r, 0, 1);
        HIPCHK(launch_fg_start(st, sc, c->stream));
        {
            TScope ts(c, SPFD_K_UPDATE, nd * (16.0 + (mixed ? 4.0 : 0.0)));
            HIPCHK(launch_fg_scale(c->d_r, V, v32, n0, st, sc, c->stream));
        }
        if (poll()) return;
        j = 0;
        queued = -1;
        rr1 = rr2 = -1.0;
    }
}

void krylov_iterations(Ctx *c, const double *b, long long bvs, Scal *sc, int nb, const spfd_solve_options &so)
{
    if (so.method == SPFD_FGMRES) {
        if (c->opt.precision == SPFD_MIXED)
            fgmres_iterations<float>(c, b, bvs, sc, so);
        else
            fgmres_iterations<double>(c, b, bvs, sc, so);
        return;
    }
    pcg_iterations(c, sc, nb, so);
}

// r = b - A x for the batch and ||r||^2 (mode 0: start of a warm-started solve,
// mode 1: true residual kept in zq)
void resid_b(Ctx *c, const double *b, long long bvs, Scal *sc, double *r, int mode, int nb)
{
    Level &L0 = c->lv[0];
    const Topo topo = cg_topo(c);
    {
        TScope ts(c, SPFD_K_RESID, (c->np ? 1 : nb) * (double)L0.dofs * (16.0 + (r ? 8.0 : 0.0) + op_bytes<double>(c, 0)));
        HIPCHK(launch_resid(level_op<double>(c, 0), topo, b, c->d_x, r, c->d_part, c->np ? 0 : bvs, cg_batch(c, nb),
                            c->stream));
    }
    finish(c, cg_step_parts(topo_count(topo)), mode == 0 ? FIN_RESID0 : FIN_RESID1, sc, 0, nb, nullptr, ROWS_CG_GROUPS);
}


__global__ void k_rearm_if(Scal *sc, double tol, int nb, const int *again)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb && again[i]) {
        sc[i].done = 0;
        sc[i].status = 0;
        sc[i].tol2 = tol * tol * sc[i].bb;
    }
}

// Solve A x = b for a batch of nb right sides b[i] = b + i*bvs (brick layout,
// FP64) whose scalars (with ||b||^2 from the right-side kernel) live in sc[i];
// write the gauged solutions as dense node arrays psi + i*nn (also the start
// iterates when use_x0).  Uses the handle's solve buffers (nb <= nbat).
spfd_status solve_batch(Ctx *c, const double *b, long long bvs, Scal *sc, Scal *hsc, int nb,
                        const spfd_solve_options &so, double *psi, spfd_rhs_info *info)
{
    Level &L0 = c->lv[0];
    const Topo topo = L0.topo();
    const long long n0 = L0.nodes();
    const long long nn = (long long)c->g.Nx * c->g.Ny * c->g.Nz;
    // packed models share one vector of each kind
    const int nvec = c->np ? 1 : nb;
    HIPCHK(launch_scal_init(sc, so.rel_tol, so.use_x0, nb, c->stream));
    c->r32_ready = false;
    if (so.use_x0) {
        for (int i = 0; i < nvec; ++i)
            HIPCHK(launch_psi_in(psi + i * nn, c->d_comp, L0.d_coord, L0.nb, c->g, c->d_x + i * n0, c->stream));
        resid_b(c, b, bvs, sc, c->d_r, 0, nb);
    } else {
        // x = 0, r = b and (FP32 cycle) the FP32 copy of r for the first cycle, in one pass
        const bool mixed = c->opt.precision == SPFD_MIXED && so.method != SPFD_FGMRES;
        HIPCHK(launch_start(n0, b, bvs, c->d_x, c->d_r, mixed ? c->d_r32 : nullptr, nvec, c->stream,
                            mixed && r32_scaled(c) ? c->lv[0].d_dinv32 : nullptr));
        c->r32_ready = mixed;
    }
    // no host round trip here: a right side that is already done (b = 0, or an exact x0) stops the
    // kernels through its device-side flag, and ||b||^2 comes back with the final scalars
    std::vector<double> bb(nb), relres(nb, 0.0);
    std::vector<int> status(nb, 0), iters(nb, 0);
    bool any = true;
    int *again = c->d_again;
    // gauge and dense output of every right side: zero mean per connected component, 0 outside the
    // conductor (packed models: one gauge pass over the shared vector, no component spans two models)
    auto emit = [&]() {
        if (c->np) {
            TScope ts(c, SPFD_K_GAUGE, (double)L0.dofs * 24.0 + c->mnodes_off[c->np] * 8.0);
            HIPCHK(launch_comp_mean(topo, c->d_x, c->d_comp, c->ncomp, c->d_counts, c->d_means, c->d_cpart, c->stream));
        }
        for (int i = 0; i < nb; ++i) {
            if (c->np) {
                HIPCHK(launch_psi_out(c->d_x, c->d_comp, c->d_means, L0.d_slot_of, c->mgrid[i], psi + c->mnodes_off[i],
                                      c->stream, &c->g, c->mbox.zoff[i]));
            } else {
                TScope ts(c, SPFD_K_GAUGE,
                          (double)L0.dofs * (12.0 * (c->ncomp < 16 ? c->ncomp : 1) + 12.0) + nn * 8.0);
                HIPCHK(launch_comp_mean(topo, c->d_x + i * n0, c->d_comp, c->ncomp, c->d_counts, c->d_means,
                                        c->d_cpart, c->stream));
                HIPCHK(launch_psi_out(c->d_x + i * n0, c->d_comp, c->d_means, L0.d_slot_of, c->g, psi + i * nn,
                                      c->stream));
            }
        }
    };
    for (int pass = 0; pass < 3 && any; ++pass) {
        krylov_iterations(c, b, bvs, sc, nb, so);
        // true residual of every iterate (also of those that converged in an earlier pass); r itself is
        // only needed for a restart and is formed again then
        resid_b(c, b, bvs, sc, nullptr, 1, nb);
        HIPCHK(hipMemcpyAsync(hsc, sc, nb * sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
        // the output is formed before the host has seen the residuals (no idle GPU during that round
        // trip); a restart forms it again
        emit();
        HIPCHK(hipStreamSynchronize(c->stream));
        any = false;
        std::vector<int> redo(nb, 0);
        for (int i = 0; i < nb; ++i) {
            bb[i] = hsc[i].bb;
            relres[i] = bb[i] > 0.0 ? sqrt(hsc[i].zq / bb[i]) : 0.0;
            status[i] = hsc[i].status;
            iters[i] = hsc[i].iters;
            // the recursive residual drifted from the true one: restart from the true residual
            if (bb[i] > 0.0 && status[i] == 0 && relres[i] > so.rel_tol && iters[i] < so.max_iter && pass < 2) {
                redo[i] = 1;
                any = true;
            }
        }
        if (any) {
            resid_b(c, b, bvs, sc, c->d_r, 1, nb);
            HIPCHK(hipMemcpyAsync(again, redo.data(), nb * sizeof(int), hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_rearm_if, dim3(1), dim3(64), 0, c->stream, sc, so.rel_tol, nb, again);
            HIPCHK(hipGetLastError());
        }
    }
    spfd_status worst = SPFD_OK;
    for (int i = 0; i < nb; ++i) {
        if (bb[i] > 0.0 && status[i] == 0 && relres[i] > so.rel_tol) status[i] = SPFD_NOT_CONVERGED;
        if (status[i] != 0 && worst == SPFD_OK) worst = (spfd_status)status[i];
        if (info) {
            info[i].iterations = iters[i];
            info[i].rel_residual = relres[i];
            info[i].status = status[i];
        }
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return worst;
}

spfd_status do_solve(Ctx *c, const spfd_solve_options &so, double *psi, spfd_rhs_info *info)
{
    const long long n0 = c->lv[0].nodes();
    spfd_status worst = solve_batch(c, c->d_bs, n0, c->d_scal, c->h_scal, c->nrhs, so, psi, info);
    if (worst != SPFD_OK)
        c->err = worst == SPFD_BREAKDOWN ? "breakdown in CG (non-positive curvature or non-finite value)"
                                         : "maximum iteration count reached";
    return worst;
}

// Several handles (each with its own hierarchy, sources and stream) advanced
// in lockstep: every iteration enqueues one CG step per unfinished handle on
// that handle's stream, so the kernels of small problems run side by side on
// the GPU, and one host poll serves all.  Handles that need a restart from the
// true residual finish alone with solve_batch.
spfd_status solve_many(Ctx **hs, int n, const spfd_solve_options &so, double **psi, spfd_rhs_info *info)
{
    std::vector<int> active(n, 0), steps(n, 0), off(n, 0);
    int tot = 0;
    for (int k = 0; k < n; ++k) {
        off[k] = tot;
        tot += hs[k]->nrhs;
    }
    // start: x0 = 0, r = b and the FP32 copy of r, as in solve_batch (the same first cycle)
    for (int k = 0; k < n; ++k) {
        Ctx *c = hs[k];
        const long long n0 = c->lv[0].nodes();
        HIPCHK(hipSetDevice(c->device));
        c->cg_flexible = so.flexible != 0;
        HIPCHK(launch_scal_init(c->d_scal, so.rel_tol, 0, c->nrhs, c->stream));
        const bool mixed = c->opt.precision == SPFD_MIXED;
        HIPCHK(launch_start(n0, c->d_bs, n0, c->d_x, c->d_r, mixed ? c->d_r32 : nullptr, c->np ? 1 : c->nrhs,
                            c->stream, mixed && r32_scaled(c) ? c->lv[0].d_dinv32 : nullptr));
        c->r32_ready = mixed;
        HIPCHK(hipMemcpyAsync(c->h_scal, c->d_scal, c->nrhs * sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
    }
    for (int k = 0; k < n; ++k) {
        Ctx *c = hs[k];
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int i = 0; i < c->nrhs; ++i) active[k] = active[k] || !c->h_scal[i].done;
        if (active[k]) {
            c->step_ctx = 1;
            pcg_begin_any(c, c->d_scal, c->nrhs);
            c->step_ctx = 0;
        }
    }
    int left = 0;
    for (int k = 0; k < n; ++k) left += active[k];
    // every handle one step ahead, as in pcg_iterations
    auto enqueue = [&](int k) {
        Ctx *c = hs[k];
        const int it = steps[k]++;
        pcg_step_enqueue(c, c->d_scal, c->h_ring + (it & 1) * c->nrhs, c->nrhs, it, so.max_iter, so.eager != 0);
        HIPCHK(hipEventRecord(c->ev_it[it & 1], c->stream));
    };
    for (int k = 0; k < n; ++k)
        if (active[k]) enqueue(k);
    for (int it = 0; it < so.max_iter + 1 && left > 0; ++it) {
        for (int k = 0; k < n; ++k)
            if (active[k] && it + 1 <= so.max_iter) enqueue(k);
        for (int k = 0; k < n; ++k)
            if (active[k]) {
                Ctx *c = hs[k];
                HIPCHK(hipEventSynchronize(c->ev_it[it & 1]));
                const Scal *hs_it = c->h_ring + (it & 1) * c->nrhs;
                bool all = true;
                for (int i = 0; i < c->nrhs; ++i) all = all && hs_it[i].done;
                if (all) {
                    pcg_end(c, c->d_scal, c->nrhs, steps[k]);
                    active[k] = 0;
                    --left;
                }
            }
    }
    for (int k = 0; k < n; ++k)
        if (active[k]) pcg_end(hs[k], hs[k]->d_scal, hs[k]->nrhs, steps[k]);
    // true residuals, restarts, gauge and output
    spfd_status worst = SPFD_OK;
    for (int k = 0; k < n; ++k) {
        Ctx *c = hs[k];
        const int nb = c->nrhs;
        const long long n0 = c->lv[0].nodes();
        const long long nn = (long long)c->g.Nx * c->g.Ny * c->g.Nz;
        resid_b(c, c->d_bs, n0, c->d_scal, c->d_r, 1, nb);
        HIPCHK(hipMemcpyAsync(c->h_scal, c->d_scal, nb * sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        bool redo = false;
        for (int i = 0; i < nb; ++i) {
            const double bb = c->h_scal[i].bb;
            const double rel = bb > 0.0 ? sqrt(c->h_scal[i].zq / bb) : 0.0;
            if (bb > 0.0 && c->h_scal[i].status == 0 && rel > so.rel_tol && c->h_scal[i].iters < so.max_iter) redo = true;
        }
        spfd_status st;
        if (redo) {
            st = solve_batch(c, c->d_bs, n0, c->d_scal, c->h_scal, nb, so, psi[k], info ? info + off[k] : nullptr);
        } else {
            st = SPFD_OK;
            const Level &L0 = c->lv[0];
            for (int i = 0; i < nb; ++i) {
                const double bb = c->h_scal[i].bb;
                int status = c->h_scal[i].status;
                const double rel = bb > 0.0 ? sqrt(c->h_scal[i].zq / bb) : 0.0;
                if (bb > 0.0 && status == 0 && rel > so.rel_tol) status = SPFD_NOT_CONVERGED;
                if (status != 0 && st == SPFD_OK) st = (spfd_status)status;
                TScope ts(c, SPFD_K_GAUGE, (double)L0.dofs * 24.0 + nn * 8.0);
                HIPCHK(launch_comp_mean(L0.topo(), c->d_x + i * n0, c->d_comp, c->ncomp, c->d_counts, c->d_means,
                                        c->d_cpart, c->stream));
                HIPCHK(launch_psi_out(c->d_x + i * n0, c->d_comp, c->d_means, L0.d_slot_of, c->g, psi[k] + i * nn,
                                      c->stream));
                if (info) {
                    info[off[k] + i].iterations = c->h_scal[i].iters;
                    info[off[k] + i].rel_residual = rel;
                    info[off[k] + i].status = status;
                }
            }
        }
        if (st != SPFD_OK && worst == SPFD_OK) worst = st;
    }
    for (int k = 0; k < n; ++k) HIPCHK(hipStreamSynchronize(hs[k]->stream));
    return worst;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

}  // namespace

// ============================================================================
// C-ABI
// ============================================================================
struct spfd_ctx : Ctx {};

#define API_GUARD(c)                                                                 \
    catch (const HipFail &f)                                                         \
    {                                                                                \
        (c)->err = std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.e); \
        return f.e == hipErrorOutOfMemory ? SPFD_OUT_OF_MEMORY : SPFD_HIP_ERROR;     \
    }                                                                                \
    catch (...)                                                                      \
    {                                                                                \
        (c)->err = "internal error";                                                 \
        return SPFD_HIP_ERROR;                                                       \
    }

extern "C" {

spfd_status spfd_create(int device, void *hip_stream, const spfd_allocator *alloc, spfd_handle *out)
{
    if (!out) return SPFD_INVALID_ARG;
    *out = nullptr;
    if (alloc && (!alloc->alloc != !alloc->free)) return SPFD_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SPFD_INVALID_ARG;
    spfd_ctx *c = new (std::nothrow) spfd_ctx();
    if (!c) return SPFD_OUT_OF_MEMORY;
    c->device = device;
    c->user_stream = (hipStream_t)hip_stream;
    if (alloc && alloc->alloc) c->alloc = *alloc;
    try {
        HIPCHK(hipSetDevice(device));
        // own stream (default priority, no implicit sync with the null stream), ordered after the caller's
        HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        for (hipEvent_t &e : c->ev_side) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_user, hipEventDisableTiming));
        for (hipEvent_t &e : c->ev_it) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->d_ints = dalloc<int>(c, c->geo_allocs, 64);
        HIPCHK(hipHostMalloc((void **)&c->h_ints, 64 * sizeof(int), hipHostMallocDefault));
    } catch (const HipFail &f) {
        release_device(c);
        if (c->ev_user) (void)hipEventDestroy(c->ev_user);
        for (hipEvent_t e : c->ev_it)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : c->ev_side)
            if (e) (void)hipEventDestroy(e);
        if (c->side) (void)hipStreamDestroy(c->side);
        if (c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return f.e == hipErrorOutOfMemory ? SPFD_OUT_OF_MEMORY : SPFD_HIP_ERROR;
    }
    *out = c;
    return SPFD_OK;
}

void spfd_destroy(spfd_handle h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->side) (void)hipStreamSynchronize(h->side);
    drop_graphs(h);
    release_device(h);
    if (h->h_scal) (void)hipHostFree(h->h_scal);
    if (h->h_ring) (void)hipHostFree(h->h_ring);
    for (hipEvent_t e : h->ev_it)
        if (e) (void)hipEventDestroy(e);
    if (h->h_ints) (void)hipHostFree(h->h_ints);
    if (h->h_stage) (void)hipHostFree(h->h_stage);
    for (int k = 0; k < SPFD_K_COUNT; ++k)
        for (hipEvent_t e : h->tev[k]) (void)hipEventDestroy(e);
    if (h->ev_user) (void)hipEventDestroy(h->ev_user);
    for (hipEvent_t e : h->ev_side)
        if (e) (void)hipEventDestroy(e);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char *spfd_last_error(spfd_handle h) { return h ? h->err.c_str() : "null handle"; }

// labels NULL: every voxel air (the packed grid of several models, filled by the caller)
spfd_status set_geometry(spfd_handle h, int nx, int ny, int nz, double hx, double hy, double hz, const uint8_t *labels)
{
    const long long nvox = (long long)nx * ny * nz;
    const long long nn = (long long)(nx + 1) * (ny + 1) * (nz + 1);
    if (nn > 0x7fffffffLL * 4) return fail(h, SPFD_INVALID_ARG, "grid too large");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        HIPCHK(hipStreamSynchronize(h->stream));
        HIPCHK(hipStreamSynchronize(h->side));
        free_all(h, h->rhs_allocs);
        free_all(h, h->hier_allocs);
        free_all(h, h->geo_allocs);
        h->d_adj_b = h->d_adj_c = h->d_adj_lam = h->d_adj_labpart = h->d_adj_labout = nullptr;
        h->d_adj_scal = nullptr;
        h->d_sel_work = nullptr;
        h->d_sel_out = nullptr;
        h->d_fgV = nullptr;
        h->d_fgZ = nullptr;
        h->d_fgst = nullptr;
        h->d_fgpart = nullptr;
        h->fg_m = 0;
        h->d_ints = dalloc<int>(h, h->geo_allocs, 64);
        h->lv.clear();
        h->g.nx = nx; h->g.ny = ny; h->g.nz = nz;
        h->g.Nx = nx + 1; h->g.Ny = ny + 1; h->g.Nz = nz + 1;
        h->g.Gx = (nx + 1 + 7) / 8; h->g.Gy = (ny + 1 + 7) / 8; h->g.Gz = (nz + 1 + 7) / 8;
        h->h[0] = hx; h->h[1] = hy; h->h[2] = hz;
        // dual facet area / edge length / 4 (one quarter per voxel sharing the edge)
        h->geo4[0] = 0.25 * (hy * hz / hx);
        h->geo4[1] = 0.25 * (hx * hz / hy);
        h->geo4[2] = 0.25 * (hx * hy / hz);
        h->np = 0;
        h->d_mtables = nullptr;
        h->seg_cache.clear();
        h->d_labels = dalloc<uint8_t>(h, h->geo_allocs, nvox);
        if (labels)
            HIPCHK(hipMemcpyAsync(h->d_labels, labels, nvox, hipMemcpyDefault, h->stream));
        else
            HIPCHK(hipMemsetAsync(h->d_labels, 0, nvox, h->stream));
        h->d_table64 = dalloc<double>(h, h->geo_allocs, MAX_LABELS);
        h->d_table32 = dalloc<float>(h, h->geo_allocs, MAX_LABELS);
        h->d_sigvox = nullptr;
        h->voxel_mode = false;
        h->nlab = 0;
        HIPCHK(hipStreamSynchronize(h->stream));
        h->state = 1;
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_set_geometry(spfd_handle h, int nx, int ny, int nz, double hx, double hy, double hz,
                              const uint8_t *labels)
{
    if (!h) return SPFD_INVALID_ARG;
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(h, SPFD_INVALID_ARG, "grid sizes must be positive");
    if (!finite_pos(hx) || !finite_pos(hy) || !finite_pos(hz)) return fail(h, SPFD_INVALID_ARG, "voxel sizes must be finite and positive");
    if (!labels) return fail(h, SPFD_INVALID_ARG, "labels is NULL");
    return set_geometry(h, nx, ny, nz, hx, hy, hz, labels);
}

spfd_status spfd_set_sigma_table(spfd_handle h, const double *sigma, int n_labels)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->np) return fail(h, SPFD_BAD_STATE, "not available for packed voxel models (spfd_set_geometry_many)");
    if (h->state < 1) return fail(h, SPFD_BAD_STATE, "set_geometry first");
    if (!sigma || n_labels <= 0 || n_labels > MAX_LABELS) return fail(h, SPFD_INVALID_ARG, "need 1..256 labels");
    for (int i = 0; i < n_labels; ++i)
        if (!isfinite(sigma[i]) || sigma[i] < 0.0) return fail(h, SPFD_INVALID_ARG, "sigma must be finite and >= 0");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        float t32[MAX_LABELS];
        for (int i = 0; i < MAX_LABELS; ++i) {
            h->table[i] = i < n_labels ? sigma[i] : 0.0;
            t32[i] = (float)h->table[i];
        }
        HIPCHK(hipMemcpyAsync(h->d_table64, h->table, sizeof(double) * MAX_LABELS, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d_table32, t32, sizeof(float) * MAX_LABELS, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->nlab = n_labels;
        h->voxel_mode = false;
        h->state = 2;
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_set_sigma_voxel(spfd_handle h, const double *sigma_voxel)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->np) return fail(h, SPFD_BAD_STATE, "not available for packed voxel models (spfd_set_geometry_many)");
    if (h->state < 1) return fail(h, SPFD_BAD_STATE, "set_geometry first");
    if (!sigma_voxel) return fail(h, SPFD_INVALID_ARG, "sigma_voxel is NULL");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        const long long nvox = (long long)h->g.nx * h->g.ny * h->g.nz;
        if (!h->d_sigvox) h->d_sigvox = dalloc<double>(h, h->geo_allocs, nvox);
        HIPCHK(hipMemcpyAsync(h->d_sigvox, sigma_voxel, nvox * sizeof(double), hipMemcpyDefault, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->voxel_mode = true;
        if (h->nlab == 0) h->nlab = 1;
        h->state = 2;
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_set_geometry_many(spfd_handle h, int n, const int *dims, double hx, double hy, double hz,
                                   const uint8_t *const *labels)
{
    if (!h) return SPFD_INVALID_ARG;
    if (n < 1 || n > MAX_MODELS) return fail(h, SPFD_INVALID_ARG, "n must be in 1..16");
    if (!dims || !labels) return fail(h, SPFD_INVALID_ARG, "dims and labels are required");
    if (!finite_pos(hx) || !finite_pos(hy) || !finite_pos(hz)) return fail(h, SPFD_INVALID_ARG, "voxel sizes must be finite and positive");
    ModelBoxes mb{};
    mb.np = n;
    int NX = 0, NY = 0;
    long long z = 0;
    for (int m = 0; m < n; ++m) {
        const int nx = dims[3 * m], ny = dims[3 * m + 1], nz = dims[3 * m + 2];
        if (nx <= 0 || ny <= 0 || nz <= 0) return fail(h, SPFD_INVALID_ARG, "grid sizes must be positive");
        if (!labels[m]) return fail(h, SPFD_INVALID_ARG, "a label pointer is NULL");
        mb.nx[m] = nx;
        mb.ny[m] = ny;
        mb.nz[m] = nz;
        mb.zoff[m] = (int)z;
        NX = std::max(NX, nx);
        NY = std::max(NY, ny);
        // the next model starts on the next aligned node layer above this model's top node layer
        z = (z + nz + 1 + MODEL_ALIGN - 1) / MODEL_ALIGN * MODEL_ALIGN;
        if (z > (1 << 24)) return fail(h, SPFD_INVALID_ARG, "models too large");
    }
    const int NZ = mb.zoff[n - 1] + mb.nz[n - 1];
    const long long nn = (long long)(NX + 1) * (NY + 1) * (NZ + 1);
    if (nn > 0x7fffffffLL * 4) return fail(h, SPFD_INVALID_ARG, "models too large");
    const spfd_status st = set_geometry(h, NX, NY, NZ, hx, hy, hz, nullptr);
    if (st != SPFD_OK) return st;
    try {
        for (int m = 0; m < n; ++m)
            HIPCHK(launch_pack_labels(labels[m], mb.nx[m], mb.ny[m], mb.nz[m], h->d_labels, NX, NY, mb.zoff[m],
                                      h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->np = n;
        h->mbox = mb;
        long long off = 0;
        for (int m = 0; m < n; ++m) {
            Grid &g = h->mgrid[m];
            g.nx = mb.nx[m]; g.ny = mb.ny[m]; g.nz = mb.nz[m];
            g.Nx = g.nx + 1; g.Ny = g.ny + 1; g.Nz = g.nz + 1;
            g.Gx = (g.Nx + 7) / 8; g.Gy = (g.Ny + 7) / 8; g.Gz = (g.Nz + 7) / 8;
            h->mnodes_off[m] = off;
            off += (long long)g.Nx * g.Ny * g.Nz;
        }
        h->mnodes_off[n] = off;
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_set_sigma_tables(spfd_handle h, const double *const *tables, const int *n_labels)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 1 || !h->np) return fail(h, SPFD_BAD_STATE, "set_geometry_many first");
    if (!tables || !n_labels) return fail(h, SPFD_INVALID_ARG, "tables and n_labels are required");
    // labels a model's table does not cover get NaN: the build rejects them (non-finite conductivity)
    std::vector<double> tab((size_t)h->np * MAX_LABELS, NAN);
    for (int m = 0; m < h->np; ++m) {
        if (!tables[m] || n_labels[m] < 1 || n_labels[m] > MAX_LABELS)
            return fail(h, SPFD_INVALID_ARG, "each model needs a table of 1..256 conductivities");
        for (int l = 0; l < n_labels[m]; ++l) {
            const double v = tables[m][l];
            if (!isfinite(v) || v < 0.0) return fail(h, SPFD_INVALID_ARG, "conductivities must be finite and >= 0");
            tab[(size_t)m * MAX_LABELS + l] = v;
        }
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        const long long nvox = (long long)h->g.nx * h->g.ny * h->g.nz;
        if (!h->d_mtables) h->d_mtables = dalloc<double>(h, h->geo_allocs, (size_t)MAX_MODELS * MAX_LABELS);
        double *dt = h->d_mtables;
        HIPCHK(hipMemcpyAsync(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
        if (!h->d_sigvox) h->d_sigvox = dalloc<double>(h, h->geo_allocs, nvox);
        HIPCHK(launch_pack_sigma(h->d_labels, h->g, h->mbox, dt, h->d_sigvox, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->voxel_mode = true;
        h->nlab = MAX_LABELS;
        h->state = 2;
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_build(spfd_handle h, const spfd_amg_options *opt)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 2) return fail(h, SPFD_BAD_STATE, "set geometry and conductivities first");
    spfd_amg_options o{};
    if (opt) o = *opt;
    const bool tune = o.short_segment_bricks == 0;   // the default: segments tuned per level
    if (o.cycle != SPFD_CYCLE_V) return fail(h, SPFD_INVALID_ARG, "unknown cycle (only SPFD_CYCLE_V)");
    if (o.cg_window != 0 && (o.cg_window < 2 || o.cg_window > MAX_PHIST || (o.cg_window & 1)))
        return fail(h, SPFD_INVALID_ARG, "cg_window must be 0 or an even number from 2 to 32");
    if (o.smoother != SPFD_SMOOTH_CHEBYSHEV && o.smoother != SPFD_SMOOTH_L1_JACOBI && o.smoother != SPFD_SMOOTH_CHEBYSHEV4)
        return fail(h, SPFD_INVALID_ARG, "unknown smoother");
    set_defaults(o);
    // packed models sit MODEL_ALIGN node layers apart: bricks of the structured levels up to level 3
    // (64 fine nodes) never span two models, and split aggregates never do
    if (h->np && (o.no_split || o.split_level > 3))
        return fail(h, SPFD_INVALID_ARG, "packed voxel models need split aggregation from level 3 or finer");
    h->opt = o;
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        spfd_status s = do_build(h);
        if (s == SPFD_OK && h->np) s = model_ranges(h);
        if (s != SPFD_OK) {
            h->state = 2;
            return s;
        }
        h->state = 3;
        s = do_set_num_rhs(h, 1);
        if (s == SPFD_OK && tune) tune_segments(h);
        return s;
    }
    API_GUARD(h)
}

spfd_status spfd_get_info(spfd_handle h, long long *n_dofs, int *n_components, int *n_levels, size_t *device_bytes)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 3) return fail(h, SPFD_BAD_STATE, "build first");
    if (n_dofs) *n_dofs = h->lv[0].dofs;
    if (n_components) *n_components = h->ncomp;
    if (n_levels) *n_levels = (int)h->lv.size();
    if (device_bytes) *device_bytes = h->bytes;
    return SPFD_OK;
}

spfd_status spfd_level_info(spfd_handle h, int level, int *kind, long long *unknowns, long long *slots,
                            int *row_entries, int *segment)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 3) return fail(h, SPFD_BAD_STATE, "build first");
    if (level < 0 || level >= (int)h->lv.size()) return fail(h, SPFD_INVALID_ARG, "level out of range");
    const Level &L = h->lv[level];
    if (kind) *kind = L.ell ? 1 : 0;
    if (unknowns) *unknowns = L.ell ? (long long)L.nrow : L.dofs;
    if (slots) *slots = L.nodes();
    if (row_entries) *row_entries = L.ell ? 1 + L.K : 7;
    if (segment) {
        const bool fp32 = h->opt.precision == SPFD_MIXED;
        if (L.ell || level + 1 == (int)h->lv.size())
            *segment = 0;
        else if (!fp32)
            *segment = 4;
        else if (level == 0 && !h->voxel_mode)
            *segment = 8;
        else
            *segment = L.seg ? L.seg : (L.nb < h->opt.short_segment_bricks ? 4 : 8);
    }
    return SPFD_OK;
}

spfd_status spfd_set_num_rhs(spfd_handle h, int nrhs)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 3) return fail(h, SPFD_BAD_STATE, "build first");
    if (nrhs <= 0 || nrhs > 4096) return fail(h, SPFD_INVALID_ARG, "nrhs must be in 1..4096");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        return do_set_num_rhs(h, nrhs);
    }
    API_GUARD(h)
}

spfd_status spfd_set_source(spfd_handle h, int rhs, const double *a)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 3) return fail(h, SPFD_BAD_STATE, "build first");
    if (rhs < 0 || rhs >= h->nrhs) return fail(h, SPFD_INVALID_ARG, "rhs index out of range");
    if (!a) return fail(h, SPFD_INVALID_ARG, "a is NULL");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        Level &L0 = h->lv[0];
        HIPCHK(hipMemsetAsync(h->d_scal + rhs, 0, sizeof(Scal), h->stream));
        if (h->np) {
            // model rhs: its bricks of the shared vector, its dense a, ||b||^2 from its own row of partials
            Topo t = L0.topo();
            t.np = 1;
            t.prange = h->d_mrange + rhs;
            t.pmax = h->mcount[rhs];
            double *part = h->d_part + (long long)rhs * h->pstride;
            {
                TScope ts(h, SPFD_K_RHS, (double)t.pmax * BS * (24.0 + 8.0 + op_bytes<double>(h, 0)));
                HIPCHK(launch_rhs(level_op<double>(h, 0), t, L0.d_coord, h->mgrid[rhs], a, h->d_bs, part,
                                  h->d_scal + rhs, h->stream, h->mbox.zoff[rhs]));
            }
            HIPCHK(launch_finish(part, t.pmax, FIN_BB, h->d_scal + rhs, 0, h->stream));
        } else {
            {
                TScope ts(h, SPFD_K_RHS, (double)L0.dofs * (24.0 + 8.0 + op_bytes<double>(h, 0)));
                HIPCHK(launch_rhs(level_op<double>(h, 0), L0.topo(), L0.d_coord, h->g, a, h->d_bs + rhs * L0.nodes(),
                                  h->d_part, h->d_scal + rhs, h->stream));
            }
            finish(h, L0.nb, FIN_BB, h->d_scal + rhs, 0);
        }
        HIPCHK(hipMemcpyAsync(h->h_scal + rhs, h->d_scal + rhs, sizeof(Scal), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (!isfinite(h->h_scal[rhs].bb)) return fail(h, SPFD_INVALID_ARG, "source potentials must be finite");
        h->has_source[rhs] = 1;
        h->state = 4;
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_solve(spfd_handle h, const spfd_solve_options *opt, double *psi, spfd_rhs_info *info)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->state < 4) return fail(h, SPFD_BAD_STATE, "set the sources first");
    for (int i = 0; i < h->nrhs; ++i)
        if (!h->has_source[i]) return fail(h, SPFD_BAD_STATE, "a right-hand side has no source");
    if (!psi) return fail(h, SPFD_INVALID_ARG, "psi is NULL");
    spfd_solve_options so{};
    so.rel_tol = 1e-8;
    so.max_iter = 500;
    if (opt) so = *opt;
    if (!(so.rel_tol > 0.0) || !isfinite(so.rel_tol)) return fail(h, SPFD_INVALID_ARG, "rel_tol must be positive");
    if (so.max_iter <= 0) return fail(h, SPFD_INVALID_ARG, "max_iter must be positive");
    if (const char *e = check_method(so, h->np ? 2 : h->nrhs)) return fail(h, SPFD_INVALID_ARG, e);
    if (h->np && so.use_x0) return fail(h, SPFD_INVALID_ARG, "packed voxel models start from zero (use_x0 = 0)");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        return do_solve(h, so, psi, info);
    }
    API_GUARD(h)
}

spfd_status spfd_efield(spfd_handle h, double omega, int nsrc, const double *a, const double *psi, double *u_edges,
                        double *emag)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->np) return fail(h, SPFD_BAD_STATE, "not available for packed voxel models (spfd_set_geometry_many)");
    if (h->state < 2) return fail(h, SPFD_BAD_STATE, "set geometry and conductivities first");
    if (!a || !psi || !emag) return fail(h, SPFD_INVALID_ARG, "a, psi and emag are required");
    if (nsrc < 1) return fail(h, SPFD_INVALID_ARG, "nsrc must be >= 1");
    if (!isfinite(omega)) return fail(h, SPFD_INVALID_ARG, "omega must be finite");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        const double *sv = h->voxel_mode ? h->d_sigvox : nullptr;
        const long long nvl = (long long)h->g.nx * h->g.ny * h->g.nz;
        const long long nnl = (long long)h->g.Nx * h->g.Ny * h->g.Nz;
        const double nvox = (double)nvl, nn = (double)nnl;
        const double body = h->state >= 3 ? (double)h->lv[0].dofs : nvox;
        for (int k = 0; k < nsrc; ++k) {
            const double *ak = a + (long long)k * 3 * nnl;
            const double *pk = psi + (long long)k * nnl;
            {
                // labels of all voxels, |E| of all voxels; psi (8 corners) and a (12 edges) counted once per body node
                TScope ts(h, SPFD_K_EFIELD, nvox * (1.0 + 8.0) + body * (8.0 + 24.0));
                HIPCHK(launch_efield(h->d_labels, h->d_table64, sv, h->g, h->h, omega, ak, pk, emag + k * nvl,
                                     h->stream));
            }
            if (u_edges) {
                TScope ts(h, SPFD_K_EFIELD, nvox * 1.0 + nn * 24.0 + body * (8.0 + 24.0));
                HIPCHK(launch_uedges(h->d_labels, h->d_table64, sv, h->g, ak, pk, u_edges + (long long)k * 3 * nnl,
                                     h->stream));
            }
        }
        HIPCHK(hipStreamSynchronize(h->stream));
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_adjoint(spfd_handle h, double omega, const double *a, const double *psi, const double *grad_emag,
                         const spfd_solve_options *opt, double *grad_sigma_voxel, double *grad_sigma_table,
                         spfd_rhs_info *info)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->np) return fail(h, SPFD_BAD_STATE, "not available for packed voxel models (spfd_set_geometry_many)");
    if (h->state < 3) return fail(h, SPFD_BAD_STATE, "build first");
    if (!a || !psi || !grad_emag || !grad_sigma_voxel)
        return fail(h, SPFD_INVALID_ARG, "a, psi, grad_emag and grad_sigma_voxel are required");
    if (!isfinite(omega)) return fail(h, SPFD_INVALID_ARG, "omega must be finite");
    spfd_solve_options so{};
    so.rel_tol = 1e-8;
    so.max_iter = 500;
    if (opt) so = *opt;
    so.use_x0 = 0;
    if (!(so.rel_tol > 0.0) || !isfinite(so.rel_tol)) return fail(h, SPFD_INVALID_ARG, "rel_tol must be positive");
    if (so.max_iter <= 0) return fail(h, SPFD_INVALID_ARG, "max_iter must be positive");
    if (const char *e = check_method(so, 1)) return fail(h, SPFD_INVALID_ARG, e);
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        Level &L0 = h->lv[0];
        const Grid &g = h->g;
        const long long nvox = (long long)g.nx * g.ny * g.nz;
        const long long nn = (long long)g.Nx * g.Ny * g.Nz;
        const int nlab = h->voxel_mode ? MAX_LABELS : h->nlab;
        const int gb = adj_grad_blocks(g);
        if (!h->d_adj_b) {
            h->d_adj_b = dalloc<double>(h, h->hier_allocs, L0.nodes());
            h->d_adj_c = dalloc<double>(h, h->hier_allocs, 3 * nvox);
            h->d_adj_lam = dalloc<double>(h, h->hier_allocs, nn);
            h->d_adj_labpart = dalloc<double>(h, h->hier_allocs, (size_t)gb * MAX_LABELS);
            h->d_adj_labout = dalloc<double>(h, h->hier_allocs, MAX_LABELS);
            h->d_adj_scal = dalloc<Scal>(h, h->hier_allocs, 1);
        }
        const double *sv = h->voxel_mode ? h->d_sigvox : nullptr;
        HIPCHK(hipMemsetAsync(h->d_adj_scal, 0, sizeof(Scal), h->stream));
        {
            TScope ts(h, SPFD_K_RHS, (double)nvox * (1.0 + 8.0 + 24.0) + (double)L0.dofs * (32.0 + 24.0 + 8.0));
            HIPCHK(launch_adj_voxel(h->d_labels, h->d_table64, sv, g, h->h, omega, a, psi, grad_emag, h->d_adj_c,
                                    h->stream));
            HIPCHK(launch_adj_rhs(L0.topo(), L0.d_coord, g, h->d_adj_c, h->d_adj_b, h->d_part, h->stream));
        }
        finish(h, L0.nb, FIN_BB, h->d_adj_scal, 0);
        spfd_rhs_info inf{};
        spfd_status st = solve_batch(h, h->d_adj_b, 0, h->d_adj_scal, h->h_scal + h->nrhs, 1, so, h->d_adj_lam, &inf);
        {
            TScope ts(h, SPFD_K_EFIELD, (double)nvox * (1.0 + 8.0) + (double)L0.dofs * (8.0 + 8.0 + 24.0));
            HIPCHK(launch_adj_grad(h->d_labels, h->d_table64, sv, g, h->geo4, a, psi, h->d_adj_lam, grad_sigma_voxel,
                                   h->d_adj_labpart, nlab, h->d_adj_labout, h->stream));
        }
        if (grad_sigma_table)
            HIPCHK(hipMemcpyAsync(grad_sigma_table, h->d_adj_labout, nlab * sizeof(double), hipMemcpyDeviceToHost,
                                  h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (info) *info = inf;
        if (st != SPFD_OK)
            h->err = st == SPFD_BREAKDOWN ? "breakdown in the adjoint CG" : "adjoint solve did not converge";
        return st;
    }
    API_GUARD(h)
}

spfd_status spfd_solve_many(spfd_handle *hs, int n, const spfd_solve_options *opt, double **psi, spfd_rhs_info *info)
{
    if (!hs || n <= 0 || !psi) return SPFD_INVALID_ARG;
    for (int k = 0; k < n; ++k) {
        if (!hs[k]) return SPFD_INVALID_ARG;
        if (hs[k]->np) return fail(hs[k], SPFD_BAD_STATE, "packed voxel models solve with spfd_solve");
        if (hs[k]->state < 4) return fail(hs[k], SPFD_BAD_STATE, "set the sources first");
        for (int i = 0; i < hs[k]->nrhs; ++i)
            if (!hs[k]->has_source[i]) return fail(hs[k], SPFD_BAD_STATE, "a right-hand side has no source");
        if (!psi[k]) return fail(hs[k], SPFD_INVALID_ARG, "psi is NULL");
        if (hs[k]->device != hs[0]->device) return fail(hs[k], SPFD_INVALID_ARG, "all handles must share one device");
        for (int j = 0; j < k; ++j)
            if (hs[j] == hs[k]) return fail(hs[k], SPFD_INVALID_ARG, "a handle appears twice");
    }
    spfd_solve_options so{};
    so.rel_tol = 1e-8;
    so.max_iter = 500;
    if (opt) so = *opt;
    so.use_x0 = 0;
    if (!(so.rel_tol > 0.0) || !isfinite(so.rel_tol)) return fail(hs[0], SPFD_INVALID_ARG, "rel_tol must be positive");
    if (so.max_iter <= 0) return fail(hs[0], SPFD_INVALID_ARG, "max_iter must be positive");
    if (so.method != SPFD_CG) return fail(hs[0], SPFD_INVALID_ARG, "the lockstep solve uses CG (method SPFD_CG)");
    std::vector<Ctx *> cs(hs, hs + n);
    try {
        HIPCHK(hipSetDevice(hs[0]->device));
        for (Ctx *c : cs) enter(c);
        spfd_status st = solve_many(cs.data(), n, so, psi, info);
        if (st != SPFD_OK) hs[0]->err = "a right-hand side did not converge or broke down";
        return st;
    }
    API_GUARD(hs[0])
}

spfd_status spfd_edge_potentials(spfd_handle h, const double *flux, double *a)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->np) return fail(h, SPFD_BAD_STATE, "not available for packed voxel models (spfd_set_geometry_many)");
    if (h->state < 1) return fail(h, SPFD_BAD_STATE, "set the geometry first");
    if (!flux || !a) return fail(h, SPFD_INVALID_ARG, "flux and a are required");
    if (flux == a) return fail(h, SPFD_INVALID_ARG, "flux and a must not alias");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        const double nn = (double)h->g.Nx * h->g.Ny * h->g.Nz;
        {
            TScope ts(h, SPFD_K_RHS, nn * (16.0 + 24.0));
            HIPCHK(launch_tree_cotree(flux, a, h->g, h->stream));
        }
        HIPCHK(hipStreamSynchronize(h->stream));
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_percentile(spfd_handle h, const double *emag, double q, double *out_body, double *out_labels)
{
    if (!h) return SPFD_INVALID_ARG;
    if (h->np) return fail(h, SPFD_BAD_STATE, "not available for packed voxel models (spfd_set_geometry_many)");
    if (h->state < 2) return fail(h, SPFD_BAD_STATE, "set geometry and conductivities first");
    if (!emag || !out_body) return fail(h, SPFD_INVALID_ARG, "emag and out_body are required");
    if (!(q > 0.0 && q <= 1.0)) return fail(h, SPFD_INVALID_ARG, "q must be in (0, 1]");
    try {
        HIPCHK(hipSetDevice(h->device));
        enter(h);
        const int nlab = h->voxel_mode ? MAX_LABELS : h->nlab;
        const int ng = 1 + nlab;
        if (!h->d_sel_work) {
            h->d_sel_work = dalloc<uint8_t>(h, h->geo_allocs, sel_work_bytes(1 + MAX_LABELS));
            h->d_sel_out = dalloc<double>(h, h->geo_allocs, 1 + MAX_LABELS);
        }
        const long long nvox = (long long)h->g.nx * h->g.ny * h->g.nz;
        {
            TScope ts(h, SPFD_K_EFIELD, 8.0 * nvox * 9.0);
            HIPCHK(launch_quantiles(h->d_labels, h->d_table64, h->voxel_mode ? h->d_sigvox : nullptr, nvox, emag, ng, q,
                                    h->d_sel_work, h->d_sel_out, h->stream));
        }
        double out[1 + MAX_LABELS];
        HIPCHK(hipMemcpyAsync(out, h->d_sel_out, ng * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        *out_body = out[0];
        if (out_labels)
            for (int l = 0; l < nlab; ++l) out_labels[l] = out[1 + l];
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_timing(spfd_handle h, unsigned int class_mask)
{
    if (!h) return SPFD_INVALID_ARG;
    try {
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->tcold = (class_mask & SPFD_TIMING_COLD) != 0;
        h->tmask = class_mask & ~(unsigned)SPFD_TIMING_COLD;
        if (h->tcold && !h->d_flush) {
            h->d_flush = dalloc<uint8_t>(h, h->flush_allocs, FLUSH_BYTES);
            HIPCHK(hipMemsetAsync(h->d_flush, 0, FLUSH_BYTES, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        } else if (!h->tcold && h->d_flush) {
            free_all(h, h->flush_allocs);
            h->d_flush = nullptr;
        }
        for (int k = 0; k < SPFD_K_COUNT; ++k) {
            h->tused[k] = 0;
            h->tlaunch[k] = 0;
            h->tbytes[k] = 0.0;
            h->ttimed[k] = 0;
            h->ttbytes[k] = 0.0;
        }
        return SPFD_OK;
    }
    API_GUARD(h)
}

spfd_status spfd_timing_get(spfd_handle h, int kclass, long long *launches, double *algorithmic_bytes,
                            long long *timed_launches, double *timed_ms, double *timed_bytes)
{
    if (!h) return SPFD_INVALID_ARG;
    if (kclass < 0 || kclass >= SPFD_K_COUNT) return fail(h, SPFD_INVALID_ARG, "unknown kernel class");
    try {
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipStreamSynchronize(h->stream));
        double ms = 0.0;
        const std::vector<hipEvent_t> &v = h->tev[kclass];
        for (size_t i = 0; i + 1 < h->tused[kclass]; i += 2) {
            float e = 0.0f;
            HIPCHK(hipEventElapsedTime(&e, v[i], v[i + 1]));
            ms += e;
        }
        if (launches) *launches = h->tlaunch[kclass];
        if (algorithmic_bytes) *algorithmic_bytes = h->tbytes[kclass];
        if (timed_launches) *timed_launches = h->ttimed[kclass];
        if (timed_ms) *timed_ms = ms;
        if (timed_bytes) *timed_bytes = h->ttbytes[kclass];
        return SPFD_OK;
    }
    API_GUARD(h)
}

}  // extern "C"

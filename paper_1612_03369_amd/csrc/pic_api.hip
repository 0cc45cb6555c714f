// C ABI of the particle hot path: context, mesh set-up, store binding and
// launch sequencing.  The kernels live in pic_kernels.hip / pic_adjoint.hip;
// this file only prepares tables and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cerrno>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pic.h"
#include "pic_kernels.hip"
#include "pic_adjoint.hip"

using namespace pic;

namespace {

struct ProfEvent {
    const char *name;
    hipEvent_t a, b;
};

}  // namespace

// Fixed device scratch of pic_seed_mh_static (the generation call for
// callers that cannot allocate): header words, the cell starts being built
// and the packed density.  Every GPU the library runs on holds its own copy
// until the process ends.  Its address on each device is looked up once, at
// the first pic_create on that device; host code uses that address, never
// the symbol itself.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
namespace {
constexpr int STATIC_MAX_DEVICES = 64;
void *g_scratch_ptr[STATIC_MAX_DEVICES];
hipError_t g_scratch_err[STATIC_MAX_DEVICES];
std::once_flag g_scratch_once[STATIC_MAX_DEVICES];
}  // namespace

struct pic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // mesh
    bool have_mesh = false;
    MeshDev mesh{};
    std::vector<void *> mesh_allocs;
    std::vector<double> node_xyz;        // host copy of Q2 node coordinates
    std::vector<uint8_t> node_hanging;
    std::vector<std::pair<int64_t, int64_t>> hanging;   // (node, constraining leaf), coarse first
    std::vector<int32_t> h_cell_nodes;                  // octree [n_cells][27]
    std::vector<uint8_t> h_level;
    std::vector<int32_t> h_anchor;
    // field
    void *u64 = nullptr, *u32 = nullptr;
    bool have_field = false;
    // field at the end of the field step (time interpolation) and the time
    // elapsed since its start (one double in device memory)
    void *u1_64 = nullptr, *u1_32 = nullptr;
    double *d_tau = nullptr;
    // store
    bool bound = false;
    pic_store store{};
    ScratchDev scr{};
    int tile = 64;
    // device problem descriptor and work lists
    ProblemDev h_prob{};
    ProblemDev *d_prob = nullptr;
    WorkItem *d_work = nullptr;
    int n_work = 0;
    ScanItem *d_scan = nullptr;
    int n_scan = 0;
    RangeItem *d_rp = nullptr;   // particle ranges over the capacity
    int n_rp = 0;
    RangeItem *d_rc = nullptr;   // cell ranges
    int n_rc = 0;
    BlockItem *d_blk[2] = {nullptr, nullptr};   // uniform meshes: cell blocks for F64 / F32 evaluation
    int n_blk[2] = {0, 0};
    BlockItem *d_blk_adj = nullptr;             // uniform meshes: cell blocks of the reverse (adjoint) step
    int n_blk_adj = 0;
    double last_dt = std::nan("");
    // profiling
    bool profile = false;
    std::vector<ProfEvent> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<double, int64_t>> prof;
    // graph of the fused step sequence of pic_advance, captured on a stream of
    // the context's own (the caller's may be the legacy default stream, which
    // cannot be captured) and replayed between events on the two streams;
    // key = {n_steps, scheme, precision, property equations, time field}
    bool graphs = false;
    hipStream_t gstream = nullptr;
    hipEvent_t g_ev[2] = {nullptr, nullptr};
    hipGraph_t g_graph = nullptr;
    hipGraphExec_t g_exec = nullptr;
    int g_key[5] = {-1, -1, -1, -1, -1};
    // adjoint
    int64_t adj_steps = 0, adj_every = 0;
    double adj_dt = 0.0;
    int adj_scheme = 0;
};

namespace {

pic_status fail(pic_ctx *c, pic_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIPCHK(c, expr)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((c), e_ == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                     \
    } while (0)

hipEvent_t take_event(pic_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

// Launch with optional event pair for profiling.
template <typename K, typename... A>
pic_status launch(pic_ctx *c, const char *name, K kernel, unsigned grid, unsigned block, A... args)
{
    if (grid == 0) return PIC_OK;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (c->profile) {
        ea = take_event(c);
        eb = take_event(c);
        (void)hipEventRecord(ea, c->stream);
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, c->stream, args...);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, PIC_EDEVICE, "launch %s: %s", name, hipGetErrorString(e));
    if (c->profile) {
        (void)hipEventRecord(eb, c->stream);
        c->pending.push_back({name, ea, eb});
    }
    return PIC_OK;
}

#define LAUNCH(c, name, kernel, grid, block, ...)                          \
    do {                                                                   \
        pic_status s_ = launch((c), (name), (kernel), (grid), (block), __VA_ARGS__); \
        if (s_ != PIC_OK) return s_;                                       \
    } while (0)

pic_status collect_profile(pic_ctx *c)
{
    if (c->pending.empty()) return PIC_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, p.a, p.b);
        auto &slot = c->prof[p.name];
        slot.first += ms;
        slot.second += 1;
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
    return PIC_OK;
}

template <typename T> pic_status dalloc(pic_ctx *c, T **p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    HIPCHK(c, hipMalloc((void **)p, n * sizeof(T)));
    return PIC_OK;
}

template <typename T> pic_status mesh_upload(pic_ctx *c, const T *host, size_t n, const T **dev)
{
    T *d = nullptr;
    pic_status s = dalloc(c, &d, n);
    if (s) return s;
    c->mesh_allocs.push_back(d);
    HIPCHK(c, hipMemcpy(d, host, n * sizeof(T), hipMemcpyHostToDevice));
    *dev = d;
    return PIC_OK;
}

void drop_adv_graph(pic_ctx *c);
void free_mesh(pic_ctx *c)
{
    drop_adv_graph(c);
    for (void *p : c->mesh_allocs) hipFree(p);
    c->mesh_allocs.clear();
    if (c->u64) hipFree(c->u64);
    if (c->u32) hipFree(c->u32);
    if (c->u1_64) hipFree(c->u1_64);
    if (c->u1_32) hipFree(c->u1_32);
    c->u64 = c->u32 = c->u1_64 = c->u1_32 = nullptr;
    c->h_prob.ti = 0;
    c->have_mesh = false;
    c->node_xyz.clear();
    c->node_hanging.clear();
    c->hanging.clear();
    c->h_cell_nodes.clear();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t n_chunks(int64_t nc) { return (nc + scan_chunk_cells(nc) - 1) / scan_chunk_cells(nc); }

// Layout of the caller's scratch buffer.
size_t scratch_layout(int64_t cap, int64_t nc, char *base, ScratchDev *s)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    char *key0 = take(4 * (size_t)cap);
    char *key1 = take(4 * (size_t)cap);
    char *src = take(4 * (size_t)cap);
    char *stay = take(4 * (size_t)nc);
    char *arr = take(4 * (size_t)nc);
    char *cur = take(4 * (size_t)(nc + 1));
    char *chk = take(8 * (size_t)(n_chunks(nc) + 1));
    char *st = take(8 * (size_t)ST_COUNT * STAT_STRIPES);
    char *nid = take(8 * (size_t)(1 + STAT_STRIPES));
    char *fl = take(16);
    if (s) {
        s->key[0] = (uint32_t PIC_G *)key0;
        s->key[1] = (uint32_t PIC_G *)key1;
        s->src = (int32_t PIC_G *)src;
        s->n_stay = (int32_t PIC_G *)stay;
        s->n_arrive = (int32_t PIC_G *)arr;
        s->cursor = (int32_t PIC_G *)cur;
        s->chunk = (int64_t PIC_G *)chk;
        s->stats = (unsigned long long *)st;
        s->next_id = (unsigned long long *)nid;
        s->flags = (int32_t *)fl;
    }
    return off;
}

// Derived mesh quantities shared by all kinds.
void mesh_common(MeshDev &m)
{
    double hmin[3];
    for (int a = 0; a < 3; ++a) {
        m.h[a] = (m.hi[a] - m.lo[a]) / (m.n[a] > 0 ? m.n[a] : 1);
        m.inv_h[a] = 1.0 / m.h[a];
        hmin[a] = m.kind == MESH_OCTREE ? m.fine_h[a] : m.h[a];
    }
    for (int a = 0; a < 3; ++a) m.bnd_tol[a] = NEAR_TOL * hmin[a];
}

pic_status upload_problem(pic_ctx *c)
{
    if (!c->d_prob) {
        pic_status s = dalloc(c, &c->d_prob, 1);
        if (s) return s;
    }
    if (c->bound) {
        // the current-buffer index is device state (kernels flip it): keep it
        HIPCHK(c, hipMemcpyAsync(&c->h_prob.cur, &c->d_prob->cur, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->d_prob, &c->h_prob, sizeof(ProblemDev), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

#ifndef PIC_USE_BLOCK_ADVECT
#define PIC_USE_BLOCK_ADVECT 1
#endif

std::vector<BlockItem> block_items_shape(const MeshDev &m, const int *b, int problem)
{
    std::vector<BlockItem> v;
    const int nz = m.dim == 3 ? m.n[2] : 1, bz = m.dim == 3 ? b[2] : 1;
    for (int k = 0; k < nz; k += bz)
        for (int j = 0; j < m.n[1]; j += b[1])
            for (int i = 0; i < m.n[0]; i += b[0]) v.push_back({problem, i, j, k});
    return v;
}

std::vector<BlockItem> block_items(const MeshDev &m, int prec, int problem)
{
    const int *b = block_shape(m.dim, prec);
    std::vector<BlockItem> v;
    const int nz = m.dim == 3 ? m.n[2] : 1, bz = m.dim == 3 ? b[2] : 1;
    for (int k = 0; k < nz; k += bz)
        for (int j = 0; j < m.n[1]; j += b[1])
            for (int i = 0; i < m.n[0]; i += b[0]) v.push_back({problem, i, j, k});
    return v;
}

void drop_adv_graph(pic_ctx *c)
{
    if (c->g_exec) hipGraphExecDestroy(c->g_exec);
    if (c->g_graph) hipGraphDestroy(c->g_graph);
    c->g_exec = nullptr;
    c->g_graph = nullptr;
    for (int &k : c->g_key) k = -1;
}

// Work lists for one problem (a captured step sequence holds their pointers).
pic_status build_work(pic_ctx *c)
{
    drop_adv_graph(c);
    const int64_t nc = c->mesh.n_cells;
    const int64_t cap = c->store.capacity;
    std::vector<WorkItem> w;
    // octree tiles hold at most OCT_TILE leaves (their nodes are staged in LDS)
    const int64_t tile = c->mesh.kind == MESH_OCTREE ? std::min(c->tile, OCT_TILE) : c->tile;
    for (int64_t k = 0; k < nc; k += tile) w.push_back({0, (int32_t)k, (int32_t)std::min<int64_t>(nc, k + tile)});
    std::vector<ScanItem> sc;
    for (int64_t k = 0; k < n_chunks(nc); ++k) sc.push_back({0, (int32_t)k});
    std::vector<RangeItem> rp, rc;
    for (int64_t k = 0; k < cap; k += BLOCK) rp.push_back({0, 0, k, std::min<int64_t>(cap, k + BLOCK)});
    for (int64_t k = 0; k < nc; k += BLOCK) rc.push_back({0, 0, k, std::min<int64_t>(nc, k + BLOCK)});
    for (void *p : {(void *)c->d_work, (void *)c->d_scan, (void *)c->d_rp, (void *)c->d_rc})
        if (p) hipFree(p);
    c->d_work = nullptr;
    c->d_scan = nullptr;
    c->d_rp = nullptr;
    c->d_rc = nullptr;
    pic_status s;
    if ((s = dalloc(c, &c->d_work, w.size()))) return s;
    if ((s = dalloc(c, &c->d_scan, sc.size()))) return s;
    if ((s = dalloc(c, &c->d_rp, rp.size()))) return s;
    if ((s = dalloc(c, &c->d_rc, rc.size()))) return s;
    HIPCHK(c, hipMemcpy(c->d_work, w.data(), w.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_scan, sc.data(), sc.size() * sizeof(ScanItem), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_rp, rp.data(), rp.size() * sizeof(RangeItem), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_rc, rc.data(), rc.size() * sizeof(RangeItem), hipMemcpyHostToDevice));
    for (int pr = 0; pr < 2; ++pr) {
        if (c->d_blk[pr]) hipFree(c->d_blk[pr]);
        c->d_blk[pr] = nullptr;
        c->n_blk[pr] = 0;
        if (c->mesh.kind != MESH_UNIFORM) continue;
        std::vector<BlockItem> bl = block_items(c->mesh, pr, 0);
        if ((s = dalloc(c, &c->d_blk[pr], bl.size()))) return s;
        HIPCHK(c, hipMemcpy(c->d_blk[pr], bl.data(), bl.size() * sizeof(BlockItem), hipMemcpyHostToDevice));
        c->n_blk[pr] = (int)bl.size();
    }
    if (c->d_blk_adj) hipFree(c->d_blk_adj);
    c->d_blk_adj = nullptr;
    c->n_blk_adj = 0;
    if (c->mesh.kind == MESH_UNIFORM) {
        std::vector<BlockItem> bl = block_items_shape(c->mesh, c->mesh.dim == 3 ? ADJ3 : ADJ2, 0);
        if ((s = dalloc(c, &c->d_blk_adj, bl.size()))) return s;
        HIPCHK(c, hipMemcpy(c->d_blk_adj, bl.data(), bl.size() * sizeof(BlockItem), hipMemcpyHostToDevice));
        c->n_blk_adj = (int)bl.size();
    }
    c->n_work = (int)w.size();
    c->n_scan = (int)sc.size();
    c->n_rp = (int)rp.size();
    c->n_rc = (int)rc.size();
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// kernel dispatch over (dim, scheme, precision, mesh kind)
// ---------------------------------------------------------------------------
pic_status require_ready(pic_ctx *c, bool field)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_mesh) return fail(c, PIC_ESTATE, "no mesh");
    if (!c->bound) return fail(c, PIC_ESTATE, "no store bound");
    if (field && !c->have_field) return fail(c, PIC_ESTATE, "no velocity field");
    return PIC_OK;
}

pic_status set_dt(pic_ctx *c, double dt)
{
    if (dt == c->last_dt) return PIC_OK;
    c->last_dt = dt;
    c->h_prob.dt = dt;
    HIPCHK(c, hipMemcpyAsync(&c->d_prob->dt, &c->h_prob.dt, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

// scan (mode 0: stayers + arrivals, 1: population packed); flip: the buffer
// flip of a fused step is still pending (mode 0 only)
template <int MODE, int PT> pic_status enqueue_scan_t(pic_ctx *c, ProblemDev *dp, bool flip)
{
    LAUNCH(c, "scan_reduce", (k_scan_reduce<MODE, PT>), (unsigned)c->n_scan, BLOCK, (const ProblemDev *)dp, (const ScanItem *)c->d_scan,
           c->n_scan, dp, flip ? 1 : 0);
    LAUNCH(c, "scan_down", (k_scan_down<MODE, PT>), (unsigned)c->n_scan, BLOCK, (const ProblemDev *)dp, (const ScanItem *)c->d_scan,
           c->n_scan);
    return PIC_OK;
}
pic_status enqueue_scan(pic_ctx *c, ProblemDev *dp, int mode, bool flip = false)
{
    const bool short_chunks = scan_per_thread(c->mesh.n_cells) == 2;
    if (mode == 0) return short_chunks ? enqueue_scan_t<0, 2>(c, dp, flip) : enqueue_scan_t<0, SCAN_PT_MAX>(c, dp, flip);
    return short_chunks ? enqueue_scan_t<1, 2>(c, dp, false) : enqueue_scan_t<1, SCAN_PT_MAX>(c, dp, false);
}

// arrival order after the placement of a buffer sorted by cell
pic_status enqueue_fix_sorted(pic_ctx *c, ProblemDev *dp)
{
    LAUNCH(c, "fix", k_fix, (unsigned)xcd_span(c->n_rc), BLOCK, (const ProblemDev *)dp, (const RangeItem *)c->d_rc, c->n_rc);
    return PIC_OK;
}

// place + fix + gather + flip after the counts are in n_stay / n_arrive;
// unsorted = the current buffer is an unsorted input (every particle arrives);
// flip = a fused step's flip is pending (done by the scan)
pic_status enqueue_sort(pic_ctx *c, ProblemDev *dp, int count_step, bool unsorted = false, bool flip = false)
{
    pic_status s = enqueue_scan(c, dp, 0, flip);
    if (s) return s;
    if (unsorted) {
        LAUNCH(c, "place", k_place_unsorted, (unsigned)c->n_rp, BLOCK, (const ProblemDev *)dp, (const RangeItem *)c->d_rp, c->n_rp);
        LAUNCH(c, "fix", k_fix, (unsigned)xcd_span(c->n_rc), BLOCK, (const ProblemDev *)dp, (const RangeItem *)c->d_rc, c->n_rc);
    } else {
        LAUNCH(c, "place", k_place_waves, (unsigned)xcd_span(c->n_work), BLOCK, (const ProblemDev *)dp, (const WorkItem *)c->d_work, c->n_work);
        if ((s = enqueue_fix_sorted(c, dp))) return s;
    }
    LAUNCH(c, "gather", k_gather, (unsigned)xcd_span(c->n_rp), BLOCK, (const ProblemDev *)dp, (const RangeItem *)c->d_rp, c->n_rp);
    LAUNCH(c, "flip", k_flip, 1u, 64u, dp, 1, count_step);
    return PIC_OK;
}

#ifndef PIC_FUSE_STEPS
#define PIC_FUSE_STEPS 1
#endif
// n steps on a uniform mesh: the first step's advect, then n-1 times
// (re-sort fused with the next advect), then the last re-sort.  Identical
// arithmetic to n separate steps.  The buffer flip after a fused advect is
// done by the scan that follows it.
pic_status enqueue_steps_fused(pic_ctx *c, ProblemDev *dp, int scheme, int prec, int n)
{
    const int pr = prec == PIC_F32;
    const bool ode = dp == c->d_prob && c->h_prob.odes != 0;
    const bool ti = dp == c->d_prob && c->h_prob.ti != 0;
    BlockFn fa = block_kernel(c->mesh.dim, scheme, prec, false, ode, ti);
    BlockFn ff = block_kernel(c->mesh.dim, scheme, prec, true, ode, ti);
    LAUNCH(c, "advect", fa, (unsigned)xcd_span(c->n_blk[pr]), ADV_BLOCK, (const ProblemDev *)dp, (const BlockItem *)c->d_blk[pr], c->n_blk[pr]);
    for (int k = 1; k < n; ++k) {
        pic_status s = enqueue_scan(c, dp, 0, k > 1);
        if (s) return s;
        LAUNCH(c, "place", k_place_waves, (unsigned)xcd_span(c->n_work), BLOCK, (const ProblemDev *)dp, (const WorkItem *)c->d_work, c->n_work);
        if ((s = enqueue_fix_sorted(c, dp))) return s;
        LAUNCH(c, "gather_advect", ff, (unsigned)xcd_span(c->n_blk[pr]), ADV_BLOCK, (const ProblemDev *)dp, (const BlockItem *)c->d_blk[pr], c->n_blk[pr]);
    }
    return enqueue_sort(c, dp, 1, false, n > 1);
}

pic_status enqueue_step(pic_ctx *c, ProblemDev *dp, int scheme, int prec)
{
    const bool ode = dp == c->d_prob && c->h_prob.odes != 0;
    const bool ti = dp == c->d_prob && c->h_prob.ti != 0;
    if (PIC_USE_BLOCK_ADVECT && c->mesh.kind == MESH_UNIFORM && c->n_blk[prec == PIC_F32]) {
        BlockFn f = block_kernel(c->mesh.dim, scheme, prec, false, ode, ti);
        const int pr = prec == PIC_F32;
        LAUNCH(c, "advect", f, (unsigned)xcd_span(c->n_blk[pr]), ADV_BLOCK, (const ProblemDev *)dp, (const BlockItem *)c->d_blk[pr],
               c->n_blk[pr]);
        return enqueue_sort(c, dp, 1);
    }
    AdvectFn f = advect_kernel(c->mesh.dim, scheme, prec, c->mesh.kind, ode, ti);
    if (!f) return fail(c, PIC_EINVAL, "unsupported combination dim=%d scheme=%d kind=%d", c->mesh.dim, scheme, c->mesh.kind);
    LAUNCH(c, "advect", f, (unsigned)xcd_span(c->n_work), BLOCK, (const ProblemDev *)dp, (const WorkItem *)c->d_work, c->n_work);
    return enqueue_sort(c, dp, 1);
}

}  // namespace

// ===========================================================================
// context
// ===========================================================================
extern "C" pic_status pic_create(pic_ctx **out, int device, void *stream)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PIC_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return PIC_EDEVICE;
    if (device < STATIC_MAX_DEVICES)
        std::call_once(g_scratch_once[device], [device] {
            g_scratch_err[device] = hipGetSymbolAddress(&g_scratch_ptr[device], HIP_SYMBOL(scratch));
            if (g_scratch_err[device] != hipSuccess) g_scratch_ptr[device] = nullptr;
        });
    pic_ctx *c = new pic_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c;
    return PIC_OK;
}

extern "C" pic_status pic_set_stream(pic_ctx *c, void *stream)
{
    if (!c) return PIC_EINVAL;
    c->stream = (hipStream_t)stream;
    return PIC_OK;
}

extern "C" void pic_destroy(pic_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    if (c->gstream) hipStreamSynchronize(c->gstream);
    drop_adv_graph(c);
    if (c->gstream) hipStreamDestroy(c->gstream);
    for (hipEvent_t e : c->g_ev)
        if (e) hipEventDestroy(e);
    free_mesh(c);
    for (void *p : {c->u64, c->u32, c->u1_64, c->u1_32, (void *)c->d_tau, (void *)c->d_prob, (void *)c->d_work, (void *)c->d_scan, (void *)c->d_rp,
                    (void *)c->d_rc, (void *)c->d_blk[0], (void *)c->d_blk[1], (void *)c->d_blk_adj})
        if (p) hipFree(p);
    for (auto &p : c->pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    for (auto e : c->pool) hipEventDestroy(e);
    delete c;
}

extern "C" const char *pic_last_error(const pic_ctx *c) { return c ? c->err.c_str() : "null context"; }

// ===========================================================================
// meshes
// ===========================================================================
extern "C" pic_status pic_mesh_uniform(pic_ctx *c, int dim, const int32_t n[3], const double lo[3], const double hi[3])
{
    if (!c) return PIC_EINVAL;
    if (dim != 2 && dim != 3) return fail(c, PIC_EINVAL, "dim must be 2 or 3");
    if (!n || !lo || !hi) return fail(c, PIC_EINVAL, "null argument");
    int64_t nc = 1;
    for (int a = 0; a < dim; ++a) {
        if (n[a] < 1) return fail(c, PIC_EINVAL, "n[%d] < 1", a);
        if (!(hi[a] > lo[a])) return fail(c, PIC_EINVAL, "hi[%d] <= lo[%d]", a, a);
        nc *= n[a];
    }
    if (nc >= (int64_t)INT32_MAX) return fail(c, PIC_EINVAL, "too many cells");
    hipSetDevice(c->device);
    free_mesh(c);
    MeshDev m{};
    m.dim = dim;
    m.kind = MESH_UNIFORM;
    for (int a = 0; a < 3; ++a) {
        m.n[a] = a < dim ? n[a] : 1;
        m.lo[a] = a < dim ? lo[a] : 0.0;
        m.hi[a] = a < dim ? hi[a] : 1.0;
    }
    m.nnx = 2 * m.n[0] + 1;
    m.nny = 2 * m.n[1] + 1;
    m.nnz = dim == 3 ? 2 * m.n[2] + 1 : 1;
    m.nvx = m.n[0] + 1;
    m.nvy = m.n[1] + 1;
    m.n_cells = nc;
    m.n_nodes = (int64_t)m.nnx * m.nny * m.nnz;
    m.n_vert = (int64_t)m.nvx * m.nvy * (dim == 3 ? m.n[2] + 1 : 1);
    mesh_common(m);
    c->mesh = m;
    // host node coordinates
    c->node_xyz.assign((size_t)dim * m.n_nodes, 0.0);
    for (int64_t g = 0; g < m.n_nodes; ++g) {
        int64_t a = g % m.nnx, b = (g / m.nnx) % m.nny, cc = g / ((int64_t)m.nnx * m.nny);
        int64_t ii[3] = {a, b, cc};
        for (int q = 0; q < dim; ++q) c->node_xyz[q * m.n_nodes + g] = m.lo[q] + 0.5 * (double)ii[q] * m.h[q];
    }
    c->have_mesh = true;
    c->have_field = false;
    c->bound = false;
    return PIC_OK;
}

extern "C" pic_status pic_mesh_displace(pic_ctx *c, const double *vertices)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_mesh || c->mesh.kind != MESH_UNIFORM) return fail(c, PIC_ESTATE, "displace needs a uniform mesh first");
    if (!vertices) return fail(c, PIC_EINVAL, "null vertices");
    MeshDev &m = c->mesh;
    const int d = m.dim;
    // boundary vertices must stay on their faces
    for (int64_t g = 0; g < m.n_vert; ++g) {
        int64_t ii[3] = {g % m.nvx, (g / m.nvx) % m.nvy, g / ((int64_t)m.nvx * m.nvy)};
        for (int a = 0; a < d; ++a) {
            double v = vertices[a * m.n_vert + g];
            if (!std::isfinite(v)) return fail(c, PIC_EINVAL, "non-finite vertex");
            if (ii[a] == 0 && v != m.lo[a]) return fail(c, PIC_EINVAL, "boundary vertex %lld left face lo[%d]", (long long)g, a);
            if (ii[a] == m.n[a] && v != m.hi[a]) return fail(c, PIC_EINVAL, "boundary vertex %lld left face hi[%d]", (long long)g, a);
        }
    }
    hipSetDevice(c->device);
    pic_status s = mesh_upload(c, vertices, (size_t)d * m.n_vert, &m.vert);
    if (s) return s;
    m.kind = MESH_DISPLACED;
    // node coordinates: Phi_K of the node's reference point
    std::vector<double> X(8 * 3);
    for (int64_t K = 0; K < m.n_cells; ++K) {
        int ijk[3] = {(int)(K % m.n[0]), (int)((K / m.n[0]) % m.n[1]), d == 3 ? (int)(K / ((int64_t)m.n[0] * m.n[1])) : 0};
        for (int v = 0; v < (1 << d); ++v) {
            int64_t g = (ijk[0] + (v & 1)) + (int64_t)m.nvx * ((ijk[1] + ((v >> 1) & 1)) + (int64_t)m.nvy * (ijk[2] + ((v >> 2) & 1)));
            for (int a = 0; a < d; ++a) X[v * 3 + a] = vertices[a * m.n_vert + g];
        }
        for (int loc = 0; loc < (d == 3 ? 27 : 9); ++loc) {
            int la = loc % 3, lb = (loc / 3) % 3, lc = loc / 9;
            double t[3] = {0.5 * la, 0.5 * lb, 0.5 * lc};
            int64_t g = (2 * ijk[0] + la) + (int64_t)m.nnx * ((2 * ijk[1] + lb) + (int64_t)m.nny * (2 * ijk[2] + lc));
            for (int a = 0; a < d; ++a) {
                double x = 0.0;
                for (int v = 0; v < (1 << d); ++v) {
                    double N = 1.0;
                    for (int q = 0; q < d; ++q) N *= ((v >> q) & 1) ? t[q] : 1.0 - t[q];
                    x += N * X[v * 3 + a];
                }
                c->node_xyz[a * m.n_nodes + g] = x;
            }
        }
    }
    c->h_prob.ti = 0;                    // both fields must be set again on the new geometry
    if (c->bound) {
        c->h_prob.mesh = m;
        s = upload_problem(c);
        if (s) return s;
    }
    c->have_field = false;
    return PIC_OK;
}

#include "pic_octree.inc"

extern "C" pic_status pic_mesh_info(pic_ctx *c, int32_t *dim, int64_t *n_cells, int64_t *n_nodes)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_mesh) return fail(c, PIC_ESTATE, "no mesh");
    if (dim) *dim = c->mesh.dim;
    if (n_cells) *n_cells = c->mesh.n_cells;
    if (n_nodes) *n_nodes = c->mesh.n_nodes;
    return PIC_OK;
}

extern "C" pic_status pic_q2_nodes(pic_ctx *c, double *xyz, uint8_t *is_hanging)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_mesh) return fail(c, PIC_ESTATE, "no mesh");
    if (xyz) std::memcpy(xyz, c->node_xyz.data(), c->node_xyz.size() * sizeof(double));
    if (is_hanging) {
        if (c->node_hanging.empty()) std::memset(is_hanging, 0, (size_t)c->mesh.n_nodes);
        else std::memcpy(is_hanging, c->node_hanging.data(), c->node_hanging.size());
    }
    return PIC_OK;
}

// ===========================================================================
// field
// ===========================================================================
namespace {
// Repack U (device [dim][n_nodes], prec) into the node-major arrays d64 / d32
// (allocated on first use), reject non-finite values, resolve hanging nodes.
pic_status load_field(pic_ctx *c, const void *U, int prec, void **d64, void **d32)
{
    if (!U) return fail(c, PIC_EINVAL, "null field");
    if (prec != PIC_F64 && prec != PIC_F32) return fail(c, PIC_EINVAL, "bad precision");
    hipSetDevice(c->device);
    const int d = c->mesh.dim;
    const int64_t nn = c->mesh.n_nodes;
    const size_t w = d == 3 ? 4 : 2;
    pic_status s;
    if (!*d64 && (s = dalloc(c, (double **)d64, w * (size_t)nn))) return s;
    if (!*d32 && (s = dalloc(c, (float **)d32, w * (size_t)nn))) return s;
    int *flag = nullptr;
    s = dalloc(c, &flag, 1);
    if (s) return s;
    HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
    unsigned grid = (unsigned)((nn + BLOCK - 1) / BLOCK);
    // first a pass that only checks the values, so that a rejected field
    // leaves the previous one in place
    auto pass = [&](int *f) {
        if (d == 3)
            hipLaunchKernelGGL(k_repack_field<3>, dim3(grid), dim3(BLOCK), 0, c->stream, U, prec == PIC_F32, nn, *d64, *d32, f);
        else
            hipLaunchKernelGGL(k_repack_field<2>, dim3(grid), dim3(BLOCK), 0, c->stream, U, prec == PIC_F32, nn, *d64, *d32, f);
    };
    pass(flag);
    int hflag = 0;
    HIPCHK(c, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipFree(flag);
    if (hflag) return fail(c, PIC_ENONFINITE, "velocity has NaN or infinite values");
    pass(nullptr);
    HIPCHK(c, hipGetLastError());
    if (c->mesh.kind == MESH_OCTREE) return resolve_hanging(c, *d64, *d32);
    return PIC_OK;
}

pic_status set_field_time(pic_ctx *c, double tau)
{
    if (!c->d_tau) {
        pic_status s = dalloc(c, &c->d_tau, 1);
        if (s) return s;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_tau, &tau, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

pic_status publish_fields(pic_ctx *c)
{
    c->h_prob.u64 = c->u64;
    c->h_prob.u32 = c->u32;
    c->h_prob.u1_64 = c->u1_64;
    c->h_prob.u1_32 = c->u1_32;
    c->h_prob.tau = c->d_tau;
    if (c->bound) return upload_problem(c);
    return PIC_OK;
}
}  // namespace

extern "C" pic_status pic_set_velocity(pic_ctx *c, const void *U, int prec)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_mesh) return fail(c, PIC_ESTATE, "no mesh");
    pic_status s = load_field(c, U, prec, &c->u64, &c->u32);
    if (s) return s;
    c->have_field = true;
    return publish_fields(c);
}

extern "C" pic_status pic_set_velocity_end(pic_ctx *c, const void *U1, int prec, double dt_u)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_field) return fail(c, PIC_ESTATE, "set the field at the start of the field step first");
    if (!U1) {
        c->h_prob.ti = 0;
        return publish_fields(c);
    }
    if (!(std::isfinite(dt_u) && dt_u > 0.0)) return fail(c, PIC_EINVAL, "dt_u must be finite and positive");
    pic_status s = load_field(c, U1, prec, &c->u1_64, &c->u1_32);
    if (s) return s;
    if ((s = set_field_time(c, 0.0))) return s;
    c->h_prob.ti = 1;
    c->h_prob.dt_u = dt_u;
    return publish_fields(c);
}

extern "C" pic_status pic_shift_velocity(pic_ctx *c, const void *U_next, int prec, double dt_u)
{
    if (!c) return PIC_EINVAL;
    if (!c->have_field || !c->h_prob.ti) return fail(c, PIC_ESTATE, "no field at the end of the field step");
    if (!(std::isfinite(dt_u) && dt_u > 0.0)) return fail(c, PIC_EINVAL, "dt_u must be finite and positive");
    if (!U_next) return fail(c, PIC_EINVAL, "null field");
    // the end field becomes the start field; U_next is loaded over the old start
    std::swap(c->u64, c->u1_64);
    std::swap(c->u32, c->u1_32);
    pic_status s = load_field(c, U_next, prec, &c->u1_64, &c->u1_32);
    if (s) {
        // keep a consistent pair: the previous end field is still the start field
        c->h_prob.ti = 0;
        publish_fields(c);
        return s;
    }
    if ((s = set_field_time(c, 0.0))) return s;
    c->h_prob.dt_u = dt_u;
    return publish_fields(c);
}

extern "C" pic_status pic_set_field_time(pic_ctx *c, double tau)
{
    if (!c) return PIC_EINVAL;
    if (!c->h_prob.ti) return fail(c, PIC_ESTATE, "no field at the end of the field step");
    if (!std::isfinite(tau)) return fail(c, PIC_EINVAL, "time must be finite");
    return set_field_time(c, tau);
}

extern "C" pic_status pic_field_time(pic_ctx *c, double *tau)
{
    if (!c || !tau) return PIC_EINVAL;
    if (!c->h_prob.ti) return fail(c, PIC_ESTATE, "no field at the end of the field step");
    HIPCHK(c, hipMemcpyAsync(tau, c->d_tau, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

// ===========================================================================
// store
// ===========================================================================
extern "C" pic_status pic_scratch_bytes(pic_ctx *c, int64_t capacity, int64_t *bytes)
{
    if (!c || !bytes) return PIC_EINVAL;
    if (!c->have_mesh) return fail(c, PIC_ESTATE, "no mesh");
    if (capacity < 0) return fail(c, PIC_EINVAL, "negative capacity");
    *bytes = (int64_t)scratch_layout(capacity, c->mesh.n_cells, nullptr, nullptr);
    return PIC_OK;
}

extern "C" pic_status pic_bind_store(pic_ctx *c, const pic_store *s)
{
    if (!c || !s) return PIC_EINVAL;
    if (!c->have_mesh) return fail(c, PIC_ESTATE, "no mesh");
    if (s->capacity < 1 || s->capacity >= (int64_t)INT32_MAX) return fail(c, PIC_EINVAL, "capacity out of range");
    if (s->n_prop < 0 || s->n_prop > 64) return fail(c, PIC_EINVAL, "n_prop out of range");
    if (s->prop_prec != PIC_F64 && s->prop_prec != PIC_F32) return fail(c, PIC_EINVAL, "bad prop precision");
    for (int b = 0; b < 2; ++b)
        if (!s->x[b] || !s->xr[b] || !s->cell[b] || !s->id[b] || !s->cell_start[b] || (s->n_prop && !s->prop[b]))
            return fail(c, PIC_EINVAL, "null store array in buffer %d", b);
    int64_t need = (int64_t)scratch_layout(s->capacity, c->mesh.n_cells, nullptr, nullptr);
    if (!s->scratch || s->scratch_bytes < need) return fail(c, PIC_EINVAL, "scratch too small: need %lld bytes", (long long)need);
    hipSetDevice(c->device);
    c->bound = false;                    // a new store starts in buffer A
    c->store = *s;
    scratch_layout(s->capacity, c->mesh.n_cells, (char *)s->scratch, &c->scr);
    ProblemDev &P = c->h_prob;
    const int ti = P.ti;                 // the field pair belongs to the mesh, not the store
    const double dt_u = P.dt_u;
    P = ProblemDev{};
    P.mesh = c->mesh;
    for (int b = 0; b < 2; ++b)
        P.store[b] = make_store((double *)s->x[b], (double *)s->xr[b], (int32_t *)s->cell[b], (uint32_t *)s->id[b],
                                s->prop[b], (int32_t *)s->cell_start[b]);
    P.cur = 0;
    P.n_prop = s->n_prop;
    P.prop_f64 = s->prop_prec == PIC_F64;
    P.cap = s->capacity;
    P.dt = 0.0;
    P.u64 = c->u64;
    P.u32 = c->u32;
    P.ti = ti;
    P.dt_u = dt_u;
    P.u1_64 = c->u1_64;
    P.u1_32 = c->u1_32;
    P.tau = c->d_tau;
    P.scr = c->scr;
    c->last_dt = 0.0;
    // zeroed state: empty buffers, zero counters
    const int64_t nc = c->mesh.n_cells;
    HIPCHK(c, hipMemsetAsync(s->cell_start[0], 0, sizeof(int32_t) * (nc + 1), c->stream));
    HIPCHK(c, hipMemsetAsync(s->cell_start[1], 0, sizeof(int32_t) * (nc + 1), c->stream));
    HIPCHK(c, hipMemsetAsync(s->scratch, 0, (size_t)need, c->stream));
    pic_status st = upload_problem(c);
    if (st) return st;
    c->bound = true;
    return build_work(c);
}

extern "C" pic_status pic_set_tile(pic_ctx *c, int32_t tile_cells)
{
    if (!c) return PIC_EINVAL;
    if (tile_cells < 1 || tile_cells > MAX_TILE) return fail(c, PIC_EINVAL, "tile must be in [1, %d]", MAX_TILE);
    c->tile = tile_cells;
    if (c->bound) return build_work(c);
    return PIC_OK;
}

extern "C" pic_status pic_current_buffer(pic_ctx *c, int32_t *which)
{
    if (!c || !which) return PIC_EINVAL;
    if (!c->bound) return fail(c, PIC_ESTATE, "no store bound");
    int v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, &c->d_prob->cur, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *which = v;
    return PIC_OK;
}

// ===========================================================================
// generation
// ===========================================================================
namespace {
template <int D>
pic_status seed_ref_launch(pic_ctx *c, const double *xr, const uint32_t *ids, int64_t n, int pi, const void *pin,
                           uint64_t seed, uint32_t first_id)
{
    unsigned grid = (unsigned)((c->mesh.n_cells + BLOCK / 64 - 1) / (BLOCK / 64));
    switch (c->mesh.kind) {
    case MESH_UNIFORM:
        LAUNCH(c, "seed", (k_seed_reference<D, MESH_UNIFORM>), grid, BLOCK, c->d_prob, 0, xr, ids, n, pi, pin, seed,
               first_id);
        break;
    case MESH_DISPLACED:
        LAUNCH(c, "seed", (k_seed_reference<D, MESH_DISPLACED>), grid, BLOCK, c->d_prob, 0, xr, ids, n, pi, pin, seed,
               first_id);
        break;
    default:
        if constexpr (D == 3)
            LAUNCH(c, "seed", (k_seed_reference<D, MESH_OCTREE>), grid, BLOCK, c->d_prob, 0, xr, ids, n, pi, pin, seed,
                   first_id);
    }
    return PIC_OK;
}
template <int D>
pic_status seed_pos_launch(pic_ctx *c, const double *x, const uint32_t *ids, int64_t n, int pi, const void *pin)
{
    unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
    switch (c->mesh.kind) {
    case MESH_UNIFORM:
        LAUNCH(c, "seed_positions", (k_seed_positions<D, MESH_UNIFORM>), grid, BLOCK, c->d_prob, 0, x, ids, n, pi, pin);
        break;
    case MESH_DISPLACED:
        LAUNCH(c, "seed_positions", (k_seed_positions<D, MESH_DISPLACED>), grid, BLOCK, c->d_prob, 0, x, ids, n, pi, pin);
        break;
    default:
        if constexpr (D == 3)
            LAUNCH(c, "seed_positions", (k_seed_positions<D, MESH_OCTREE>), grid, BLOCK, c->d_prob, 0, x, ids, n, pi, pin);
    }
    return PIC_OK;
}
}  // namespace

namespace {
// Reference-local generation into the current buffer: counts per cell
// (device), cell_start = their exclusive scan.  xr == NULL: reference points
// from the counter hash with ids first_id + position (n = -1: the sum of the
// counts); else xr / ids as given for n particles.
pic_status seed_cells(pic_ctx *c, const int32_t *counts, const double *xr, const uint32_t *ids, int64_t n,
                      int32_t prop_init, const void *prop_in, uint64_t seed, uint32_t first_id)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (!counts || (xr && n > 0 && !ids)) return fail(c, PIC_EINVAL, "null argument");
    if (prop_init != PIC_PROP_GIVEN && prop_init != PIC_PROP_INITIAL_POSITION) return fail(c, PIC_EINVAL, "bad prop_init");
    hipSetDevice(c->device);
    // cell_start of the current buffer = exclusive scan of counts; check the total
    std::vector<int32_t> h(c->mesh.n_cells);
    HIPCHK(c, hipMemcpyAsync(h.data(), counts, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> cs(h.size() + 1, 0);
    int64_t run = 0;
    for (size_t k = 0; k < h.size(); ++k) {
        if (h[k] < 0) return fail(c, PIC_EINVAL, "negative count");
        cs[k] = (int32_t)run;
        run += h[k];
    }
    cs[h.size()] = (int32_t)run;
    if (!xr) n = run;
    if (n < 0 || n > c->store.capacity) return fail(c, PIC_ECAPACITY, "n=%lld exceeds capacity %lld", (long long)n, (long long)c->store.capacity);
    if (run != n) return fail(c, PIC_EINVAL, "sum of counts %lld != n %lld", (long long)run, (long long)n);
    if (!xr && (uint64_t)first_id + (uint64_t)n > 0x100000000ull) return fail(c, PIC_EINVAL, "ids beyond 2^32");
    if (prop_init == PIC_PROP_GIVEN && c->store.n_prop > 0 && n > 0 && !prop_in) return fail(c, PIC_EINVAL, "null prop_in");
    int32_t cur = 0;
    if ((s = pic_current_buffer(c, &cur))) return s;
    HIPCHK(c, hipMemcpyAsync(c->store.cell_start[cur], cs.data(), sizeof(int32_t) * cs.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->scr.next_id, 0, 8 * (1 + STAT_STRIPES), c->stream));
    s = c->mesh.dim == 2 ? seed_ref_launch<2>(c, xr, ids, n, prop_init, prop_in, seed, first_id)
                         : seed_ref_launch<3>(c, xr, ids, n, prop_init, prop_in, seed, first_id);
    if (s) return s;
    LAUNCH(c, "seed", k_reduce_next_id, 1u, (unsigned)STAT_STRIPES, (const ProblemDev *)c->d_prob);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}
}  // namespace

extern "C" pic_status pic_seed_reference(pic_ctx *c, const int32_t *counts, const double *xr, const uint32_t *ids, int64_t n,
                                         int32_t prop_init, const void *prop_in)
{
    if (c && n > 0 && !xr) return fail(c, PIC_EINVAL, "null argument");
    static const double none = 0.0;     // marks "given" for an empty input (never read)
    return seed_cells(c, counts, n > 0 ? xr : &none, ids, n, prop_init, prop_in, 0, 0);
}

extern "C" pic_status pic_seed_per_cell(pic_ctx *c, const int32_t *counts, uint64_t seed, uint32_t first_id,
                                        int32_t prop_init, const void *prop_in)
{
    return seed_cells(c, counts, nullptr, nullptr, -1, prop_init, prop_in, seed, first_id);
}

extern "C" pic_status pic_seed_positions(pic_ctx *c, const double *x, const uint32_t *ids, int64_t n, int32_t prop_init,
                                         const void *prop_in)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (n < 0 || n > c->store.capacity) return fail(c, PIC_ECAPACITY, "n exceeds capacity");
    if (n > 0 && (!x || !ids)) return fail(c, PIC_EINVAL, "null argument");
    if (prop_init == PIC_PROP_GIVEN && c->store.n_prop > 0 && n > 0 && !prop_in) return fail(c, PIC_EINVAL, "null prop_in");
    hipSetDevice(c->device);
    int32_t cur = 0;
    if ((s = pic_current_buffer(c, &cur))) return s;
    const int64_t nc = c->mesh.n_cells;
    // every point is an "arrival": no stayers; live count of the unsorted input = n
    HIPCHK(c, hipMemsetAsync(c->scr.n_stay, 0, sizeof(int32_t) * nc, c->stream));
    HIPCHK(c, hipMemsetAsync(c->scr.n_arrive, 0, sizeof(int32_t) * nc, c->stream));
    HIPCHK(c, hipMemsetAsync(c->scr.cursor, 0, sizeof(int32_t) * (nc + 1), c->stream));
    HIPCHK(c, hipMemsetAsync(c->scr.next_id, 0, 8 * (1 + STAT_STRIPES), c->stream));
    int32_t n32 = (int32_t)n;
    HIPCHK(c, hipMemcpyAsync(c->store.cell_start[cur] + nc, &n32, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    s = c->mesh.dim == 2 ? seed_pos_launch<2>(c, x, ids, n, prop_init, prop_in) : seed_pos_launch<3>(c, x, ids, n, prop_init, prop_in);
    if (s) return s;
    LAUNCH(c, "seed_positions", k_reduce_next_id, 1u, (unsigned)STAT_STRIPES, (const ProblemDev *)c->d_prob);
    s = enqueue_sort(c, c->d_prob, 0, true);
    if (s) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

namespace {
template <int D>
pic_status transfer_launch(pic_ctx *c, const ProblemDev *src, int64_t n)
{
    const unsigned grid = (unsigned)std::max<int64_t>(1, (n + BLOCK - 1) / BLOCK);
    switch (c->mesh.kind) {
    case MESH_UNIFORM: LAUNCH(c, "transfer", (k_transfer_in<D, MESH_UNIFORM>), grid, BLOCK, src, c->d_prob, 0, n); break;
    case MESH_DISPLACED: LAUNCH(c, "transfer", (k_transfer_in<D, MESH_DISPLACED>), grid, BLOCK, src, c->d_prob, 0, n); break;
    default:
        if constexpr (D == 3) LAUNCH(c, "transfer", (k_transfer_in<3, MESH_OCTREE>), grid, BLOCK, src, c->d_prob, 0, n);
    }
    return PIC_OK;
}
}  // namespace

extern "C" pic_status pic_transfer(pic_ctx *from, pic_ctx *to)
{
    if (!from || !to || from == to) return PIC_EINVAL;
    pic_status s = require_ready(to, false);
    if (s) return s;
    if ((s = require_ready(from, false))) return fail(to, s, "source: %s", from->err.c_str());
    if (from->device != to->device) return fail(to, PIC_EINVAL, "both problems must be on one device");
    if (from->mesh.dim != to->mesh.dim) return fail(to, PIC_EINVAL, "dimensions differ");
    if (from->store.n_prop != to->store.n_prop || (from->store.n_prop && from->store.prop_prec != to->store.prop_prec))
        return fail(to, PIC_EINVAL, "property count or precision differs");
    for (int a = 0; a < to->mesh.dim; ++a)
        if (from->mesh.lo[a] != to->mesh.lo[a] || from->mesh.hi[a] != to->mesh.hi[a])
            return fail(to, PIC_EINVAL, "the two meshes cover different boxes");
    hipSetDevice(to->device);
    // the source's pending work, then its live count
    HIPCHK(to, hipStreamSynchronize(from->stream));
    int32_t scur = 0, n32 = 0;
    if ((s = pic_current_buffer(from, &scur))) return fail(to, s, "source: %s", from->err.c_str());
    HIPCHK(to, hipMemcpy(&n32, from->store.cell_start[scur] + from->mesh.n_cells, sizeof(int32_t), hipMemcpyDeviceToHost));
    const int64_t n = n32;
    if (n > to->store.capacity) return fail(to, PIC_ECAPACITY, "%lld particles exceed capacity %lld", (long long)n, (long long)to->store.capacity);
    int32_t cur = 0;
    if ((s = pic_current_buffer(to, &cur))) return s;
    const int64_t nc = to->mesh.n_cells;
    HIPCHK(to, hipMemsetAsync(to->scr.n_stay, 0, sizeof(int32_t) * nc, to->stream));
    HIPCHK(to, hipMemsetAsync(to->scr.n_arrive, 0, sizeof(int32_t) * nc, to->stream));
    HIPCHK(to, hipMemsetAsync(to->scr.cursor, 0, sizeof(int32_t) * (nc + 1), to->stream));
    HIPCHK(to, hipMemsetAsync(to->scr.next_id, 0, 8 * (1 + STAT_STRIPES), to->stream));
    HIPCHK(to, hipMemcpyAsync(to->store.cell_start[cur] + nc, &n32, sizeof(int32_t), hipMemcpyHostToDevice, to->stream));
    s = to->mesh.dim == 2 ? transfer_launch<2>(to, from->d_prob, n) : transfer_launch<3>(to, from->d_prob, n);
    if (s) return s;
    LAUNCH(to, "transfer", k_reduce_next_id, 1u, (unsigned)STAT_STRIPES, (const ProblemDev *)to->d_prob);
    if ((s = enqueue_sort(to, to->d_prob, 0, true))) return s;
    HIPCHK(to, hipStreamSynchronize(to->stream));
    return PIC_OK;
}

// ===========================================================================
// advance
// ===========================================================================
extern "C" pic_status pic_set_property_odes(pic_ctx *c, int32_t damage_prop, int32_t deform_prop, double alpha,
                                            double beta)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (damage_prop < 0 && deform_prop < 0) {
        c->h_prob.odes = 0;
        return upload_problem(c);
    }
    const int d = c->mesh.dim, np = c->store.n_prop;
    if (c->store.prop_prec != PIC_F64) return fail(c, PIC_EINVAL, "property equations need double-precision properties");
    if (damage_prop < 0 || deform_prop < 0 || damage_prop >= np || deform_prop + d * d > np)
        return fail(c, PIC_EINVAL, "damage_prop and deform_prop .. deform_prop + dim^2 - 1 must be properties");
    if (damage_prop >= deform_prop && damage_prop < deform_prop + d * d)
        return fail(c, PIC_EINVAL, "the damage property lies inside the deformation gradient");
    if (!(std::isfinite(alpha) && std::isfinite(beta))) return fail(c, PIC_EINVAL, "alpha and beta must be finite");
    c->h_prob.odes = 1;
    c->h_prob.ode_dmg = damage_prop;
    c->h_prob.ode_F = deform_prop;
    c->h_prob.ode_alpha = alpha;
    c->h_prob.ode_beta = beta;
    return upload_problem(c);
}

namespace {
// The fused step sequence from its captured graph (captured at the first call
// with a new key), ordered after the caller's earlier work and before its
// later work by one event on each stream.
pic_status advance_graph(pic_ctx *c, int scheme, int prec, int n)
{
    if (!c->gstream) {
        HIPCHK(c, hipStreamCreate(&c->gstream));
        for (hipEvent_t &e : c->g_ev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    const int key[5] = {n, scheme, prec, c->h_prob.odes ? 1 : 0, c->h_prob.ti ? 1 : 0};
    if (!c->g_exec || !std::equal(key, key + 5, c->g_key)) {
        drop_adv_graph(c);
        HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        hipStream_t caller = c->stream;
        c->stream = c->gstream;
        pic_status s = enqueue_steps_fused(c, c->d_prob, scheme, prec, n);
        c->stream = caller;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->gstream, &g);
        if (s || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return s ? s : fail(c, PIC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        }
        c->g_graph = g;
        HIPCHK(c, hipGraphInstantiate(&c->g_exec, g, nullptr, nullptr, 0));
        std::copy(key, key + 5, c->g_key);
    }
    HIPCHK(c, hipEventRecord(c->g_ev[0], c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->gstream, c->g_ev[0], 0));
    HIPCHK(c, hipGraphLaunch(c->g_exec, c->gstream));
    HIPCHK(c, hipEventRecord(c->g_ev[1], c->gstream));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->g_ev[1], 0));
    return PIC_OK;
}
}  // namespace

extern "C" pic_status pic_set_launch_graphs(pic_ctx *c, int32_t enable)
{
    if (!c) return PIC_EINVAL;
    c->graphs = enable != 0;
    if (!c->graphs) drop_adv_graph(c);
    return PIC_OK;
}

extern "C" pic_status pic_advance(pic_ctx *c, double dt, int32_t n_steps, int32_t scheme, int32_t eval_prec)
{
    pic_status s = require_ready(c, true);
    if (s) return s;
    if (!(std::isfinite(dt)) || dt < 0.0) return fail(c, PIC_EINVAL, "dt must be finite and >= 0");
    if (n_steps < 0) return fail(c, PIC_EINVAL, "n_steps < 0");
    if (scheme != PIC_EULER && scheme != PIC_RK2 && scheme != PIC_RK4) return fail(c, PIC_EINVAL, "bad scheme");
    if (eval_prec != PIC_F64 && eval_prec != PIC_F32) return fail(c, PIC_EINVAL, "bad eval precision");
    if (c->mesh.kind == MESH_OCTREE && c->mesh.dim != 3) return fail(c, PIC_EINVAL, "octree is 3D");
    hipSetDevice(c->device);
    if ((s = set_dt(c, dt))) return s;
    if (PIC_FUSE_STEPS && PIC_USE_BLOCK_ADVECT && n_steps > 1 && c->mesh.kind == MESH_UNIFORM && c->n_blk[eval_prec == PIC_F32]) {
        if (c->graphs && !c->profile) return advance_graph(c, scheme, eval_prec, n_steps);
        return enqueue_steps_fused(c, c->d_prob, scheme, eval_prec, n_steps);
    }
    for (int k = 0; k < n_steps; ++k)
        if ((s = enqueue_step(c, c->d_prob, scheme, eval_prec))) return s;
    return PIC_OK;
}

// ===========================================================================
// population management
// ===========================================================================
extern "C" pic_status pic_population(pic_ctx *c, int32_t min_pc, int32_t max_pc, uint64_t seed, uint64_t step)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (min_pc < 0 || max_pc < 1 || min_pc > max_pc) return fail(c, PIC_EINVAL, "need 0 <= min <= max, max >= 1");
    hipSetDevice(c->device);
    // total after the clamp must fit: computed exactly by the scan, checked here
    if (c->h_prob.pop_min != min_pc || c->h_prob.pop_max != max_pc) {
        c->h_prob.pop_min = min_pc;
        c->h_prob.pop_max = max_pc;
        int32_t mm[2] = {min_pc, max_pc};
        HIPCHK(c, hipMemcpyAsync(&c->d_prob->pop_min, mm, sizeof(mm), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if ((s = enqueue_scan(c, c->d_prob, 1))) return s;
    // capacity check needs the total: read it (population is not a graph-captured call)
    int32_t cur = 0;
    if ((s = pic_current_buffer(c, &cur))) return s;
    int32_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, c->store.cell_start[1 - cur] + c->mesh.n_cells, sizeof(int32_t), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if ((int64_t)total > c->store.capacity) return fail(c, PIC_ECAPACITY, "population needs capacity %d", total);
    unsigned grid = (unsigned)((c->mesh.n_cells + BLOCK / 64 - 1) / (BLOCK / 64));
    switch (c->mesh.kind) {
    case MESH_UNIFORM:
        if (c->mesh.dim == 2) LAUNCH(c, "population", (k_population<2, MESH_UNIFORM>), grid, BLOCK, (const ProblemDev *)c->d_prob, 0, seed, step);
        else LAUNCH(c, "population", (k_population<3, MESH_UNIFORM>), grid, BLOCK, (const ProblemDev *)c->d_prob, 0, seed, step);
        break;
    case MESH_DISPLACED:
        if (c->mesh.dim == 2) LAUNCH(c, "population", (k_population<2, MESH_DISPLACED>), grid, BLOCK, (const ProblemDev *)c->d_prob, 0, seed, step);
        else LAUNCH(c, "population", (k_population<3, MESH_DISPLACED>), grid, BLOCK, (const ProblemDev *)c->d_prob, 0, seed, step);
        break;
    default:
        LAUNCH(c, "population", (k_population<3, MESH_OCTREE>), grid, BLOCK, (const ProblemDev *)c->d_prob, 0, seed, step);
    }
    LAUNCH(c, "population_finish", k_population_finish, 1u, 1u, c->d_prob, 0);
    return PIC_OK;
}

// ===========================================================================
// interpolation
// ===========================================================================
extern "C" pic_status pic_interpolate(pic_ctx *c, int32_t kind, double *out, double *aux, int32_t *count)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (!out || !count) return fail(c, PIC_EINVAL, "null output");
    hipSetDevice(c->device);
    unsigned grid = (unsigned)((c->mesh.n_cells + BLOCK / 64 - 1) / (BLOCK / 64));
    if (kind == PIC_INTERP_CELL_AVERAGE || kind == PIC_INTERP_GEOMETRIC_AVERAGE || kind == PIC_INTERP_HARMONIC_AVERAGE) {
        const int mode = kind == PIC_INTERP_CELL_AVERAGE ? 0 : (kind == PIC_INTERP_GEOMETRIC_AVERAGE ? 1 : 2);
        LAUNCH(c, "interp_average", k_interp_average, grid, BLOCK, (const ProblemDev *)c->d_prob, 0, out, count, mode);
    } else if (kind == PIC_INTERP_LINEAR_LS) {
        if (!aux) return fail(c, PIC_EINVAL, "linear least squares needs aux (xbar)");
        if (c->mesh.dim == 2) LAUNCH(c, "interp_lls", k_interp_lls<2>, grid, BLOCK, (const ProblemDev *)c->d_prob, 0, out, aux, count);
        else LAUNCH(c, "interp_lls", k_interp_lls<3>, grid, BLOCK, (const ProblemDev *)c->d_prob, 0, out, aux, count);
    } else {
        return fail(c, PIC_EINVAL, "unknown interpolation kind %d", kind);
    }
    return PIC_OK;
}

namespace {
template <int D>
pic_status interp_points_launch(pic_ctx *c, int kind, const EvalPoints &qp, double *out, int32_t *count)
{
    unsigned grid = (unsigned)((c->mesh.n_cells + BLOCK / 64 - 1) / (BLOCK / 64));
    const ProblemDev *dp = c->d_prob;
    switch (c->mesh.kind) {
    case MESH_UNIFORM: LAUNCH(c, "interp_points", (k_interp_points<D, MESH_UNIFORM>), grid, BLOCK, dp, 0, kind, qp, out, count); break;
    case MESH_DISPLACED: LAUNCH(c, "interp_points", (k_interp_points<D, MESH_DISPLACED>), grid, BLOCK, dp, 0, kind, qp, out, count); break;
    default:
        if constexpr (D == 3) LAUNCH(c, "interp_points", (k_interp_points<3, MESH_OCTREE>), grid, BLOCK, dp, 0, kind, qp, out, count);
    }
    return PIC_OK;
}
}  // namespace

extern "C" pic_status pic_interpolate_points(pic_ctx *c, int32_t kind, const double *qhat, int32_t n_q, double *out,
                                             int32_t *count)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (kind != PIC_INTERP_NEAREST && kind != PIC_INTERP_INV_DISTANCE && kind != PIC_INTERP_SHAPE_WEIGHTED)
        return fail(c, PIC_EINVAL, "unknown point interpolation kind %d", kind);
    if (n_q < 1 || n_q > MAX_EVAL_POINTS) return fail(c, PIC_EINVAL, "n_q must be in [1, %d]", MAX_EVAL_POINTS);
    if (!qhat || !out) return fail(c, PIC_EINVAL, "null argument");
    const int d = c->mesh.dim;
    EvalPoints qp{};
    qp.n = n_q;
    for (int a = 0; a < d; ++a)
        for (int q = 0; q < n_q; ++q) {
            const double v = qhat[a * n_q + q];
            if (!(v >= 0.0 && v <= 1.0)) return fail(c, PIC_EINVAL, "evaluation points must lie in the reference cell");
            qp.q[a][q] = v;
        }
    hipSetDevice(c->device);
    const int k = kind - PIC_INTERP_NEAREST;
    return d == 2 ? interp_points_launch<2>(c, k, qp, out, count) : interp_points_launch<3>(c, k, qp, out, count);
}

// ===========================================================================
// Metropolis-Hastings generation
// ===========================================================================
namespace {
// Pack the density into the node-vector layout R (flag: zeroed by the
// caller, set for a non-finite value), then run the chains; synchronises.
template <int D>
pic_status seed_mh_kernels(pic_ctx *c, const double *rho, int J, uint64_t seed, uint32_t first_id,
                           typename NodeVec<D, double>::type *R, int *flag, unsigned long long *d_longest)
{
    const int64_t nn = c->mesh.n_nodes;
    hipLaunchKernelGGL(k_pack_density<D>, dim3((unsigned)((nn + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, c->stream, rho, nn, R, flag);
    int hflag = 0;
    if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, PIC_EDEVICE, "density copy");
    if (hflag) return fail(c, PIC_ENONFINITE, "density has NaN or infinite values");
    const unsigned grid = (unsigned)((c->mesh.n_cells + BLOCK - 1) / BLOCK);
    ProblemDev *dp = c->d_prob;
    switch (c->mesh.kind) {
    case MESH_UNIFORM: hipLaunchKernelGGL((k_seed_mh<D, MESH_UNIFORM>), dim3(grid), dim3(BLOCK), 0, c->stream, dp, 0, R, J, seed, first_id, d_longest); break;
    case MESH_DISPLACED: hipLaunchKernelGGL((k_seed_mh<D, MESH_DISPLACED>), dim3(grid), dim3(BLOCK), 0, c->stream, dp, 0, R, J, seed, first_id, d_longest); break;
    default:
        if constexpr (D == 3) hipLaunchKernelGGL((k_seed_mh<3, MESH_OCTREE>), dim3(grid), dim3(BLOCK), 0, c->stream, dp, 0, R, J, seed, first_id, d_longest);
    }
    if (hipGetLastError() != hipSuccess) return fail(c, PIC_EDEVICE, "seed_mh launch");
    return PIC_OK;
}

template <int D>
pic_status seed_mh_launch(pic_ctx *c, const double *rho, int J, uint64_t seed, uint32_t first_id,
                          unsigned long long *d_longest)
{
    using V = typename NodeVec<D, double>::type;
    const int64_t nn = c->mesh.n_nodes;
    V *R = nullptr;
    int *flag = nullptr;
    pic_status s;
    if ((s = dalloc(c, &R, (size_t)nn))) return s;
    if ((s = dalloc(c, &flag, 1))) {
        hipFree(R);
        return s;
    }
    if (hipMemsetAsync(flag, 0, sizeof(int), c->stream) != hipSuccess) s = fail(c, PIC_EDEVICE, "memset");
    if (!s) s = seed_mh_kernels<D>(c, rho, J, seed, first_id, R, flag, d_longest);
    hipStreamSynchronize(c->stream);
    hipFree(R);
    hipFree(flag);
    return s;
}
}  // namespace

extern "C" pic_status pic_seed_mh(pic_ctx *c, const int32_t *counts, const double *rho, int32_t J, uint64_t seed,
                                  uint32_t first_id, int64_t *longest_run)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (!counts || !rho) return fail(c, PIC_EINVAL, "null argument");
    if (J < 1) return fail(c, PIC_EINVAL, "J must be at least 1");
    hipSetDevice(c->device);
    std::vector<int32_t> h(c->mesh.n_cells);
    HIPCHK(c, hipMemcpyAsync(h.data(), counts, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> cs(h.size() + 1, 0);
    int64_t run = 0;
    for (size_t k = 0; k < h.size(); ++k) {
        if (h[k] < 0) return fail(c, PIC_EINVAL, "negative count");
        cs[k] = (int32_t)run;
        run += h[k];
    }
    cs[h.size()] = (int32_t)run;
    if (run > c->store.capacity) return fail(c, PIC_ECAPACITY, "%lld particles exceed capacity %lld", (long long)run, (long long)c->store.capacity);
    if ((uint64_t)first_id + (uint64_t)run > 0xFFFFFFFFull) return fail(c, PIC_EINVAL, "ids would overflow 32 bits");
    int32_t cur = 0;
    if ((s = pic_current_buffer(c, &cur))) return s;
    HIPCHK(c, hipMemcpyAsync(c->store.cell_start[cur], cs.data(), sizeof(int32_t) * cs.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->scr.next_id, 0, 8 * (1 + STAT_STRIPES), c->stream));
    unsigned long long *d_longest = nullptr;
    if ((s = dalloc(c, &d_longest, 1))) return s;
    HIPCHK(c, hipMemsetAsync(d_longest, 0, sizeof(unsigned long long), c->stream));
    s = c->mesh.dim == 2 ? seed_mh_launch<2>(c, rho, J, seed, first_id, d_longest) : seed_mh_launch<3>(c, rho, J, seed, first_id, d_longest);
    if (!s) {
        LAUNCH(c, "seed", k_reduce_next_id, 1u, (unsigned)STAT_STRIPES, (const ProblemDev *)c->d_prob);
        unsigned long long hl = 0;
        if (hipMemcpyAsync(&hl, d_longest, sizeof(hl), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            s = fail(c, PIC_EDEVICE, "copy of the longest run");
        if (!s && longest_run) *longest_run = (int64_t)hl;
    }
    hipFree(d_longest);
    return s;
}

extern "C" pic_status pic_seed_mh_static(pic_ctx *c, const int32_t *counts, const double *rho, int32_t J, uint64_t seed,
                                         uint32_t first_id, int64_t *longest_run)
{
    pic_status s = require_ready(c, false);
    if (s) return s;
    if (!counts || !rho) return fail(c, PIC_EINVAL, "null argument");
    if (J < 1) return fail(c, PIC_EINVAL, "J must be at least 1");
    if (c->device >= STATIC_MAX_DEVICES || !g_scratch_ptr[c->device])
        return fail(c, PIC_EDEVICE, "no address of the static scratch on device %d: %s", c->device,
                    c->device < STATIC_MAX_DEVICES ? hipGetErrorString(g_scratch_err[c->device]) : "device index too large");
    hipSetDevice(c->device);
    const int64_t nc = c->mesh.n_cells, nn = c->mesh.n_nodes;
    const size_t vbytes = c->mesh.dim == 3 ? sizeof(double4) : sizeof(double2);
    const size_t cs_off = 256, r_off = cs_off + align256(sizeof(int32_t) * (size_t)(nc + 1));
    const size_t need = r_off + vbytes * (size_t)nn;
    if (need > STATIC_SCRATCH_BYTES)
        return fail(c, PIC_EINVAL, "the mesh (%lld cells, %lld nodes) needs %zu bytes of scratch; the static scratch holds %zu",
                    (long long)nc, (long long)nn, need, STATIC_SCRATCH_BYTES);
    unsigned char *base = (unsigned char *)g_scratch_ptr[c->device];
    int32_t *flags = (int32_t *)base;                       // [0] non-finite density, [1] negative count
    auto *d_longest = (unsigned long long *)(base + 8);
    auto *d_total = (int64_t *)(base + 16);
    auto *d_cs = (int32_t *)(base + cs_off);
    // cell starts = exclusive scan of the counts, built in the scratch and
    // copied to the store only once the counts are known to fit
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, c->stream, base, (int64_t)24);
    hipLaunchKernelGGL(k_counts_scan, dim3(1), dim3(BLOCK), 0, c->stream, counts, nc, d_cs, d_total, flags + 1);
    struct {
        int32_t flag[2];
        unsigned long long longest;
        int64_t total;
    } h{};
    static_assert(sizeof(h) == 24, "header layout");
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&h, base, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h.flag[1]) return fail(c, PIC_EINVAL, "negative count");
    if (h.total > c->store.capacity)
        return fail(c, PIC_ECAPACITY, "%lld particles exceed capacity %lld", (long long)h.total, (long long)c->store.capacity);
    if ((uint64_t)first_id + (uint64_t)h.total > 0xFFFFFFFFull) return fail(c, PIC_EINVAL, "ids would overflow 32 bits");
    int32_t cur = 0;
    if ((s = pic_current_buffer(c, &cur))) return s;
    HIPCHK(c, hipMemcpyAsync(c->store.cell_start[cur], d_cs, sizeof(int32_t) * (size_t)(nc + 1), hipMemcpyDeviceToDevice,
                             c->stream));
    const int64_t nid = 8 * (1 + STAT_STRIPES);
    hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)((nid + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, c->stream,
                       (unsigned char *)c->scr.next_id, nid);
    s = c->mesh.dim == 2 ? seed_mh_kernels<2>(c, rho, J, seed, first_id, (double2 *)(base + r_off), flags, d_longest)
                         : seed_mh_kernels<3>(c, rho, J, seed, first_id, (double4 *)(base + r_off), flags, d_longest);
    if (s) return s;
    hipLaunchKernelGGL(k_reduce_next_id, dim3(1), dim3(STAT_STRIPES), 0, c->stream, (const ProblemDev *)c->d_prob);
    unsigned long long hl = 0;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&hl, d_longest, sizeof(hl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (longest_run) *longest_run = (int64_t)hl;
    return PIC_OK;
}

// ===========================================================================
// statistics and profiling
// ===========================================================================
extern "C" pic_status pic_stats_read(pic_ctx *c, pic_stats *out)
{
    if (!c || !out) return PIC_EINVAL;
    if (!c->bound) return fail(c, PIC_ESTATE, "no store bound");
    hipSetDevice(c->device);
    std::vector<unsigned long long> stripes((size_t)ST_COUNT * STAT_STRIPES);
    HIPCHK(c, hipMemcpyAsync(stripes.data(), c->scr.stats, stripes.size() * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, c->stream));
    int32_t cur = 0;
    pic_status s = pic_current_buffer(c, &cur);
    if (s) return s;
    int32_t live = 0;
    HIPCHK(c, hipMemcpyAsync(&live, c->store.cell_start[cur] + c->mesh.n_cells, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unsigned long long st[ST_COUNT] = {0};
    for (int q = 0; q < STAT_STRIPES; ++q)
        for (int k = 0; k < ST_COUNT; ++k) st[k] += stripes[(size_t)q * ST_COUNT + k];
    out->live = live;
    out->lost = (int64_t)st[ST_LOST];
    out->moved = (int64_t)st[ST_MOVED];
    out->near_face = (int64_t)st[ST_NEAR];
    out->first_try = (int64_t)st[ST_FIRST_TRY];
    out->fallback = (int64_t)st[ST_FALLBACK];
    out->newton_fail = (int64_t)st[ST_NEWTON_FAIL];
    out->added = (int64_t)st[ST_ADDED];
    out->deleted = (int64_t)st[ST_DELETED];
    out->steps = (int64_t)st[ST_STEPS];
    out->particle_steps = (int64_t)st[ST_PSTEPS];
    out->searches = (int64_t)st[ST_SEARCHES];
    out->searched = (int64_t)st[ST_SEARCHED];
    return PIC_OK;
}

extern "C" pic_status pic_stats_reset(pic_ctx *c)
{
    if (!c) return PIC_EINVAL;
    if (!c->bound) return fail(c, PIC_ESTATE, "no store bound");
    hipSetDevice(c->device);
    HIPCHK(c, hipMemsetAsync(c->scr.stats, 0, sizeof(unsigned long long) * ST_COUNT * STAT_STRIPES, c->stream));
    return PIC_OK;
}

extern "C" pic_status pic_profile_enable(pic_ctx *c, int32_t enable)
{
    if (!c) return PIC_EINVAL;
    pic_status s = collect_profile(c);
    if (s) return s;
    c->profile = enable != 0;
    if (enable) c->prof.clear();
    return PIC_OK;
}

extern "C" pic_status pic_profile_read(pic_ctx *c, const char *kernel, double *total_ms, int64_t *launches)
{
    if (!c || !kernel) return PIC_EINVAL;
    pic_status s = collect_profile(c);
    if (s) return s;
    auto it = c->prof.find(kernel);
    if (it == c->prof.end()) {
        if (total_ms) *total_ms = 0.0;
        if (launches) *launches = 0;
        static const char *known[] = {"advect", "scan_reduce", "scan_down", "place", "fix", "gather", "flip",
                                      "seed", "seed_positions", "population", "population_finish", "interp_average",
                                      "interp_lls", "interp_points", "transfer", "adjoint_step", "adjoint_save", "batch_advect",
                                      "gather_advect"};
        for (const char *k : known)
            if (!std::strcmp(k, kernel)) return PIC_OK;
        return fail(c, PIC_EINVAL, "unknown kernel name %s", kernel);
    }
    if (total_ms) *total_ms = it->second.first;
    if (launches) *launches = it->second.second;
    return PIC_OK;
}

#include "pic_adjoint_api.inc"
#include "pic_batch.inc"

// HIP kernels of the particle hot path for gfx950.
//
// One time step = advect (per tile of cells) -> scan of per-cell counts ->
// place (destination of every particle) -> fix (arrival order) -> gather
// (permute the store into the other buffer).
#include "pic_common.h"
#include "pic_internal.h"
#include "pic_advect.h"

namespace pic {

// ===========================================================================
// scan of the new per-cell counts (two phases over chunks of cells)
// ===========================================================================

// int64 workgroup exclusive scan; returns the prefix, sets total.
__device__ __forceinline__ int64_t block_scan_i64(int64_t v, int64_t *s_tmp, int64_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t n = __shfl_up(inc, o, 64);
        if (lane >= o) inc += n;
    }
    if (lane == 63) s_tmp[wid] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        int64_t c = s_tmp[w];
        off += (w < wid) ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// Count of a cell after the step from the two words loaded for it: stayers +
// arrivals (MODE 0: x = n_stay[K], y = n_arrive[K]), or the population clamp
// (MODE 1: x = cs[K], y = cs[K + 1] of the current buffer; packed as
// count | additions << 32).  The words of all of a thread's cells are loaded
// before the first is used, so that the loads are in flight together.
template <int MODE> struct CellWords {
    const int32_t PIC_G *x, *y;
    int pop_min, pop_max;
    __device__ __forceinline__ explicit CellWords(const ProblemDev &P)
    {
        if (MODE == 0) {
            x = P.scr.n_stay;
            y = P.scr.n_arrive;
        } else {
            x = P.store[P.cur].cs;
            y = x + 1;
        }
        pop_min = P.pop_min;
        pop_max = P.pop_max;
    }
    __device__ __forceinline__ int64_t value(int32_t a, int32_t b) const
    {
        if (MODE == 0) return (int64_t)a + (int64_t)b;
        const int64_t n = (int64_t)b - a;
        const int64_t keep = n > pop_max ? pop_max : n;
        const int64_t add = keep < pop_min ? pop_min - keep : 0;
        return (keep + add) | (add << 32);
    }
};

// Flip the current buffer of a problem; a counted step also advances the time
// since t^n of a field that changes in time.
__device__ __forceinline__ void flip_problem(ProblemDev &P, int count_step)
{
    P.cur = 1 - P.cur;
    if (count_step) {
        atomicAdd(&P.scr.stats[ST_STEPS], 1ull);
        if (P.ti) *P.tau = *P.tau + P.dt;
    }
}

// Chunk totals of the counts.  A sequence of fused steps leaves the flip of
// the step its last launch advanced to the next scan: mode 0 reads neither
// the buffers nor the buffer index, so workgroup 0 flips problems
// [0, flip_n) (counting the step) alongside the reduction.  PT: cells per
// thread of the chunks (0: from each problem's mesh, for launches over
// several problems).
template <int MODE, int PT>
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const ProblemDev *__restrict__ probs, const ScanItem *__restrict__ items,
                                                       int n_items, ProblemDev *flip_probs, int flip_n)
{
    constexpr int NK = PT ? PT : SCAN_PT_MAX;
    __shared__ int64_t s_tmp[BLOCK / 64];
    if (blockIdx.x == 0)
        for (int q = threadIdx.x; q < flip_n; q += BLOCK) flip_problem(flip_probs[q], 1);
    for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
        const ScanItem it = items[w];
        const ProblemDev &P = probs[it.problem];
        const int64_t nc = P.mesh.n_cells;
        const int pt = PT ? PT : scan_per_thread(nc);
        const CellWords<MODE> cw(P);
        int32_t a[NK], b[NK];
        bool ok[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int64_t K = (int64_t)it.chunk * BLOCK * pt + (int64_t)k * BLOCK + threadIdx.x;
            ok[k] = k < pt && K < nc;
            const int64_t Kc = ok[k] ? K : 0;
            a[k] = cw.x[Kc];
            b[k] = cw.y[Kc];
        }
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < NK; ++k) sum += ok[k] ? cw.value(a[k], b[k]) : 0;
        int64_t total;
        block_scan_i64(sum, s_tmp, total);
        if (threadIdx.x == 0) P.scr.chunk[it.chunk] = total;
    }
}

// Local scan + chunk offset -> cell_start of the other buffer.  The chunk's
// offset is the sum of the preceding chunks' totals of its problem, added up
// by the workgroup itself (a few hundred values at most).  Mode 0 also
// resets the arrival counters and sets each cell's placement cursor to its
// first arrival slot (after its stayers).  PT as for k_scan_reduce.
template <int MODE, int PT>
__global__ __launch_bounds__(BLOCK) void k_scan_down(const ProblemDev *__restrict__ probs, const ScanItem *__restrict__ items,
                                                     int n_items)
{
    constexpr int NK = PT ? PT : SCAN_PT_MAX;
    __shared__ int64_t s_tmp[BLOCK / 64];
    for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
        const ScanItem it = items[w];
        const ProblemDev &P = probs[it.problem];
        const int64_t nc = P.mesh.n_cells;
        const StoreDev nxt = P.store[1 - P.cur];
        const int pt = PT ? PT : scan_per_thread(nc);
        const CellWords<MODE> cw(P);
        const int64_t K0 = (int64_t)it.chunk * BLOCK * pt + (int64_t)threadIdx.x * pt;
        int32_t a[NK], b[NK];
        bool ok[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int64_t K = K0 + k;
            ok[k] = k < pt && K < nc;
            const int64_t Kc = ok[k] ? K : 0;
            a[k] = cw.x[Kc];
            b[k] = cw.y[Kc];
        }
        int64_t before = 0, offset, total;
        for (int c = threadIdx.x; c < it.chunk; c += BLOCK) before += P.scr.chunk[c];
        int64_t v[NK];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            v[k] = ok[k] ? cw.value(a[k], b[k]) : 0;
            sum += v[k];
        }
        block_scan_i64(before, s_tmp, offset);
        int64_t run = block_scan_i64(sum, s_tmp, total) + offset;
        const int64_t nch = (nc + (int64_t)BLOCK * pt - 1) / ((int64_t)BLOCK * pt);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int64_t K = K0 + k;
            if (ok[k]) {
                if (MODE == 0) {
                    nxt.cs[K] = (int32_t)run;
                    P.scr.n_arrive[K] = 0;
                    P.scr.cursor[K] = (int32_t)run + a[k];          // after the cell's stayers
                } else {
                    nxt.cs[K] = (int32_t)(run & 0xFFFFFFFFll);
                    P.scr.cursor[K] = (int32_t)(run >> 32);     // first new-id offset of the cell
                }
            }
            run += v[k];
        }
        if (it.chunk == nch - 1 && threadIdx.x == 0) {
            const int64_t tot = offset + total;
            nxt.cs[nc] = (int32_t)(MODE == 0 ? tot : (tot & 0xFFFFFFFFll));
            if (MODE == 1) P.scr.cursor[nc] = (int32_t)(tot >> 32);
        }
    }
}

// ===========================================================================
// place / fix / gather: the stable re-sort by (new cell, moved)
// ===========================================================================
/*
 * Destination of every particle of a tile of cells, each wavefront on its
 * own with no workgroup barrier.  Stayers go to new_start[K] + (rank among
 * the cell's stayers); arrivals get a provisional slot after the destination
 * cell's stayers from an atomic cursor (each cell's first arrival slot, set by
 * the scan), and k_fix orders them afterwards.  A wave takes a run of up to 16
 * consecutive cells of the tile (their particles are consecutive), locates
 * each particle's cell from the run's cell starts, and ranks the stayers of
 * the run with a ballot per 64 particles (the stayers of a cell are the run's
 * stayers minus those of its earlier cells, whose counts are known).  The
 * particles are taken PLACE_BATCH chunks of 64 at a time: the chunks' keys
 * are loaded together, then their cursor atomics are issued together (one
 * per destination cell and chunk: the particles of a cell that leave it tend
 * to leave for the same neighbour), then the arrivals' slots are written.
 */
constexpr int PLACE_RUN = 16;
#ifndef PIC_PLACE_BATCH
#define PIC_PLACE_BATCH 2
#endif
constexpr int PLACE_BATCH = PIC_PLACE_BATCH;
// index of the last of the run's first nr cells whose range starts at or
// before slot sl (the starts are non-decreasing; aq holds them wave-uniform)
__device__ __forceinline__ int run_cell(const int (&aq)[PLACE_RUN], int nr, int sl)
{
    int c = 0;
#pragma unroll
    for (int q = 1; q < PLACE_RUN; ++q) c += (q < nr && aq[q] <= sl) ? 1 : 0;
    return c;
}

__global__ __launch_bounds__(BLOCK) void k_place_waves(const ProblemDev *__restrict__ probs,
                                                       const WorkItem *__restrict__ work, int n_work)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int wb = blockIdx.x; wb < xcd_span(n_work); wb += gridDim.x) {
        const int w = xcd_item(wb, n_work);
        if (w >= n_work) continue;
        const WorkItem wi = work[w];
        const ProblemDev &P = probs[wi.problem];
        const StoreDev cur = P.store[P.cur];
        const StoreDev nxt = P.store[1 - P.cur];
        const uint32_t PIC_G *keys = P.scr.key[P.cur];
        int32_t PIC_G *cursor = P.scr.cursor;
        int32_t PIC_G *src = P.scr.src;
        for (int r0 = wi.c0 + wv * PLACE_RUN; r0 < wi.c1; r0 += (BLOCK / 64) * PLACE_RUN) {
            const int nr = min(PLACE_RUN, wi.c1 - r0);
            // lane q <= nr: old start of cell r0 + q (lane nr: the run's end);
            // lane q < nr: its new start and its stayers
            int a_q = 0, b_q = 0, s_q = 0;
            if (lane <= nr) a_q = cur.cs[r0 + lane];
            if (lane < nr) {
                b_q = nxt.cs[r0 + lane];
                s_q = P.scr.n_stay[r0 + lane];
            }
            int ex = s_q;
#pragma unroll
            for (int o = 1; o < PLACE_RUN; o <<= 1) {
                const int v = __shfl_up(ex, o, 64);
                if (lane >= o) ex += v;
            }
            // the k-th stayer of the run (counting the earlier cells' stayers)
            // that lies in cell q goes to slot d_q + k
            const int d_q = b_q - (ex - s_q);
            int aq[PLACE_RUN];
#pragma unroll
            for (int q = 0; q < PLACE_RUN; ++q) aq[q] = __builtin_amdgcn_readlane(a_q, q);
            const int p0 = aq[0], p1 = __shfl(a_q, nr, 64);
            int carry = 0;
            for (int base = p0; base < p1; base += 64 * PLACE_BATCH) {
                uint32_t key[PLACE_BATCH];
#pragma unroll
                for (int u = 0; u < PLACE_BATCH; ++u) {
                    const int pp = base + 64 * u + lane;
                    key[u] = pp < p1 ? keys[pp] : LOST;
                }
                // stayers' slots by ballot (written at once)
                uint32_t arr = 0;
#pragma unroll
                for (int u = 0; u < PLACE_BATCH; ++u) {
                    const int pp = base + 64 * u + lane;
                    const int c = run_cell(aq, nr, pp);
                    const bool stay = pp < p1 && key[u] == (uint32_t)(r0 + c);
                    const unsigned long long mm = __ballot(stay);
                    const int sl = __shfl(d_q, c, 64) + carry + __popcll(mm & below);
                    if (stay) src[sl] = pp;
                    arr |= (uint32_t)(!stay && key[u] != LOST) << u;
                    carry += __popcll(mm);
                }
                // arrivals: the lanes of a chunk with one destination take
                // consecutive slots in lane order from one atomic, issued by
                // the first of them (lane lead)
                int lead[PLACE_BATCH], rank[PLACE_BATCH], aslot[PLACE_BATCH];
#pragma unroll
                for (int u = 0; u < PLACE_BATCH; ++u) {
                    const bool mine = (arr >> u) & 1u;
                    unsigned long long todo = __ballot(mine);
                    int cnt = 0;
                    lead[u] = 0;
                    rank[u] = 0;
                    while (todo) {
                        const int l = __ffsll((long long)todo) - 1;
                        const uint32_t k = __builtin_amdgcn_readlane(key[u], l);
                        const unsigned long long m = __ballot(mine && key[u] == k);
                        if ((m >> lane) & 1ull) {
                            lead[u] = l;
                            rank[u] = __popcll(m & below);
                        }
                        if (lane == l) cnt = __popcll(m);
                        todo &= ~m;
                    }
                    if (cnt) aslot[u] = atomicAdd(&cursor[key[u]], cnt);
                }
                // the slots are read in straight-line code, so that one wait
                // covers all the atomics (read inside the stores' branches,
                // each would wait for all memory operations again)
#pragma unroll
                for (int u = 0; u < PLACE_BATCH; ++u) {
                    asm volatile("" : "+v"(aslot[u]));
                    aslot[u] = __shfl(aslot[u], lead[u], 64) + rank[u];
                }
#pragma unroll
                for (int u = 0; u < PLACE_BATCH; ++u)
                    if ((arr >> u) & 1u) src[aslot[u]] = base + 64 * u + lane;
            }
        }
    }
}

// Runs of equal keys among consecutive lanes of a wavefront (LOST = no key):
// the lane's run starts at lane `head` and ends before lane `next`.  Every
// lane of the wavefront must call it.
struct WaveRun {
    int lane, head, next;
};
__device__ __forceinline__ WaveRun wave_run(uint32_t key)
{
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool starts = lane == 0 || prev != key;
    const unsigned long long H = __ballot(starts);
    const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    WaveRun r;
    r.lane = lane;
    r.head = 63 - __clzll(H & le);
    const unsigned long long gt = H & ~le;
    r.next = gt ? __ffsll((long long)gt) - 1 : 64;
    return r;
}

// count[key] += 1 for every lane with a key: one atomic per run.
__device__ __forceinline__ void wave_count(int32_t *count, uint32_t key)
{
    const WaveRun r = wave_run(key);
    if (key != LOST && r.lane == r.head) atomicAdd(&count[key], r.next - r.head);
}

// Slot cursor[key]++ for every lane with a key (unspecified for the others):
// one atomic per run; the lanes of a run take consecutive slots in lane order.
__device__ __forceinline__ int32_t wave_take(int32_t *cursor, uint32_t key)
{
    const WaveRun r = wave_run(key);
    int32_t base = 0;
    if (key != LOST && r.lane == r.head) base = atomicAdd(&cursor[key], r.next - r.head);
    base = __shfl(base, r.head, 64);
    return base + (r.lane - r.head);
}

// Wavefront maximum of v, then one atomicMax by lane 0 when it is non-zero.
__device__ __forceinline__ void wave_max_to(unsigned long long *dst, unsigned long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    if ((threadIdx.x & 63) == 0 && v) atomicMax(dst, v);
}

// Placement of an unsorted input (prescribed locations, particles of another
// mesh): every particle is an arrival in its cell; consecutive particles with
// one key take consecutive slots with one atomic.
__global__ __launch_bounds__(BLOCK) void k_place_unsorted(const ProblemDev *__restrict__ probs,
                                                          const RangeItem *__restrict__ items, int n_items)
{
    for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
        const RangeItem it = items[w];
        const ProblemDev &P = probs[it.problem];
        const StoreDev cur = P.store[P.cur];
        const int64_t n = cur.cs[P.mesh.n_cells];
        const int64_t i = it.begin + threadIdx.x;
        const bool mine = i < n && i < it.end;
        const uint32_t key = mine ? P.scr.key[P.cur][i] : LOST;
        const int32_t slot = wave_take(P.scr.cursor, key);
        if (key != LOST) P.scr.src[slot] = (int32_t)i;
    }
}

// Sort each cell's arrivals by their previous position (= previous global
// order, since the previous store was sorted by cell); one thread per cell.
// Up to eight arrivals (most cells) are ranked in registers, up to FIX_LDS
// in LDS (thread t's list interleaved with the others' so that the threads of
// a wave hit distinct banks).  Cells with more (an unsorted input, a
// coarsened mesh) are sorted afterwards one at a
// time by the whole workgroup: each arrival's rank among the cell's arrivals
// (the positions are distinct) is its slot; beyond what LDS holds, the ranks
// are counted over LDS-sized tiles (n^2 / 256 LDS reads per thread).
constexpr int FIX_LDS = 32;
#ifndef PIC_FIX_REGS
#define PIC_FIX_REGS 1                  // 1: up to 8 arrivals ranked in registers; 2: up to 16
#endif

// Sort a[0..n) (distinct values, 2 <= n <= R) in place: every value is loaded
// into registers (loads past the end re-read the last one), and each goes to
// its rank among the others; only the slots whose value changes are written.
template <int R> __device__ __forceinline__ void rank_in_registers(int32_t PIC_G *a, int n)
{
    int32_t r[R];
#pragma unroll
    for (int q = 0; q < R; ++q) r[q] = a[min(q, n - 1)];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        int k = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) k += (j < n && r[j] < r[q]) ? 1 : 0;
        if (q < n && k != q) a[k] = r[q];
    }
}

// Sort a[0..nn) (distinct values) by the whole workgroup: each value's rank
// among the others is its place.  In LDS while the values and their sorted
// copy fit (s_v holds FIX_LDS * BLOCK ints), else counted over LDS-sized tiles
// with the sorted list built in t[0..nn) (memory unused until the next
// advect writes it) and copied back.  Every thread of the workgroup calls it.
__device__ void wg_rank_sort(int32_t PIC_G *a, int nn, int32_t PIC_G *t, int32_t *s_v)
{
    if (2 * nn <= FIX_LDS * BLOCK) {
        int32_t *v = s_v, *o = s_v + nn;
        for (int q = threadIdx.x; q < nn; q += BLOCK) v[q] = a[q];
        __syncthreads();
        for (int q = threadIdx.x; q < nn; q += BLOCK) {
            const int32_t x = v[q];
            int r = 0;
            for (int j = 0; j < nn; ++j) r += v[j] < x;
            o[r] = x;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nn; q += BLOCK) a[q] = o[q];
        __syncthreads();
        return;
    }
    constexpr int TILE = FIX_LDS * BLOCK;
    for (int q0 = 0; q0 < nn; q0 += BLOCK) {
        const int q = q0 + (int)threadIdx.x;
        const int32_t x = q < nn ? a[q] : 0;
        int r = 0;
        for (int j0 = 0; j0 < nn; j0 += TILE) {
            const int m = min(TILE, nn - j0);
            __syncthreads();
            for (int j = threadIdx.x; j < m; j += BLOCK) s_v[j] = a[j0 + j];
            __syncthreads();
            if (q < nn)
                for (int j = 0; j < m; ++j) r += s_v[j] < x;
        }
        if (q < nn) t[r] = x;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nn; q += BLOCK) a[q] = t[q];
    __syncthreads();
}

__global__ __launch_bounds__(BLOCK) void k_fix(const ProblemDev *__restrict__ probs, const RangeItem *__restrict__ items,
                                               int n_items)
{
    __shared__ int32_t s_v[FIX_LDS * BLOCK];
    __shared__ int s_nbig;
    __shared__ int64_t s_big_b[BLOCK];
    __shared__ int s_big_n[BLOCK];
    for (int wb = blockIdx.x; wb < xcd_span(n_items); wb += gridDim.x) {
        const int w = xcd_item(wb, n_items);
        if (w >= n_items) continue;
        const RangeItem it = items[w];
        const ProblemDev &P = probs[it.problem];
        const int64_t K = it.begin + threadIdx.x;
        const bool mine = K < it.end && K < P.mesh.n_cells;
        const StoreDev nxt = P.store[1 - P.cur];
        int64_t b = 0;
        int n = 0;
        if (mine) {                              // the three loads in flight together
            const int32_t c0 = nxt.cs[K], c1 = nxt.cs[K + 1], ns = P.scr.n_stay[K];
            b = (int64_t)c0 + ns;
            n = (int)(c1 - b);
        }
        if (threadIdx.x == 0) s_nbig = 0;
        __syncthreads();
        if (n > FIX_LDS) {
            const int slot = atomicAdd(&s_nbig, 1);
            s_big_b[slot] = b;
            s_big_n[slot] = n;
        } else if (n >= 2 && n <= 8 && PIC_FIX_REGS) {
            // up to eight arrivals (the common case) ranked in registers
            rank_in_registers<8>((gptr_mut<int32_t>)(P.scr.src + b), n);
        } else if (n >= 2 && n <= 16 && PIC_FIX_REGS > 1) {
            rank_in_registers<16>((gptr_mut<int32_t>)(P.scr.src + b), n);
        } else if (n >= 2) {
            auto a = (gptr_mut<int32_t>)(P.scr.src + b);
            int32_t *v = s_v + threadIdx.x;
            // eight loads in flight before the first is stored to LDS (loads
            // past the end re-read the cell's last arrival)
#pragma unroll
            for (int q0 = 0; q0 < FIX_LDS; q0 += 8) {
                if (q0 < n) {
                    int32_t r[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) r[q] = a[min(q0 + q, n - 1)];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (q0 + q < n) v[(q0 + q) * BLOCK] = r[q];
                }
            }
            // each slot's rank among the cell's arrivals (the positions are
            // distinct) is where it goes: n^2 independent LDS reads instead of
            // an insertion sort's chain of dependent ones
            for (int q = 0; q < n; ++q) {
                const int32_t x = v[q * BLOCK];
                int r = 0;
#pragma unroll 8
                for (int j = 0; j < n; ++j) r += v[j * BLOCK] < x;
                a[r] = x;
            }
        }
        __syncthreads();
        const int nbig = s_nbig;
        for (int c = 0; c < nbig; ++c)
            wg_rank_sort((gptr_mut<int32_t>)(P.scr.src + s_big_b[c]), s_big_n[c],
                         (gptr_mut<int32_t>)((int32_t *)P.scr.key[1 - P.cur] + s_big_b[c]), s_v);
        __syncthreads();
    }
}

// Permute the store into the other buffer: new[p] = old[src[p]].
__global__ __launch_bounds__(BLOCK) void k_gather(const ProblemDev *__restrict__ probs, const RangeItem *__restrict__ items,
                                                  int n_items)
{
    for (int wb = blockIdx.x; wb < xcd_span(n_items); wb += gridDim.x) {
        const int w = xcd_item(wb, n_items);
        if (w >= n_items) continue;
        const RangeItem it = items[w];
        const ProblemDev &P = probs[it.problem];
        const StoreDev cur = P.store[P.cur];
        const StoreDev nxt = P.store[1 - P.cur];
        const int64_t n = nxt.cs[P.mesh.n_cells];
        const int64_t p = it.begin + threadIdx.x;
        if (p >= n || p >= it.end) continue;
        const int64_t cap = P.cap;
        const int64_t s = P.scr.src[p];
        const int D = P.mesh.dim;
        const uint32_t K = P.scr.key[P.cur][s];
        if (P.mesh.kind == MESH_UNIFORM) {
            // reference coordinates by the closed form that located the
            // particle (the uniform-mesh advect kernels do not store them)
            int ijk[3];
            cell_ijk(P.mesh, K, ijk);
            for (int a = 0; a < D; ++a) {
                const double x = cur.x[a * cap + s];
                nxt.x[a * cap + p] = x;
                nxt.xr[a * cap + p] = (x - fma((double)ijk[a], P.mesh.h[a], P.mesh.lo[a])) * P.mesh.inv_h[a];
            }
        } else {
            for (int a = 0; a < D; ++a) {
                nxt.x[a * cap + p] = cur.x[a * cap + s];
                nxt.xr[a * cap + p] = cur.xr[a * cap + s];
            }
        }
        nxt.id[p] = cur.id[s];
        nxt.cell[p] = (int32_t)K;
        if (P.prop_f64) {
            const double *ps = (const double *)cur.prop;
            double *pd = (double *)nxt.prop;
            for (int j = 0; j < P.n_prop; ++j) pd[j * cap + p] = ps[j * cap + s];
        } else {
            const float *ps = (const float *)cur.prop;
            float *pd = (float *)nxt.prop;
            for (int j = 0; j < P.n_prop; ++j) pd[j * cap + p] = ps[j * cap + s];
        }
    }
}

// Flip the current buffer of every problem and count the step (a counted
// step also advances the time since t^n of a field that changes in time).
__global__ void k_flip(ProblemDev *probs, int n_probs, int count_step)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_probs) flip_problem(probs[p], count_step);
}

// ===========================================================================
// counter-based random numbers: SplitMix64 (Steele, Lea, Flood 2014) chained
// over the words of a counter (seed, step, cell, slot, axis) -> 53-bit
// uniform in [0, 1)
// ===========================================================================
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double hash_u01(uint64_t seed, uint64_t step, uint64_t cell, uint64_t slot, uint64_t axis)
{
    uint64_t h = splitmix64(seed);
    h = splitmix64(h ^ step);
    h = splitmix64(h ^ cell);
    h = splitmix64(h ^ slot);
    h = splitmix64(h ^ axis);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

// step word of the reference-local generation stream (population steps use
// their step number, Metropolis-Hastings 1 and 2)
constexpr uint64_t SEED_STREAM = ~0ull;

// ===========================================================================
// generation (Sec. 2.2)
// ===========================================================================
// Reference-local generation: one wavefront per cell K writes the cell's
// particles p in [cs[K], cs[K+1]) at x = Phi_K(xr).  xr_in == NULL: particle
// j of the cell takes xr_a = hash_u01(seed, SEED_STREAM, K, j, a) and id
// first_id + p (ids is then unused).
template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_seed_reference(ProblemDev *probs, int prob, const double *__restrict__ xr_in,
                                                          const uint32_t *__restrict__ ids, int64_t n, int prop_init,
                                                          const void *prop_in, uint64_t seed, uint32_t first_id)
{
    const ProblemDev &P = probs[prob];
    const MeshDev &m = P.mesh;
    const StoreDev cur = P.store[P.cur];
    const int64_t cap = P.cap;
    const int64_t K = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (K >= m.n_cells) return;
    const int64_t b = cur.cs[K], e = cur.cs[K + 1];
    unsigned long long idmax = 0;
    for (int64_t p = b + lane; p < e && p < n; p += 64) {
        double t[3], x[3];
        if (xr_in) {
            for (int a = 0; a < D; ++a) t[a] = xr_in[a * n + p];
        } else {
            for (int a = 0; a < D; ++a) t[a] = hash_u01(seed, SEED_STREAM, (uint64_t)K, (uint64_t)(p - b), (uint64_t)a);
        }
        map_to_real<D, KIND>(m, K, t, x);
        for (int a = 0; a < D; ++a) {
            cur.x[a * cap + p] = x[a];
            cur.xr[a * cap + p] = t[a];
        }
        cur.cell[p] = (int32_t)K;
        const uint32_t idp = xr_in ? ids[p] : first_id + (uint32_t)p;
        cur.id[p] = idp;
        for (int j = 0; j < P.n_prop; ++j) {
            double v = prop_init == 1 ? x[j % D]
                                      : (P.prop_f64 ? ((const double *)prop_in)[j * n + p] : (double)((const float *)prop_in)[j * n + p]);
            if (P.prop_f64) ((double *)cur.prop)[j * cap + p] = v;
            else ((float *)cur.prop)[j * cap + p] = (float)v;
        }
        idmax = idmax > (unsigned long long)idp + 1ull ? idmax : (unsigned long long)idp + 1ull;
    }
    if (idmax) atomicMax(&P.scr.next_id[1 + blockIdx.x % STAT_STRIPES], idmax);
}

// next_id = max over the striped maxima (one workgroup of STAT_STRIPES threads)
__global__ void k_reduce_next_id(const ProblemDev *probs)
{
    __shared__ unsigned long long s_m[STAT_STRIPES];
    const ProblemDev &P = probs[0];
    s_m[threadIdx.x] = P.scr.next_id[1 + threadIdx.x];
    __syncthreads();
    for (int o = STAT_STRIPES / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s_m[threadIdx.x] = s_m[threadIdx.x] > s_m[threadIdx.x + o] ? s_m[threadIdx.x] : s_m[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) P.scr.next_id[0] = s_m[0] > P.scr.next_id[0] ? s_m[0] : P.scr.next_id[0];
}

// Prescribed locations: locate each point with the global search and write it
// to the current buffer unsorted; key = cell (or LOST), every point counted as
// an arrival so that the sort machinery orders by (cell, input order).
// Particles of another problem's current buffer (the mesh before refinement
// or coarsening, Sec. 2.5) as an unsorted input of this problem: located in
// this mesh (a child of the old cell after refinement, the parent after
// coarsening), reference location recomputed; location, id and properties
// copied.  The re-sort that follows orders them by (new cell, old order).
template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_transfer_in(const ProblemDev *src_probs, ProblemDev *probs, int prob, int64_t n)
{
    const ProblemDev &S = src_probs[0];
    const ProblemDev &P = probs[prob];
    const MeshDev &m = P.mesh;
    const StoreDev src = S.store[S.cur];
    const StoreDev cur = P.store[P.cur];
    const int64_t scap = S.cap, cap = P.cap;
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p == 0) atomicMax(&P.scr.next_id[1], S.scr.next_id[0]);
    const bool mine = p < n;           // every lane stays for the wavefront atomics
    double x[3] = {0.0, 0.0, 0.0}, t[3];
    if (mine)
        for (int a = 0; a < D; ++a) x[a] = src.x[a * scap + p];
    int32_t K = -1;
    LocStats ls = {0, 0, 0, 0, 0};
    bool ok = mine && in_box_domain<D>(m, x);
    if (ok) {
        if constexpr (KIND == MESH_UNIFORM) {
            ok = locate<D, KIND>(m, x, 0, K, t, ls);
        } else if constexpr (KIND == MESH_OCTREE) {
            K = octree_lookup(m, x);
            map_to_ref<D, KIND>(m, K, x, t);
        } else {
            ok = global_search_displaced<D>(m, x, K, t, ls);
        }
    }
    uint32_t id = 0;
    if (mine) {
        for (int a = 0; a < D; ++a) {
            cur.x[a * cap + p] = x[a];
            cur.xr[a * cap + p] = ok ? t[a] : 0.0;
        }
        cur.cell[p] = -1;
        id = src.id[p];
        cur.id[p] = id;
        for (int j = 0; j < P.n_prop; ++j) {
            if (P.prop_f64) ((double *)cur.prop)[j * cap + p] = ((const double *)src.prop)[j * scap + p];
            else ((float *)cur.prop)[j * cap + p] = ((const float *)src.prop)[j * scap + p];
        }
        P.scr.key[P.cur][p] = ok ? (uint32_t)K : LOST;
    }
    wave_count(P.scr.n_arrive, ok ? (uint32_t)K : LOST);
    const int lost = wave_sum((int)(mine && !ok));
    if ((threadIdx.x & 63) == 0 && lost)
        atomicAdd(&P.scr.stats[(blockIdx.x % STAT_STRIPES) * ST_COUNT + ST_LOST], (unsigned long long)lost);
    wave_max_to(&P.scr.next_id[1 + blockIdx.x % STAT_STRIPES], mine ? (unsigned long long)id + 1ull : 0ull);
}

template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_seed_positions(ProblemDev *probs, int prob, const double *__restrict__ x_in,
                                                          const uint32_t *__restrict__ ids, int64_t n, int prop_init,
                                                          const void *prop_in)
{
    const ProblemDev &P = probs[prob];
    const MeshDev &m = P.mesh;
    const StoreDev cur = P.store[P.cur];
    const int64_t cap = P.cap;
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool mine = p < n;           // every lane stays for the wavefront atomics
    double x[3] = {0.0, 0.0, 0.0}, t[3];
    if (mine)
        for (int a = 0; a < D; ++a) x[a] = x_in[a * n + p];
    int32_t K = -1;
    LocStats ls = {0, 0, 0, 0, 0};
    bool ok = mine && in_box_domain<D>(m, x);
    if (ok) {
        if constexpr (KIND == MESH_UNIFORM) {
            ok = locate<D, KIND>(m, x, 0, K, t, ls);
        } else if constexpr (KIND == MESH_OCTREE) {
            K = octree_lookup(m, x);
            map_to_ref<D, KIND>(m, K, x, t);
        } else {
            ok = global_search_displaced<D>(m, x, K, t, ls);
        }
    }
    uint32_t id = 0;
    if (mine) {
        for (int a = 0; a < D; ++a) {
            cur.x[a * cap + p] = x[a];
            cur.xr[a * cap + p] = ok ? t[a] : 0.0;
        }
        cur.cell[p] = -1;
        id = ids[p];
        cur.id[p] = id;
        for (int j = 0; j < P.n_prop; ++j) {
            double v = prop_init == 1 ? x[j % D]
                                      : (P.prop_f64 ? ((const double *)prop_in)[j * n + p] : (double)((const float *)prop_in)[j * n + p]);
            if (P.prop_f64) ((double *)cur.prop)[j * cap + p] = v;
            else ((float *)cur.prop)[j * cap + p] = (float)v;
        }
        P.scr.key[P.cur][p] = ok ? (uint32_t)K : LOST;
    }
    wave_count(P.scr.n_arrive, ok ? (uint32_t)K : LOST);
    const int lost = wave_sum((int)(mine && !ok));
    if ((threadIdx.x & 63) == 0 && lost)
        atomicAdd(&P.scr.stats[(blockIdx.x % STAT_STRIPES) * ST_COUNT + ST_LOST], (unsigned long long)lost);
    wave_max_to(&P.scr.next_id[1 + blockIdx.x % STAT_STRIPES], mine ? (unsigned long long)id + 1ull : 0ull);
}

// ===========================================================================
// particle -> cell transfer (Sec. 2.7)
// ===========================================================================
__device__ __forceinline__ double load_prop(const ProblemDev &P, const StoreDev &s, int j, int64_t i)
{
    return P.prop_f64 ? ((const double *)s.prop)[j * P.cap + i] : (double)((const float *)s.prop)[j * P.cap + i];
}

// One wavefront per cell: arithmetic mean of every property (NaN if empty).
// mode 0: arithmetic mean; 1: geometric, exp of the mean logarithm; 2:
// harmonic, n over the sum of reciprocals (Sec. 2.7 (ii)).
__global__ __launch_bounds__(BLOCK) void k_interp_average(const ProblemDev *__restrict__ probs, int prob,
                                                          double *__restrict__ out, int32_t *__restrict__ count,
                                                          int mode)
{
    const ProblemDev &P = probs[prob];
    const StoreDev cur = P.store[P.cur];
    const int64_t K = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (K >= P.mesh.n_cells) return;
    const int64_t b = cur.cs[K], e = cur.cs[K + 1];
    if (lane == 0) count[K] = (int32_t)(e - b);
    for (int j = 0; j < P.n_prop; ++j) {
        double s = 0.0;
        for (int64_t i = b + lane; i < e; i += 64) {
            const double v = load_prop(P, cur, j, i);
            s += mode == 0 ? v : (mode == 1 ? log(v) : 1.0 / v);
        }
        s = wave_sum(s);
        const double n = (double)(e - b);
        if (lane == 0)
            out[K * P.n_prop + j] = (e == b) ? __builtin_nan("") : (mode == 0 ? s / n : (mode == 1 ? exp(s / n) : n / s));
    }
}

// Evaluation points in reference coordinates, the same for every cell,
// passed by value (no device allocation).
constexpr int MAX_EVAL_POINTS = 64;
struct EvalPoints {
    double q[3][MAX_EVAL_POINTS];
    int n;
};

// Wavefront minimum of (d2, index), ties to the lower index.
__device__ __forceinline__ void wave_argmin(double &d2, int64_t &idx)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double od = __shfl_xor(d2, o, 64);
        const int64_t oi = __shfl_xor(idx, o, 64);
        if (od < d2 || (od == d2 && oi < idx)) {
            d2 = od;
            idx = oi;
        }
    }
}

/*
 * One wavefront per cell: properties at the evaluation points from the
 * cell's particles (Sec. 2.7): kind 0 nearest particle in physical distance
 * (ties to the first in store order); 1 weights 1/|x_q - x_k|^2 (particles
 * at the point share the whole weight); 2 weights prod_a [(1 - q_a)(1 - xr_a)
 * + q_a xr_a], the sum over the cell's vertices of N_v(q) N_v(xr).
 * out [n_cells][n_q][n_prop], NaN for empty cells.
 */
template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_interp_points(const ProblemDev *__restrict__ probs, int prob, int kind,
                                                         EvalPoints qp, double *__restrict__ out,
                                                         int32_t *__restrict__ count)
{
    const ProblemDev &P = probs[prob];
    const MeshDev &m = P.mesh;
    const StoreDev cur = P.store[P.cur];
    const int64_t cap = P.cap;
    const int64_t K = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (K >= m.n_cells) return;
    const int64_t b = cur.cs[K], e = cur.cs[K + 1];
    const int np = P.n_prop;
    if (count && lane == 0) count[K] = (int32_t)(e - b);
    for (int q = 0; q < qp.n; ++q) {
        double* o = out + (K * qp.n + q) * np;
        if (e == b) {
            for (int j = lane; j < np; j += 64) o[j] = __builtin_nan("");
            continue;
        }
        double tq[3] = {qp.q[0][q], qp.q[1][q], D == 3 ? qp.q[2][q] : 0.0}, xq[3];
        map_to_real<D, KIND>(m, K, tq, xq);
        auto dist2 = [&](int64_t i) {
            double d2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double r = cur.x[a * cap + i] - xq[a];
                d2 = fma(r, r, d2);
            }
            return d2;
        };
        if (kind == 0) {
            double bd = __builtin_inf();
            int64_t bi = INT64_MAX;
            for (int64_t i = b + lane; i < e; i += 64) {
                const double d2 = dist2(i);
                if (d2 < bd) {
                    bd = d2;
                    bi = i;
                }
            }
            wave_argmin(bd, bi);
            for (int j = lane; j < np; j += 64) o[j] = load_prop(P, cur, j, bi);
            continue;
        }
        int hits = 0;
        if (kind == 1) {
            for (int64_t i = b + lane; i < e; i += 64) hits += dist2(i) == 0.0;
            hits = wave_sum(hits);
        }
        for (int j = 0; j < np; ++j) {
            double sw = 0.0, swp = 0.0;
            for (int64_t i = b + lane; i < e; i += 64) {
                double w;
                if (kind == 1) {
                    const double d2 = dist2(i);
                    w = hits ? (d2 == 0.0 ? 1.0 : 0.0) : 1.0 / d2;
                } else {
                    w = 1.0;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const double t = cur.xr[a * cap + i];
                        w *= (1.0 - tq[a]) * (1.0 - t) + tq[a] * t;
                    }
                }
                sw += w;
                swp = fma(w, load_prop(P, cur, j, i), swp);
            }
            sw = wave_sum(sw);
            swp = wave_sum(swp);
            if (lane == 0) o[j] = swp / sw;
        }
    }
}

// Eigenvalues of a symmetric 3x3 matrix (trigonometric closed form).
__device__ inline void sym3_eig(const double A[3][3], double ev[3])
{
    double p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double q = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    if (p1 == 0.0) {
        ev[0] = A[0][0];
        ev[1] = A[1][1];
        ev[2] = A[2][2];
        return;
    }
    double p2 = (A[0][0] - q) * (A[0][0] - q) + (A[1][1] - q) * (A[1][1] - q) + (A[2][2] - q) * (A[2][2] - q) + 2.0 * p1;
    double p = sqrt(p2 / 6.0);
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = (A[i][j] - (i == j ? q : 0.0)) / p;
    double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                  B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    double r = fmin(1.0, fmax(-1.0, detB / 2.0));
    double phi = acos(r) / 3.0;
    ev[0] = q + 2.0 * p * cos(phi);
    ev[2] = q + 2.0 * p * cos(phi + 2.0943951023931954923);
    ev[1] = 3.0 * q - ev[0] - ev[2];
}

/*
 * One wavefront per cell: least squares c0 + c.(xr - xbar) in centred
 * reference coordinates.  Two passes over the cell's particles (means, then
 * centred second moments), FP64 normal equations solved by Cramer's rule;
 * constant fit when n < dim+1 or sigma_min/sigma_max < 1e-10 (the singular
 * values of [1 | X - xbar] are sqrt(n) and those of X - xbar).
 */
template <int D>
__global__ __launch_bounds__(BLOCK) void k_interp_lls(const ProblemDev *__restrict__ probs, int prob, double *__restrict__ out,
                                                      double *__restrict__ xbar_out, int32_t *__restrict__ count)
{
    const ProblemDev &P = probs[prob];
    const StoreDev cur = P.store[P.cur];
    const int64_t cap = P.cap;
    const int64_t K = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (K >= P.mesh.n_cells) return;
    const int64_t b = cur.cs[K], e = cur.cs[K + 1], n = e - b;
    const int np = P.n_prop;
    double *o = out + K * np * (D + 1);
    if (lane == 0) count[K] = (int32_t)n;
    if (n == 0) {
        if (lane == 0) {
            for (int j = 0; j < np * (D + 1); ++j) o[j] = __builtin_nan("");
            for (int a = 0; a < D; ++a) xbar_out[K * D + a] = __builtin_nan("");
        }
        return;
    }
    double xb[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
        double s = 0.0;
        for (int64_t i = b + lane; i < e; i += 64) s += cur.xr[a * cap + i];
        xb[a] = wave_sum(s) / (double)n;
    }
    double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int r = 0; r < D; ++r)
        for (int c = r; c < D; ++c) {
            double s = 0.0;
            for (int64_t i = b + lane; i < e; i += 64) s += (cur.xr[r * cap + i] - xb[r]) * (cur.xr[c * cap + i] - xb[c]);
            s = wave_sum(s);
            C[r][c] = C[c][r] = s;
        }
    bool full = n >= D + 1;
    if (full) {
        double ev[3];
        if constexpr (D == 3) {
            sym3_eig(C, ev);
        } else {
            double tr = C[0][0] + C[1][1], det = C[0][0] * C[1][1] - C[0][1] * C[1][0];
            double disc = sqrt(fmax(0.0, tr * tr / 4.0 - det));
            ev[0] = tr / 2.0 + disc;
            ev[1] = tr / 2.0 - disc;
            ev[2] = ev[1];
        }
        double emin = ev[0], emax = ev[0];
        for (int a = 1; a < D; ++a) {
            emin = fmin(emin, ev[a]);
            emax = fmax(emax, ev[a]);
        }
        double smin = sqrt(fmax(emin, 0.0)), smax = sqrt(fmax(emax, 0.0));
        double sn = sqrt((double)n);
        full = fmin(sn, smin) >= 1e-10 * fmax(sn, smax);
    }
    for (int j = 0; j < np; ++j) {
        double s = 0.0;
        for (int64_t i = b + lane; i < e; i += 64) s += load_prop(P, cur, j, i);
        double mean = wave_sum(s) / (double)n;
        double r[3] = {0, 0, 0}, c[3] = {0, 0, 0};
        if (full) {
            for (int a = 0; a < D; ++a) {
                double q = 0.0;
                for (int64_t i = b + lane; i < e; i += 64) q += (cur.xr[a * cap + i] - xb[a]) * (load_prop(P, cur, j, i) - mean);
                r[a] = wave_sum(q);
            }
            solve_small<D>(C, r, c);
        }
        if (lane == 0) {
            o[j * (D + 1)] = mean;
            for (int a = 0; a < D; ++a) o[j * (D + 1) + 1 + a] = full ? c[a] : 0.0;
        }
    }
    if (lane == 0)
        for (int a = 0; a < D; ++a) xbar_out[K * D + a] = xb[a];
}

// ===========================================================================
// population management (Sec. 2.5; properties of new particles Sec. 2.6)
// ===========================================================================
// Scalar density repacked into the field layout (value in the first component).
template <int D>
__global__ void k_pack_density(const double *__restrict__ rho, int64_t nn, typename NodeVec<D, double>::type *R,
                               int *nonfinite)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    const double v = rho[g];
    if (!isfinite(v)) atomicOr(nonfinite, 1);
    typename NodeVec<D, double>::type r{};
    r.x = v;
    R[g] = r;
}

// Exclusive scan of per-cell counts by one workgroup (cell starts of a
// generation call): each thread sums a contiguous run of cells, a workgroup
// scan offsets the runs.  out[nc] = total, *total = the same as int64, and
// *negative = 1 if a count is negative.
__global__ __launch_bounds__(BLOCK) void k_counts_scan(const int32_t *__restrict__ counts, int64_t nc, int32_t *out,
                                                       int64_t *total, int32_t *negative)
{
    __shared__ int64_t s_tmp[BLOCK / 64];
    const int64_t per = (nc + BLOCK - 1) / BLOCK;
    const int64_t b = (int64_t)threadIdx.x * per, e = b + per < nc ? b + per : nc;
    int64_t sum = 0;
    bool neg = false;
    for (int64_t K = b; K < e; ++K) {
        const int32_t v = counts[K];
        neg |= v < 0;
        sum += v > 0 ? v : 0;
    }
    int64_t tot;
    int64_t run = block_scan_i64(sum, s_tmp, tot);
    for (int64_t K = b; K < e; ++K) {
        out[K] = (int32_t)run;
        const int32_t v = counts[K];
        run += v > 0 ? v : 0;
    }
    if (neg) atomicOr(negative, 1);
    if (threadIdx.x == 0) {
        out[nc] = (int32_t)tot;
        *total = tot;
    }
}

// Zero n bytes (a kernel rather than a memset, so that it can sit anywhere in
// a stream, graphs included).
__global__ void k_zero_bytes(unsigned char *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

/*
 * Metropolis-Hastings generation (Sec. 2.2), one thread per cell K: a chain
 * in the reference cell with a proposal uniform in it, starting at its
 * centre; state i proposes coordinates hash_u01(seed, 1, K, i, axis) and moves
 * there when hash_u01(seed, 2, K, i, 0) * rho^(current) < rho^(proposal),
 * rho^ = max(0, rho_h) |det grad Phi_K|.  States J-1, 2J-1, ... are written
 * to the cell's slots of the current buffer (cell_start already set), ids
 * first_id + slot, properties = initial position.  The longest run of equal
 * consecutive states goes to *longest.
 */
template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_seed_mh(ProblemDev *probs, int prob,
                                                   const typename NodeVec<D, double>::type *__restrict__ R, int J,
                                                   uint64_t seed, uint32_t first_id, unsigned long long *longest)
{
    const ProblemDev &P = probs[prob];
    const MeshDev &m = P.mesh;
    const StoreDev cur = P.store[P.cur];
    const int64_t cap = P.cap;
    const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= m.n_cells) return;
    auto density = [&](const double *t) {
        double u[3], Jm[3][3];
        eval_q2<D, double, KIND>(m, R, K, t, u);
        map_jacobian<D, KIND>(m, K, t, Jm);
        const double det = D == 2 ? Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]
                                  : Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                                        Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                                        Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
        return fmax(u[0], 0.0) * fabs(det);
    };
    const int64_t b = cur.cs[K], e = cur.cs[K + 1];
    double t[3] = {0.5, 0.5, 0.5};
    double rc = density(t);
    long long run = 0, best = 0;
    unsigned long long idmax = 0;
    const long long n_states = (long long)J * (e - b);
    int64_t p = b;
    for (long long i = 0; i < n_states; ++i) {
        double tp[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) tp[a] = hash_u01(seed, 1, (uint64_t)K, (uint64_t)i, (uint64_t)a);
        const double rp = density(tp);
        const double u = hash_u01(seed, 2, (uint64_t)K, (uint64_t)i, 0);
        if (u * rc < rp) {
            for (int a = 0; a < D; ++a) t[a] = tp[a];
            rc = rp;
            run = 1;
        } else {
            ++run;
        }
        best = run > best ? run : best;
        if ((i + 1) % J == 0) {
            double x[3];
            map_to_real<D, KIND>(m, K, t, x);
            for (int a = 0; a < D; ++a) {
                cur.x[a * cap + p] = x[a];
                cur.xr[a * cap + p] = t[a];
            }
            cur.cell[p] = (int32_t)K;
            const uint32_t id = first_id + (uint32_t)p;
            cur.id[p] = id;
            for (int j = 0; j < P.n_prop; ++j) {
                if (P.prop_f64) ((double *)cur.prop)[j * cap + p] = x[j % D];
                else ((float *)cur.prop)[j * cap + p] = (float)x[j % D];
            }
            idmax = idmax > (unsigned long long)id + 1ull ? idmax : (unsigned long long)id + 1ull;
            ++p;
        }
    }
    if (best) atomicMax(longest, (unsigned long long)best);
    if (idmax) atomicMax(&P.scr.next_id[1 + blockIdx.x % STAT_STRIPES], idmax);
}

/*
 * One wavefront per cell.  Keeps the cell's particles except the ones whose
 * id is among the (n - max) largest (stable compaction by ballot), then
 * appends min - kept new particles.  The packed scan left the new cell_start
 * in the other buffer and each cell's first new-id offset in cursor[].
 */
template <int D, int KIND>
__global__ __launch_bounds__(BLOCK) void k_population(const ProblemDev *__restrict__ probs, int prob, uint64_t seed,
                                                      uint64_t step)
{
    const ProblemDev &P = probs[prob];
    const MeshDev &m = P.mesh;
    const StoreDev cur = P.store[P.cur];
    const StoreDev nxt = P.store[1 - P.cur];
    const int64_t cap = P.cap;
    const int64_t K = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (K >= m.n_cells) return;
    const int64_t b = cur.cs[K], e = cur.cs[K + 1], n = e - b;
    const int64_t del = n > P.pop_max ? n - P.pop_max : 0;
    int64_t q = nxt.cs[K];
    const int np = P.n_prop;
    double psum[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // property sums of survivors (first 8 props by lanes)
    int kept = 0;
    for (int64_t c0 = b; c0 < e; c0 += 64) {
        const int64_t i = c0 + lane;
        bool keep = false;
        if (i < e) {
            keep = true;
            if (del > 0) {
                const uint32_t myid = cur.id[i];
                int64_t larger = 0;
                for (int64_t k = b; k < e; ++k) larger += cur.id[k] > myid;
                keep = larger >= del;
            }
        }
        const unsigned long long msk = __ballot(keep);
        const int pre = __popcll(msk & ((1ull << lane) - 1ull));
        if (keep) {
            const int64_t d = q + pre;
            for (int a = 0; a < D; ++a) {
                nxt.x[a * cap + d] = cur.x[a * cap + i];
                nxt.xr[a * cap + d] = cur.xr[a * cap + i];
            }
            nxt.id[d] = cur.id[i];
            nxt.cell[d] = (int32_t)K;
            for (int j = 0; j < np; ++j) {
                double v = load_prop(P, cur, j, i);
                if (P.prop_f64) ((double *)nxt.prop)[j * cap + d] = v;
                else ((float *)nxt.prop)[j * cap + d] = (float)v;
            }
        }
        q += __popcll(msk);
        kept += __popcll(msk);
    }
    const int64_t add = kept < P.pop_min ? P.pop_min - kept : 0;
    if (add > 0) {
        const uint64_t id0 = P.scr.next_id[0] + (uint64_t)P.scr.cursor[K];
        for (int64_t s0 = 0; s0 < add; s0 += 64) {
            const int64_t s = s0 + lane;
            if (s < add) {
                double t[3], x[3];
                for (int a = 0; a < D; ++a) t[a] = hash_u01(seed, step, (uint64_t)K, (uint64_t)s, (uint64_t)a);
                map_to_real<D, KIND>(m, K, t, x);
                const int64_t d = q + s;
                for (int a = 0; a < D; ++a) {
                    nxt.x[a * cap + d] = x[a];
                    nxt.xr[a * cap + d] = t[a];
                }
                nxt.id[d] = (uint32_t)(id0 + (uint64_t)s);
                nxt.cell[d] = (int32_t)K;
            }
        }
        // properties: mean of the survivors (now at [nxt.cs[K], q)), or the initial position
        const int64_t sb = nxt.cs[K];
        for (int j = 0; j < np; ++j) {
            double sum = 0.0;
            for (int64_t i = sb + lane; i < q; i += 64)
                sum += P.prop_f64 ? ((const double *)nxt.prop)[j * cap + i] : (double)((const float *)nxt.prop)[j * cap + i];
            sum = wave_sum(sum);
            for (int64_t s = lane; s < add; s += 64) {
                const int64_t d = q + s;
                double v = kept > 0 ? sum / (double)kept : nxt.x[(j % D) * cap + d];
                if (P.prop_f64) ((double *)nxt.prop)[j * cap + d] = v;
                else ((float *)nxt.prop)[j * cap + d] = (float)v;
            }
        }
    }
    if (lane == 0) {
        unsigned long long *st = P.scr.stats + (blockIdx.x % STAT_STRIPES) * ST_COUNT;
        if (del) atomicAdd(&st[ST_DELETED], (unsigned long long)del);
        if (add) atomicAdd(&st[ST_ADDED], (unsigned long long)add);
    }
    (void)psum;
}

// next_id += total additions; flip buffers.
__global__ void k_population_finish(ProblemDev *probs, int prob)
{
    ProblemDev &P = probs[prob];
    P.scr.next_id[0] += (unsigned long long)(uint32_t)P.scr.cursor[P.mesh.n_cells];
    P.cur = 1 - P.cur;
}

// Non-finite check and repacking of the nodal field into the kernels' layout.
template <int D>
__global__ void k_repack_field(const void *U, int src_f32, int64_t nn, void *u64, void *u32, int *flag)
{
    const int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (g >= nn) return;
    double v[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) v[a] = src_f32 ? (double)((const float *)U)[a * nn + g] : ((const double *)U)[a * nn + g];
    if (flag) {                 // check pass: nothing is written but the flag
        bool bad = false;
        for (int a = 0; a < D; ++a) bad |= !isfinite(v[a]);
        if (bad) atomicOr(flag, 1);
        return;
    }
    if constexpr (D == 3) {
        ((double4 *)u64)[g] = make_double4(v[0], v[1], v[2], 0.0);
        ((float4 *)u32)[g] = make_float4((float)v[0], (float)v[1], (float)v[2], 0.f);
    } else {
        ((double2 *)u64)[g] = make_double2(v[0], v[1]);
        ((float2 *)u32)[g] = make_float2((float)v[0], (float)v[1]);
    }
}

}  // namespace pic

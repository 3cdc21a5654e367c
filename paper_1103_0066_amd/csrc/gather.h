// Vertex gradients without global atomics: the adjoint writes J-bar per
// element, and one thread per vertex sums the contributions of the elements
// around it, read through a vertex-to-element incidence (CSR) built once per
// mesh.  Global atomics execute at the memory side on MI355X (they bypass
// L2), so for repeated adjoints on one mesh this gather replaces ~3 atomics
// per distinct vertex of every wave's tile by plain reads of 36 bytes per
// element and one read-modify-write per vertex.  Incidences are sorted and
// combined in a fixed order, so every run gives the same bits.
//
// Contribution of element e to its vertex a (reverse of J = [x_1 - x_0 | ...]):
// column a - 1 of J-bar for a > 0, minus the sum of its columns for a = 0.
#pragma once

#include "geometry.h"
#include "params.h"

namespace fei {

__global__ __launch_bounds__(256) void incidence_zero_kernel(int32_t *a, int64_t n)
{
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += gridDim.x * 256ll) a[i] = 0;
}

// Count and fill take the references in batches of kIncBatch per workgroup
// and first merge them per vertex in an LDS open-addressing table (CAS on the
// key, LDS atomics on the count): on a mesh with locality a batch names far
// fewer distinct vertices than references (about a fifth for consecutive Kuhn
// tets), and global atomics, which execute at the memory side, are the cost.
// The table has twice as many slots as a batch has references, so it never
// fills and every probe sequence ends.
constexpr int kIncBatch = 1024;
constexpr int kIncSlots = 2 * kIncBatch;

__device__ __forceinline__ int inc_slot(int32_t v)
{
    return int((unsigned(v) * 2654435761u) >> (32 - 11));   // 11 bits: kIncSlots
}

// Inserts v into the table; returns its slot.
__device__ __forceinline__ int inc_insert(int32_t *key, int32_t v)
{
    int h = inc_slot(v);
    for (int probe = 0; probe < kIncSlots; ++probe) {
        const int32_t old = atomicCAS(key + h, -1, v);
        if (old == -1 || old == v) break;
        h = (h + 1) & (kIncSlots - 1);
    }
    return h;
}

__device__ __forceinline__ void inc_clear(int32_t *key, int32_t *cnt)
{
    for (int i = threadIdx.x; i < kIncSlots; i += 256) {
        key[i] = -1;
        cnt[i] = 0;
    }
}

// deg[v + 1] = number of incidences of v (ptr[0] stays 0; ptr zeroed before).
__global__ __launch_bounds__(256) void incidence_count_kernel(Incidence g)
{
    __shared__ int32_t key[kIncSlots];
    __shared__ int32_t cnt[kIncSlots];
    const int64_t total = g.n_elements * g.nv;
    inc_clear(key, cnt);
    __syncthreads();
    for (int64_t base = blockIdx.x * int64_t(kIncBatch); base < total;
         base += gridDim.x * int64_t(kIncBatch)) {
#pragma unroll
        for (int k = 0; k < kIncBatch / 256; ++k) {
            const int64_t i = base + threadIdx.x + 256 * k;
            if (i < total) {
                const int32_t v = g.conn[i];
                if (v >= 0 && v < g.n_vertices) atomicAdd(cnt + inc_insert(key, v), 1);
            }
        }
        __syncthreads();
        for (int sl = threadIdx.x; sl < kIncSlots; sl += 256) {
            const int32_t v = key[sl];
            if (v >= 0) atomicAdd(g.ptr + v + 1, cnt[sl]);
        }
        __syncthreads();
        inc_clear(key, cnt);
        __syncthreads();
    }
}

// In-place inclusive scan of ptr[0 .. n) by one workgroup: each thread scans a
// contiguous chunk, the chunk totals are scanned in LDS, then added back.
// The chunk loops read 16 values per step into registers before using any,
// so a thread waits for one memory latency per 16 values, not per value.
// Used for short arrays (up to one block of the multi-block scan below, and
// that scan's block totals).
constexpr int kScanBatch = 16;
__global__ __launch_bounds__(1024) void incidence_scan_kernel(int32_t *ptr, int64_t n)
{
    __shared__ int32_t tot[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk < n ? t * chunk : n, e = (b + chunk < n) ? b + chunk : n;
    int32_t run = 0;
    int64_t i = b;
    for (; i + kScanBatch <= e; i += kScanBatch) {
        int32_t v[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) v[k] = ptr[i + k];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) run += v[k];
    }
    for (; i < e; ++i) run += ptr[i];
    tot[t] = run;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = t >= off ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int32_t acc = t > 0 ? tot[t - 1] : 0;
    i = b;
    for (; i + kScanBatch <= e; i += kScanBatch) {
        int32_t v[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) v[k] = ptr[i + k];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            acc += v[k];
            ptr[i + k] = acc;
        }
    }
    for (; i < e; ++i) {
        acc += ptr[i];
        ptr[i] = acc;
    }
}

// Multi-block inclusive scan of ptr[0 .. n): each workgroup scans its
// kScanBlock entries (loaded and stored coalesced through LDS, 16 contiguous
// values per thread, one padding word per 16 so the per-thread runs fall in
// different banks) and writes its total to sums[block]; the totals are
// scanned by incidence_scan_kernel and added back by incidence_add_kernel.
constexpr int kScanBlock = 16 * 256;
__global__ __launch_bounds__(256) void incidence_scan_blocks_kernel(int32_t *ptr, int64_t n,
                                                                    int32_t *sums)
{
    __shared__ int32_t buf[kScanBlock + kScanBlock / 16];
    __shared__ int32_t tot[256];
    const int t = threadIdx.x;
    const int64_t b0 = blockIdx.x * int64_t(kScanBlock);
    auto pad = [](int j) { return j + (j >> 4); };
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = k * 256 + t;
        buf[pad(j)] = (b0 + j < n) ? ptr[b0 + j] : 0;
    }
    __syncthreads();
    int32_t v[16];
    int32_t run = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        run += buf[pad(16 * t + k)];
        v[k] = run;
    }
    tot[t] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t x = t >= off ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += x;
        __syncthreads();
    }
    const int32_t pre = t > 0 ? tot[t - 1] : 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) buf[pad(16 * t + k)] = v[k] + pre;
    if (t == 255) sums[blockIdx.x] = tot[255];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = k * 256 + t;
        if (b0 + j < n) ptr[b0 + j] = buf[pad(j)];
    }
}

__global__ __launch_bounds__(256) void incidence_add_kernel(int32_t *ptr, int64_t n,
                                                            const int32_t *sums)
{
    const int64_t blk = blockIdx.x + 1;           // block 0 has no offset
    const int32_t off = sums[blk - 1];
    const int64_t b0 = blk * int64_t(kScanBlock);
    for (int j = threadIdx.x; j < kScanBlock; j += 256)
        if (b0 + j < n) ptr[b0 + j] += off;
}

// inc[ptr[v] + slot] = e * nv + a for every reference; the slots of one
// vertex are reserved per batch with one global atomic and handed out by LDS
// atomics, so their order is arbitrary until the sort.
__global__ __launch_bounds__(256) void incidence_fill_kernel(Incidence g)
{
    __shared__ int32_t key[kIncSlots];
    __shared__ int32_t cnt[kIncSlots];       // batch count, then the batch's base in the list
    const int64_t total = g.n_elements * g.nv;
    inc_clear(key, cnt);
    __syncthreads();
    for (int64_t base = blockIdx.x * int64_t(kIncBatch); base < total;
         base += gridDim.x * int64_t(kIncBatch)) {
        int slot[kIncBatch / 256], rank[kIncBatch / 256];
#pragma unroll
        for (int k = 0; k < kIncBatch / 256; ++k) {
            const int64_t i = base + threadIdx.x + 256 * k;
            slot[k] = -1;
            rank[k] = 0;
            if (i < total) {
                const int32_t v = g.conn[i];
                if (v >= 0 && v < g.n_vertices) {
                    slot[k] = inc_insert(key, v);
                    rank[k] = atomicAdd(cnt + slot[k], 1);
                }
            }
        }
        __syncthreads();
        for (int sl = threadIdx.x; sl < kIncSlots; sl += 256) {
            const int32_t v = key[sl];
            if (v >= 0) cnt[sl] = g.ptr[v] + atomicAdd(g.cursor + v, cnt[sl]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kIncBatch / 256; ++k)
            if (slot[k] >= 0) g.inc[cnt[slot[k]] + rank[k]] = int32_t(base + threadIdx.x + 256 * k);
        __syncthreads();
        inc_clear(key, cnt);
        __syncthreads();
    }
}

// In-place heapsort of a[0 .. n) (O(n log n) for vertices of any degree).
__device__ inline void heap_sort(int32_t *a, int32_t n)
{
    auto sift = [a](int32_t root, int32_t end) {
        for (;;) {
            int32_t c = 2 * root + 1;
            if (c >= end) return;
            if (c + 1 < end && a[c + 1] > a[c]) ++c;
            if (a[root] >= a[c]) return;
            const int32_t t = a[root];
            a[root] = a[c];
            a[c] = t;
            root = c;
        }
    };
    for (int32_t r = n / 2 - 1; r >= 0; --r) sift(r, n);
    for (int32_t end = n - 1; end > 0; --end) {
        const int32_t t = a[0];
        a[0] = a[end];
        a[end] = t;
        sift(0, end);
    }
}

// Sorts every vertex's incidences.  A wave takes kSortVerts consecutive
// vertices: their lists (up to 64 entries each, one per lane) are loaded
// together, each entry's rank is the number of smaller entries of its list
// (the entries are distinct), and every entry is stored at its rank.  Longer
// lists (vertices of degree above 64) are heap-sorted by one lane.
constexpr int kSortVerts = 8;
__global__ __launch_bounds__(256) void incidence_sort_kernel(Incidence g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * 256ll + threadIdx.x) >> 6;
    const int64_t n_waves = (int64_t(gridDim.x) * 256) >> 6;
    for (int64_t v0 = wave * kSortVerts; v0 < g.n_vertices; v0 += n_waves * kSortVerts) {
        int32_t b[kSortVerts + 1];
#pragma unroll
        for (int j = 0; j <= kSortVerts; ++j)
            b[j] = g.ptr[v0 + j < g.n_vertices ? v0 + j : g.n_vertices];
        int32_t x[kSortVerts];
#pragma unroll
        for (int j = 0; j < kSortVerts; ++j) {
            const int32_t L = b[j + 1] - b[j];
            x[j] = (L <= 64 && lane < L) ? g.inc[b[j] + lane] : 0;
        }
#pragma unroll
        for (int j = 0; j < kSortVerts; ++j) {
            const int32_t L = b[j + 1] - b[j];
            if (L <= 64) {
                int32_t r = 0;
                for (int32_t k = 0; k < L; ++k) r += __builtin_amdgcn_readlane(x[j], k) < x[j];
                if (lane < L) g.inc[b[j] + r] = x[j];
            } else if (lane == 0) {
                heap_sort(g.inc + b[j], L);
            }
        }
    }
}

// Global-memory views of the item's arrays: pointers read from the item table
// are generic; cast, their loads are plain global loads.
typedef __attribute__((address_space(1))) const int32_t g_i32;
typedef __attribute__((address_space(1))) const float g_f32;

// Eight lanes per vertex (kGatherLanes): lane k of the vertex's group sums
// incidences k, k + 8, k + 16, ... of its (sorted) list, then the eight
// partial sums are combined by a fixed butterfly; the order of every addition
// is fixed by the incidence list alone, so the result does not depend on the
// launch.

template <int DIM>
__device__ __forceinline__ void gather_vertex(const GatherItem &it, int64_t v, int k, bool live)
{
    constexpr int NV = DIM + 1, NJ = DIM * DIM;
    const g_i32 *ptr = (const g_i32 *)it.ptr;
    const g_i32 *inc = (const g_i32 *)it.inc;
    const g_f32 *jbar = (const g_f32 *)it.jbar;
    float s[DIM] = {};
    int32_t b = 0, e = 0;
    if (live) {
        b = ptr[v];
        e = ptr[v + 1];
    }
    // up to 4 of the lane's incidences per step: indices, then J-bar rows,
    // loaded together
    constexpr int U = 4;
    for (int32_t j0 = b + k; j0 < e; j0 += U * kGatherLanes) {
        int32_t idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t j = j0 + u * kGatherLanes;
            idx[u] = j < e ? inc[j] : -1;
        }
        float Jv[U][NJ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const g_f32 *J = jbar + int64_t(idx[u] >= 0 ? idx[u] / NV : 0) * NJ;
#pragma unroll
            for (int q = 0; q < NJ; ++q) Jv[u][q] = J[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (idx[u] < 0) break;
            const int a = idx[u] % NV;
#pragma unroll
            for (int al = 0; al < DIM; ++al) {
                // column a - 1 of J-bar for a > 0, minus the row sum for a = 0
                // (selected without indexing the register array at run time)
                float c = 0.f;
#pragma unroll
                for (int m = 0; m < DIM; ++m) c += Jv[u][al * DIM + m];
                c = -c;
#pragma unroll
                for (int m = 0; m < DIM; ++m) c = (a == m + 1) ? Jv[u][al * DIM + m] : c;
                s[al] += c;
            }
        }
    }
#pragma unroll
    for (int off = 1; off < kGatherLanes; off <<= 1)
#pragma unroll
        for (int al = 0; al < DIM; ++al) s[al] += __shfl_xor(s[al], off, kGatherLanes);
    if (!live || k != 0 || b == e) return;
    float *X[3] = {it.dx, it.dy, it.dz};
#pragma unroll
    for (int al = 0; al < DIM; ++al) {
        if (it.atomic) unsafeAtomicAdd(X[al] + v, s[al]);
        else X[al][v] += s[al];
    }
}

// Each vertex is summed by kGatherLanes consecutive threads, so a 256-thread
// workgroup takes kGatherVerts consecutive vertices of one item.  Workgroups
// are dispatched round-robin over the 8 XCDs; the workgroups of XCD x
// (blockIdx % 8 == x) take, item after item, the x-th eighth of each item's
// vertex blocks: every XCD gets the same share of every mesh (balanced work)
// and a contiguous vertex range of it, so the J-bar rows that neighbouring
// vertices share are re-read from that XCD's L2.  xoff[x][j] (host-built) is
// the number of XCD x's workgroups before item j; workgroups past
// xoff[x][n_items] have nothing to do.
__global__ __launch_bounds__(256) void vertex_gather_kernel(const GatherItem *items, int n_items,
                                                            const int32_t *xoff)
{
    const int x = int(blockIdx.x % 8);
    const int32_t i = int32_t(blockIdx.x / 8);
    const int32_t *o = xoff + int64_t(x) * (n_items + 1);
    if (i >= o[n_items]) return;                 // workgroup-uniform
    int lo = 0, hi = n_items - 1;                // last item j with o[j] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (o[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const GatherItem &it = items[lo];
    const int64_t blk = gather_slice_begin(it.n_vertices, x) + (i - o[lo]);
    const int64_t v = blk * kGatherVerts + threadIdx.x / kGatherLanes;
    const int k = int(threadIdx.x % kGatherLanes);
    const bool live = v < it.n_vertices;
    if (it.dim == 3) gather_vertex<3>(it, v, k, live);
    else gather_vertex<2>(it, v, k, live);
}

// The same gather for one item passed by value (single calls, which keep no
// device descriptor table): XCD x takes blocks gather_slice_begin(Nv, x) ..
// gather_slice_begin(Nv, x + 1) of the item; the grid is 8 x the largest slice.
__global__ __launch_bounds__(256) void vertex_gather_one_kernel(GatherItem it)
{
    const int x = int(blockIdx.x % 8);
    const int64_t blk = gather_slice_begin(it.n_vertices, x) + int64_t(blockIdx.x / 8);
    if (blk >= gather_slice_begin(it.n_vertices, x + 1)) return;   // workgroup-uniform
    const int64_t v = blk * kGatherVerts + threadIdx.x / kGatherLanes;
    const int k = int(threadIdx.x % kGatherLanes);
    const bool live = v < it.n_vertices;
    if (it.dim == 3) gather_vertex<3>(it, v, k, live);
    else gather_vertex<2>(it, v, k, live);
}

}  // namespace fei

// Heterogeneous batches (fei_batch_*): plan construction, graph capture and
// the autotuner over graph shapes.  Device code is in batch_dev.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "fei.h"
#include "host.h"
#include "params.h"
#include "shapes.h"

using namespace fei;
using namespace fei::host;

namespace {

struct Group {
    int form, dim;
    int off, n;         // range in the grouped item array
    int64_t tiles;
};

// One side (forward or adjoint) of a plan.
struct Side {
    std::vector<BatchItemDev> all;      // heaviest first, global tile numbering
    std::vector<BatchItemDev> grouped;  // by (form, dim) group, per-group tile numbering
    std::vector<Group> groups;
    int64_t tiles = 0;
    BatchItemDev *d_all = nullptr;
    BatchItemDev *d_grouped = nullptr;
    // adjoint with the vertex gather: the same descriptors with J-bar buffers
    std::vector<BatchItemDev> grouped_g;
    BatchItemDev *d_all_g = nullptr;
    BatchItemDev *d_grouped_g = nullptr;
    fei_batch_config cfg{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Vertex-gather state of the adjoint side, built on first use.
struct Gather {
    bool ready = false;
    std::vector<void *> bufs;           // device allocations owned by the plan
    GatherItem *d_items = nullptr;
    int32_t *d_xoff = nullptr;          // [8][n_items + 1] workgroups of each XCD per item
    int64_t blocks_per_xcd = 0;
    int n_items = 0;
    int64_t n_total = 0;                // vertices over all items
    std::vector<int32_t> keys;          // caller's item index of each gather item
    std::vector<GatherItem> host_items; // host copy of the gather descriptors
    std::vector<int64_t> n_elements;    // elements of each gather item
};

double item_bytes(const fei_batch_item &it)
{
    const int n = local_size(it.form, it.mesh.dim);
    const double per = 4.0 * (it.mesh.dim + 1) + (it.form == FEI_ELASTIC_P1 ? 8.0 : 0.0) + 4.0 * n * n;
    return per * double(it.mesh.n_elements) + 4.0 * it.mesh.dim * double(it.mesh.n_vertices);
}

int64_t tiles_of(int64_t E) { return (E + 255) / 256; }

}  // namespace

struct fei_batch {
    int device = 0;
    int n_cu = 0;
    int precision = 0;
    Side side[2];
    Gather gather;
    int32_t *d_counter = nullptr;  // [0, 8) forward, [8, 16) adjoint work counters
    hipStream_t cap = nullptr;
    hipStream_t branch[6] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[6] = {};
};

namespace {

int upload(const std::vector<BatchItemDev> &v, BatchItemDev **dst)
{
    if (v.empty()) return FEI_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), v.size() * sizeof(BatchItemDev));
    if (e != hipSuccess) return fail(FEI_ENOMEM, "batch descriptors: %s", hipGetErrorString(e));
    e = hipMemcpy(*dst, v.data(), v.size() * sizeof(BatchItemDev), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch descriptors upload");
    return FEI_OK;
}

// Orders a side heaviest first (globally and within groups) and numbers tiles.
void layout(Side &sd, std::vector<std::pair<double, BatchItemDev>> items)
{
    std::stable_sort(items.begin(), items.end(),
                     [](const auto &a, const auto &b) { return a.first > b.first; });
    int64_t t = 0;
    for (auto &it : items) {
        BatchItemDev d = it.second;
        d.tile_begin = t;
        t += tiles_of(d.fp.m.n_elements);
        sd.all.push_back(d);
    }
    sd.tiles = t;
    // groups by (form, dim), heaviest group first
    std::vector<std::pair<double, int>> keys;
    for (auto &it : items) {
        const int key = it.second.form * 4 + it.second.dim;
        auto f = std::find_if(keys.begin(), keys.end(), [&](auto &k) { return k.second == key; });
        if (f == keys.end()) keys.push_back({it.first, key});
        else f->first += it.first;
    }
    std::stable_sort(keys.begin(), keys.end(), [](auto &a, auto &b) { return a.first > b.first; });
    for (auto &k : keys) {
        Group g{k.second / 4, k.second % 4, int(sd.grouped.size()), 0, 0};
        for (auto &it : items) {
            if (it.second.form * 4 + it.second.dim != k.second) continue;
            BatchItemDev d = it.second;
            d.tile_begin = g.tiles;
            g.tiles += tiles_of(d.fp.m.n_elements);
            sd.grouped.push_back(d);
            ++g.n;
        }
        sd.groups.push_back(g);
    }
}

// Enqueues one run of a side with configuration c on stream s.
// (with c.gather on the adjoint side: J-bar per element, then the vertex gather)
hipError_t enqueue(fei_batch *b, int adj, const fei_batch_config &c, hipStream_t s)
{
    Side &sd = b->side[adj];
    const int prec = adj ? int(P_FP32) : b->precision;
    if (sd.tiles == 0) return hipSuccess;
    const bool gather = adj && c.gather;
    if (gather && !b->gather.ready) return hipErrorInvalidValue;
    const BatchItemDev *all = gather ? sd.d_all_g : sd.d_all;
    const BatchItemDev *grouped = gather ? sd.d_grouped_g : sd.d_grouped;
    hipError_t e = hipSuccess;
    if (c.mode == 0) {
        BatchLaunch L{all, int32_t(sd.all.size()), c.tiles_per_pop, sd.tiles,
                      b->d_counter + kBatchCounters * adj};
        if ((e = launch_batch_reset(L.counter, s)) != hipSuccess) return e;
        if ((e = launch_batch(adj != 0, prec, c.variant, L, c.workgroups, s)) != hipSuccess) return e;
    } else {
        // one group's kernels on stream gs
        auto run_group = [&](const Group &G, hipStream_t gs) -> hipError_t {
            hipError_t r = hipSuccess;
            if (c.mode == 2 || (adj && G.n == 1)) {
                // the single-mesh kernels, one launch per item of the group in
                // turn (a group of one mesh always runs the adjoint this way:
                // the scatter form's persistent pipelined kernel, or the gather
                // form's kernel without the group's item lookup)
                for (int k = 0; k < G.n; ++k) {
                    const BatchItemDev &d = gather ? sd.grouped_g[G.off + k] : sd.grouped[G.off + k];
                    const Variant v{d.form, d.dim, 0, prec, 0, gather ? 1 : 0};
                    if (adj) {
                        const AdjLauncher run = find_adjoint(v);
                        if (!run) return hipErrorInvalidValue;
                        if ((r = run(d.ap, gs)) != hipSuccess) return r;
                    } else {
                        const FwdLauncher run = find_forward(v);
                        if (!run) return hipErrorInvalidValue;
                        if ((r = run(d.fp, gs)) != hipSuccess) return r;
                    }
                }
                return r;
            }
            BatchLaunch L{grouped + G.off, G.n, 1, G.tiles, nullptr};
            return launch_batch_group(adj != 0, gather, G.form, G.dim, prec, c.variant, L, gs);
        };
        if (c.mode == 3) {
            // the groups one after another on the caller's stream: each kernel
            // has the whole GPU while it runs
            for (const Group &G : sd.groups)
                if ((e = run_group(G, s)) != hipSuccess) return e;
        } else {
            if ((e = hipEventRecord(b->fork, s)) != hipSuccess) return e;
            for (size_t g = 0; g < sd.groups.size(); ++g) {
                hipStream_t bs = b->branch[g];
                if ((e = hipStreamWaitEvent(bs, b->fork, 0)) != hipSuccess) return e;
                if ((e = run_group(sd.groups[g], bs)) != hipSuccess) return e;
                if ((e = hipEventRecord(b->join[g], bs)) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(s, b->join[g], 0)) != hipSuccess) return e;
            }
        }
    }
    if (gather)
        e = launch_vertex_gather(b->gather.d_items, b->gather.n_items, b->gather.d_xoff,
                                 b->gather.blocks_per_xcd, s);
    return e;
}

// Builds the vertex gather of the adjoint side: per item the vertex-to-element
// incidence of its mesh and a J-bar buffer, the descriptor copies that point
// at those buffers, and the gather table.  Reads the items' connectivity after
// synchronizing the device.
int ensure_gather(fei_batch *b)
{
    Gather &G = b->gather;
    if (G.ready) return FEI_OK;
    Side &sd = b->side[1];
    auto alloc = [&](size_t bytes, void **p) -> int {
        hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 4);
        if (e != hipSuccess) return fail(FEI_ENOMEM, "vertex gather buffers: %s", hipGetErrorString(e));
        G.bufs.push_back(*p);
        return FEI_OK;
    };
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronize before the incidence build");
    std::vector<GatherItem> items;
    std::vector<std::pair<int32_t, float *>> jbar_of;   // item key -> J-bar buffer
    std::vector<void *> scratch;
    int rc = FEI_OK;
    for (const BatchItemDev &d : sd.all) {
        const int nv = d.dim + 1;
        const int64_t E = d.ap.m.n_elements, Nv = d.ap.m.n_vertices;
        if (E * nv > int64_t(INT32_MAX))
            return fail(FEI_EUNSUPPORTED, "vertex gather needs (dim+1) * n_elements < 2^31");
        int32_t *ptr = nullptr, *inc = nullptr, *cursor = nullptr;
        float *jbar = nullptr;
        if ((rc = alloc(size_t(Nv + 1) * 4, reinterpret_cast<void **>(&ptr))) ||
            (rc = alloc(size_t(E) * nv * 4, reinterpret_cast<void **>(&inc))) ||
            (rc = alloc(size_t(E) * d.dim * d.dim * 4, reinterpret_cast<void **>(&jbar))))
            return rc;
        if ((e = hipMalloc(reinterpret_cast<void **>(&cursor), size_t(Nv > 0 ? Nv : 1) * 4)) != hipSuccess)
            return fail(FEI_ENOMEM, "incidence scratch: %s", hipGetErrorString(e));
        scratch.push_back(cursor);
        Incidence inc_g{d.ap.m.conn, E, Nv, nv, ptr, inc, cursor};
        if ((e = launch_incidence_build(inc_g, b->cap)) != hipSuccess) break;
        GatherItem gi{};
        gi.ptr = ptr;
        gi.inc = inc;
        gi.jbar = jbar;
        gi.dx = d.ap.dx;
        gi.dy = d.ap.dy;
        gi.dz = d.ap.dz;
        gi.v_begin = G.n_total;
        gi.n_vertices = Nv;
        gi.dim = d.dim;
        gi.atomic = 0;
        items.push_back(gi);
        G.keys.push_back(d.key);
        G.n_elements.push_back(E);
        jbar_of.push_back({d.key, jbar});
        G.n_total += Nv;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->cap);
    for (void *p : scratch) hipFree(p);
    if (e != hipSuccess) return hip_fail(e, "incidence build");
    // items whose gradient arrays overlap another item's accumulate atomically
    auto overlaps = [](const GatherItem &a, const GatherItem &c) {
        const float *pa[3] = {a.dx, a.dy, a.dz}, *pc[3] = {c.dx, c.dy, c.dz};
        for (int i = 0; i < a.dim; ++i)
            for (int j = 0; j < c.dim; ++j)
                if (pa[i] < pc[j] + c.n_vertices && pc[j] < pa[i] + a.n_vertices) return true;
        return false;
    };
    for (size_t i = 0; i < items.size(); ++i)
        for (size_t j = 0; j < items.size(); ++j)
            if (i != j && overlaps(items[i], items[j])) items[i].atomic = 1;
    auto with_jbar = [&](std::vector<BatchItemDev> v) {
        for (BatchItemDev &d : v)
            for (auto &kj : jbar_of)
                if (kj.first == d.key) d.ap.jbar = kj.second;
        return v;
    };
    sd.grouped_g = with_jbar(sd.grouped);
    if ((rc = upload(with_jbar(sd.all), &sd.d_all_g)) || (rc = upload(sd.grouped_g, &sd.d_grouped_g)))
        return rc;
    G.n_items = int(items.size());
    G.host_items = items;
    if (!items.empty()) {
        // per XCD, the prefix sums of its share of each item's workgroups
        const size_t ni = items.size();
        std::vector<int32_t> xoff(8 * (ni + 1));
        int64_t most = 0;
        for (int x = 0; x < 8; ++x) {
            int64_t acc = 0;
            for (size_t j = 0; j < ni; ++j) {
                xoff[x * (ni + 1) + j] = int32_t(acc);
                acc += gather_slice_begin(items[j].n_vertices, x + 1) -
                       gather_slice_begin(items[j].n_vertices, x);
                if (acc > INT32_MAX) return fail(FEI_EUNSUPPORTED, "vertex gather: too many vertices");
            }
            xoff[x * (ni + 1) + ni] = int32_t(acc);
            most = acc > most ? acc : most;
        }
        G.blocks_per_xcd = most;
        if ((rc = alloc(ni * sizeof(GatherItem), reinterpret_cast<void **>(&G.d_items))) ||
            (rc = alloc(xoff.size() * 4, reinterpret_cast<void **>(&G.d_xoff))))
            return rc;
        e = hipMemcpy(G.d_items, items.data(), ni * sizeof(GatherItem), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(G.d_xoff, xoff.data(), xoff.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "gather table upload");
    }
    G.ready = true;
    return FEI_OK;
}

void drop_graph(Side &sd)
{
    if (sd.exec) hipGraphExecDestroy(sd.exec);
    if (sd.graph) hipGraphDestroy(sd.graph);
    sd.exec = nullptr;
    sd.graph = nullptr;
}

int build_graph(fei_batch *b, int adj)
{
    Side &sd = b->side[adj];
    drop_graph(sd);
    if (sd.tiles == 0) return FEI_OK;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = enqueue(b, adj, sd.cfg, b->cap);
    e = hipStreamEndCapture(b->cap, &sd.graph);
    if (le != hipSuccess) {
        drop_graph(sd);
        return hip_fail(le, "batch capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&sd.exec, sd.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(sd);
        return hip_fail(e, "hipGraphInstantiate");
    }
    return FEI_OK;
}

void release(fei_batch *b)
{
    for (Side &sd : b->side) {
        drop_graph(sd);
        if (sd.d_all) hipFree(sd.d_all);
        if (sd.d_grouped) hipFree(sd.d_grouped);
        if (sd.d_all_g) hipFree(sd.d_all_g);
        if (sd.d_grouped_g) hipFree(sd.d_grouped_g);
    }
    for (void *p : b->gather.bufs) hipFree(p);
    if (b->d_counter) hipFree(b->d_counter);
    for (hipStream_t s : b->branch)
        if (s) hipStreamDestroy(s);
    for (hipEvent_t ev : b->join)
        if (ev) hipEventDestroy(ev);
    if (b->fork) hipEventDestroy(b->fork);
    if (b->cap) hipStreamDestroy(b->cap);
    delete b;
}

int check_item(const fei_batch_item &it, int k, MeshView &mv)
{
    int rc = check_mesh(&it.mesh, mv);
    if (rc) return fail(rc, "item %d: %s", k, fei_last_error());
    if (!valid_form(it.form)) return fail(FEI_EINVAL, "item %d: unknown form %d", k, it.form);
    if (it.mesh.coord_dtype != FEI_F32)
        return fail(FEI_EUNSUPPORTED, "item %d: batches take FP32 coordinates", k);
    if ((rc = check_coeffs(it.form, it.mu, it.lam, it.mesh.n_elements)))
        return fail(rc, "item %d: %s", k, fei_last_error());
    if (it.mesh.n_elements > 0 && (!it.A || !aligned(it.A, 16)))
        return fail(FEI_EINVAL, "item %d: A NULL or not 16-byte aligned", k);
    if (it.dA) {
        if (!aligned(it.dA, 16)) return fail(FEI_EINVAL, "item %d: dA not 16-byte aligned", k);
        if (!it.dx || !it.dy || (it.mesh.dim == 3 && !it.dz))
            return fail(FEI_EINVAL, "item %d: adjoint needs dx, dy (, dz)", k);
        if (it.form != FEI_ELASTIC_P1 && (it.dmu || it.dlam))
            return fail(FEI_EINVAL, "item %d: dmu/dlam only for elasticity", k);
    }
    return FEI_OK;
}

}  // namespace

extern "C" {

int fei_batch_create(const fei_batch_item *items, int n_items, const fei_options *opt,
                     fei_batch **out)
{
    if (!out) return fail(FEI_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(FEI_EINVAL, "bad item list");
    fei_options o = opt ? *opt : defaults();
    int rc = check_options(o);
    if (rc) return rc;
    const float tau2 = tau2_of(o.tau);

    std::vector<std::pair<double, BatchItemDev>> fwd, adj;
    int64_t total = 0;
    for (int k = 0; k < n_items; ++k) {
        const fei_batch_item &it = items[k];
        MeshView mv;
        if ((rc = check_item(it, k, mv))) return rc;
        if (it.mesh.n_elements == 0) continue;
        // each item rounds up to whole 256-element tiles; one launch covers them all
        total += (it.mesh.n_elements + 255) / 256 * 256;
        if (total > kMaxElements)
            return fail(FEI_EINVAL, "the batch exceeds %lld elements in 256-element tiles",
                        (long long)kMaxElements);
        BatchItemDev d;
        std::memset(&d, 0, sizeof d);
        d.form = it.form;
        d.dim = it.mesh.dim;
        d.key = k;
        d.fp.m = mv;
        d.fp.mu = it.mu;
        d.fp.lam = it.lam;
        d.fp.A = it.A;
        d.fp.counters = o.counters;
        d.fp.tau2 = tau2;
        d.ap.m = mv;
        d.ap.mu = it.mu;
        d.ap.lam = it.lam;
        d.ap.dA = it.dA;
        d.ap.dx = it.dx;
        d.ap.dy = it.dy;
        d.ap.dz = it.mesh.dim == 3 ? it.dz : nullptr;
        d.ap.dmu = it.dmu;
        d.ap.dlam = it.dlam;
        d.ap.counters = o.counters;
        d.ap.tau2 = tau2;
        const double w = item_bytes(it);
        fwd.push_back({w, d});
        if (it.dA) adj.push_back({w, d});
    }

    fei_batch *b = new (std::nothrow) fei_batch();
    if (!b) return fail(FEI_ENOMEM, "plan allocation");
    b->precision = o.precision;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "device query");
    }
    layout(b->side[0], fwd);
    layout(b->side[1], adj);
    for (int s = 0; s < 2; ++s) {
        Side &sd = b->side[s];
        if ((rc = upload(sd.all, &sd.d_all)) || (rc = upload(sd.grouped, &sd.d_grouped))) {
            release(b);
            return rc;
        }
        sd.cfg.mode = 1;
        sd.cfg.variant = 0;
        sd.cfg.workgroups = 2 * b->n_cu;
        sd.cfg.tiles_per_pop = 1;
        sd.cfg.ms = 0.f;
    }
    if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_counter), 2 * kBatchCounters * sizeof(int32_t))) != hipSuccess) {
        release(b);
        return fail(FEI_ENOMEM, "work counter: %s", hipGetErrorString(e));
    }
    if ((e = hipMemset(b->d_counter, 0, 2 * kBatchCounters * sizeof(int32_t))) == hipSuccess &&
        (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) == hipSuccess &&
        (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) == hipSuccess) {
        for (int g = 0; g < 6 && e == hipSuccess; ++g) {
            e = hipStreamCreateWithFlags(&b->branch[g], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[g], hipEventDisableTiming);
        }
    }
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "plan streams/events");
    }
    for (int s = 0; s < 2; ++s) {
        if ((rc = build_graph(b, s))) {
            release(b);
            return rc;
        }
    }
    *out = b;
    return FEI_OK;
}

int fei_batch_run(fei_batch *b, void *stream)
{
    if (!b) return fail(FEI_EINVAL, "plan is NULL");
    if (!b->side[0].exec) return FEI_OK;  // no elements
    hipError_t e = hipGraphLaunch(b->side[0].exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FEI_OK : hip_fail(e, "hipGraphLaunch");
}

int fei_batch_run_adjoint(fei_batch *b, void *stream)
{
    if (!b) return fail(FEI_EINVAL, "plan is NULL");
    if (!b->side[1].exec) return FEI_OK;  // no adjoint items
    hipError_t e = hipGraphLaunch(b->side[1].exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FEI_OK : hip_fail(e, "hipGraphLaunch");
}

int fei_batch_get_config(const fei_batch *b, int adjoint, fei_batch_config *out)
{
    if (!b || !out || (adjoint != 0 && adjoint != 1)) return fail(FEI_EINVAL, "bad argument");
    *out = b->side[adjoint].cfg;
    return FEI_OK;
}

int fei_batch_tune(fei_batch *b, int adjoint, void *stream, fei_batch_config *chosen)
{
    if (!b || (adjoint != 0 && adjoint != 1)) return fail(FEI_EINVAL, "bad argument");
    Side &sd = b->side[adjoint];
    if (sd.tiles == 0) {
        if (chosen) *chosen = sd.cfg;
        return FEI_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (adjoint) {
        int rc = ensure_gather(b);
        if (rc) return rc;
    }
    std::vector<fei_batch_config> cand;
    for (int gather = 0; gather <= adjoint; ++gather)
        for (int var = 0; var < 2; ++var) {
            fei_batch_config c{};
            c.mode = 1;
            c.variant = var;
            c.workgroups = 0;
            c.tiles_per_pop = 1;
            c.gather = gather;
            cand.push_back(c);
            fei_batch_config m3 = c;
            m3.mode = 3;
            cand.push_back(m3);
            if (var == 0) {
                fei_batch_config m2 = c;
                m2.mode = 2;
                cand.push_back(m2);
            }
            for (int wg : {1, 2, 4})
                for (int pop : {1, 4}) {
                    fei_batch_config p{};
                    p.mode = 0;
                    p.variant = var;
                    p.workgroups = wg * b->n_cu;
                    p.tiles_per_pop = pop;
                    p.gather = gather;
                    cand.push_back(p);
                }
        }
    hipEvent_t t0, t1;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    // every candidate is timed as what run() launches: its instantiated graph
    int best = -1;
    float best_ms = 0.f;
    for (size_t k = 0; k < cand.size() && e == hipSuccess; ++k) {
        sd.cfg = cand[k];
        if (build_graph(b, adjoint) != FEI_OK || !sd.exec) continue;
        if (hipGraphLaunch(sd.exec, s) != hipSuccess) continue;  // warm-up
        float times[3];
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            e = hipEventRecord(t0, s);
            if (e == hipSuccess) e = hipGraphLaunch(sd.exec, s);
            if (e == hipSuccess) e = hipEventRecord(t1, s);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            if (e == hipSuccess) e = hipEventElapsedTime(&times[r], t0, t1);
        }
        if (e != hipSuccess) break;
        std::sort(times, times + 3);
        cand[k].ms = times[1];
        if (best < 0 || times[1] < best_ms) {
            best = int(k);
            best_ms = times[1];
        }
    }
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "tuning run");
    if (best < 0) return fail(FEI_EDEVICE, "no batch configuration could be launched");
    sd.cfg = cand[best];
    int rc = build_graph(b, adjoint);
    if (rc) return rc;
    if (chosen) *chosen = sd.cfg;
    return FEI_OK;
}

int fei_batch_set_config(fei_batch *b, int adjoint, const fei_batch_config *cfg)
{
    if (!b || !cfg || (adjoint != 0 && adjoint != 1)) return fail(FEI_EINVAL, "bad argument");
    if ((cfg->mode < 0 || cfg->mode > 3) || (cfg->variant != 0 && cfg->variant != 1))
        return fail(FEI_EINVAL, "mode must be 0 to 3 and variant 0 or 1");
    if (cfg->mode == 0 && (cfg->workgroups < 1 || cfg->tiles_per_pop < 1))
        return fail(FEI_EINVAL, "mode 0 needs workgroups >= 1 and tiles_per_pop >= 1");
    if (cfg->gather != 0 && cfg->gather != 1) return fail(FEI_EINVAL, "gather must be 0 or 1");
    if (cfg->gather && !adjoint) return fail(FEI_EINVAL, "gather applies to the adjoint only");
    for (int r : cfg->reserved)
        if (r) return fail(FEI_EINVAL, "reserved fields must be zero");
    if (cfg->gather) {
        int rc = ensure_gather(b);
        if (rc) return rc;
    }
    b->side[adjoint].cfg = *cfg;
    return build_graph(b, adjoint);
}

int fei_batch_copy_incidence(const fei_batch *b, int item, int32_t *ptr, int32_t *inc,
                             void *stream)
{
    if (!b || !ptr || !inc) return fail(FEI_EINVAL, "bad argument");
    const Gather &G = b->gather;
    if (!G.ready) return fail(FEI_EINVAL, "the plan has not built its vertex gather");
    for (size_t j = 0; j < G.keys.size(); ++j) {
        if (G.keys[j] != item) continue;
        const GatherItem &gi = G.host_items[j];
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t nptr = size_t(gi.n_vertices + 1) * 4;
        const size_t ninc = size_t(G.n_elements[j]) * size_t(gi.dim + 1) * 4;
        hipError_t e = hipMemcpyAsync(ptr, gi.ptr, nptr, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(inc, gi.inc, ninc, hipMemcpyDeviceToDevice, s);
        return e == hipSuccess ? FEI_OK : hip_fail(e, "incidence copy");
    }
    return fail(FEI_EINVAL, "item %d has no vertex gather in this plan", item);
}

int fei_batch_destroy(fei_batch *b)
{
    if (b) release(b);
    return FEI_OK;
}

}  // extern "C"

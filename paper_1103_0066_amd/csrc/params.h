// Kernel parameter blocks and launcher declarations shared by the host layer
// (api.cpp) and the device code (kernels.hip).  Plain structs, no HIP types
// beyond hipStream_t / hipError_t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fei {

struct MeshView {
    const void *x, *y, *z;     // SoA coordinates (float or double)
    const int32_t *conn;       // [E][dim+1]
    int64_t n_elements;
    int64_t n_vertices;
};

struct FwdParams {
    MeshView m;
    const float *mu, *lam;     // elasticity only
    const float *w;            // forms with a P1 coefficient: [n_vertices]
    float *A;                  // [E][n][n]
    int32_t *counters;         // optional [2]
    float tau2;                // squared quality threshold; < 0 forces FP64
};

struct AdjParams {
    MeshView m;
    const float *mu, *lam;
    const float *dA;           // [E][n][n]
    float *dx, *dy, *dz;       // [n_vertices], accumulated
    float *dmu, *dlam;         // [E] or NULL
    int32_t *counters;
    float tau2;
    float *jbar;               // [E][dim][dim]: J-bar per element instead of the
                               // vertex scatter (gathered per vertex later); NULL: scatter
};

// Kernel selection key.
struct Variant {
    int form;       // fei::Form
    int dim;        // 2 or 3
    int coord_f64;  // 0/1
    int precision;  // fei_precision
    int rows;       // fei_options.store_rows: 0 default, -1 direct, R > 0 staged
    int gather;     // adjoint: 1 writes J-bar (AdjParams.jbar) and has no vertex scatter
    int block;      // forward: elements per workgroup (0 = 256)
};

using FwdLauncher = hipError_t (*)(const FwdParams &, hipStream_t);
using AdjLauncher = hipError_t (*)(const AdjParams &, hipStream_t);

// Returns NULL when no kernel exists for the variant.
FwdLauncher find_forward(const Variant &v);
// Forms with a P1 coefficient (v.form WLAP1 or WLAP2; FP32 contraction).
FwdLauncher find_forward_coefficient(const Variant &v);
AdjLauncher find_adjoint(const Variant &v);

// Heterogeneous batch: one work item per (mesh, form), laid out for the
// persistent batch kernels.
struct BatchItemDev {
    int32_t form;        // fei::Form
    int32_t dim;
    int32_t key;         // index of the item in the caller's list (host bookkeeping)
    int32_t pad_;
    int64_t tile_begin;  // first global tile (256 elements) of this item
    FwdParams fp;
    AdjParams ap;
};

// Work counters of the persistent batch kernel: one per contiguous range of
// tiles (one range per XCD).
constexpr int kBatchCounters = 8;

struct BatchLaunch {
    const BatchItemDev *items;  // device, sorted by tile_begin
    int32_t n_items;
    int32_t tiles_per_pop;
    int64_t n_tiles;
    int32_t *counter;           // device work counters [kBatchCounters], reset by launch_batch_reset
};

// Dynamic LDS bytes of a batch kernel variant; 0 if the variant does not exist.
size_t batch_lds_bytes(bool adjoint, int precision, int variant);
hipError_t launch_batch(bool adjoint, int precision, int variant, const BatchLaunch &b, int grid,
                        hipStream_t s);
hipError_t launch_batch_reset(int32_t *counter, hipStream_t s);
// One (form, dim) group of a batch: b.items holds only that group's items and
// b.n_tiles its tiles (one workgroup per tile).
hipError_t launch_batch_group(bool adjoint, bool gather, int form, int dim, int precision,
                              int variant, const BatchLaunch &b, hipStream_t s);

// Device-side connectivity check: writes the count of entries outside
// [0, n_vertices) into *n_bad_dev (int64, zeroed by the kernel's caller).
// Vertex-to-element incidence of one mesh (CSR, rows = vertices, entries
// e * (dim + 1) + a in increasing order) and the per-vertex gather of J-bar.
struct Incidence {
    const int32_t *conn;       // [E][nv]
    int64_t n_elements;
    int64_t n_vertices;
    int32_t nv;                // dim + 1
    int32_t *ptr;              // [n_vertices + 1]
    int32_t *inc;              // [n_elements * nv]
    int32_t *cursor;           // [n_vertices] scratch
};
// Builds ptr and inc on stream s (entries with a vertex outside [0, n_vertices)
// are left out).
hipError_t launch_incidence_build(const Incidence &g, hipStream_t s);

struct GatherItem {
    const int32_t *ptr, *inc;  // incidence of the item's mesh
    const float *jbar;         // [E][dim][dim]
    float *dx, *dy, *dz;       // accumulated
    int64_t v_begin;           // first global vertex of the item
    int64_t n_vertices;
    int32_t dim;
    int32_t atomic;            // 1 if another item accumulates into the same arrays
};
// Vertex gather geometry, shared by the kernel and the host that builds its
// XCD table: kGatherLanes threads per vertex, kGatherVerts vertices per
// 256-thread workgroup; XCD x takes the item's workgroup blocks from
// gather_slice_begin(Nv, x) to gather_slice_begin(Nv, x + 1).
constexpr int kGatherLanes = 8;
constexpr int kGatherVerts = 256 / kGatherLanes;
__host__ __device__ inline int64_t gather_slice_begin(int64_t n_vertices, int x)
{
    const int64_t nb = (n_vertices + kGatherVerts - 1) / kGatherVerts;
    return x * nb / 8;
}

// Eight threads per vertex of every item: dx[v] += sum over the vertex's
// incidences, combined in an order fixed by the sorted incidence list.
// xoff: int32[8][n_items + 1], per XCD the prefix sums of its workgroups per
// item (gather_xcd_offsets); blocks_per_xcd: the largest of its last column.
hipError_t launch_vertex_gather(const GatherItem *items, int n_items, const int32_t *xoff,
                                int64_t blocks_per_xcd, hipStream_t s);
// The gather of one item (single calls): no device tables needed.
hipError_t launch_vertex_gather_one(const GatherItem &it, hipStream_t s);

hipError_t launch_validate(const MeshView &m, int dim, unsigned long long *n_bad_dev,
                           hipStream_t s);

// Isoparametric P2 Laplacian (quadratic geometry): m.conn is [E][NB] (the
// element's P2 nodes), m.x/y/z the node coordinates (FP32).
hipError_t launch_iso(int dim, const FwdParams &p, hipStream_t s);

// Runtime-described bilinear forms (form front end): the geometric tensor
// G = |J| That^T C_e That from the operator tables W and per-element
// coefficients, contracted with the reference tensor Khat.
constexpr int kFormMaxCoef = 4;
struct FormParams {
    MeshView m;
    const float *coef;         // [n_coef][E] per-element coefficients, or NULL
    int32_t n_coef;            // 0 .. kFormMaxCoef
    const float *W;            // [n_coef + 1][M][M], M = (dim + 1) * ncomp (uniform)
    const float *K;            // [NB][NB][dim + 1][dim + 1] (uniform), scaled by 1 / kscale
    float kscale;              // Khat = K * kscale (folded into |det J|)
    float *A;                  // [E][n][n]
    int32_t *counters;
    float tau2;
};
// Launches the form kernel of (dim, degree, ncomp, symmetric, no value term);
// hipErrorInvalidValue if none exists.
hipError_t launch_form(int dim, int degree, int ncomp, bool sym, bool noval, const FormParams &p,
                       hipStream_t s);

// Fused global assembly (P1 forms): rows of the global matrix gathered by
// waves, one host-built chunk of rows per wave.
struct AsmParams {
    MeshView m;
    const float *mu, *lam;           // elasticity only
    const int32_t *ptr, *inc;        // per row: its incidences in steps of kAsmLanes (-1 pads)
    const int32_t *slots;            // per entry: its element's vertices' slots in the row, bytes
    const int32_t *rowptr, *colidx;  // the pattern: CSR over vertices, sorted columns
    const int32_t *chunks;           // [n_chunks + 1]: first row of each wave's chunk
    int64_t n_chunks;
    float *values;                   // [nnz][NC][NC]
    int32_t *counters;
    float tau2;
};
// Rows (kAsmRows) and blocks (kAsmSlots) one chunk may hold.
int assemble_chunk_rows();
int assemble_chunk_slots();
int assemble_lanes();
hipError_t launch_assemble(int form, int dim, const AsmParams &p, hipStream_t s);

}  // namespace fei

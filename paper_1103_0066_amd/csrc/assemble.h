// Fused global assembly of P1 forms: the element matrices are summed straight
// into the values of the global sparse matrix (CSR over vertices, with
// NC x NC blocks: 1 x 1 for the Laplacian, dim x dim for elasticity), so the
// n x n element matrices are never written to memory.  This is the global
// portion of the computation that element integration feeds (Sec. 1), with
// the local portion, A_e = G_e : K (Sec. 3, eq. 1), computed on the fly.
//
// Rows are gathered, not scattered: one wave owns a contiguous range of rows
// (a host-built chunk whose blocks fit the wave's LDS accumulator) and walks
// their vertex-to-element incidences, 64 at a time, one lane per incidence
// (e, a).  The lane recomputes element e's geometric tensor (eq. 8 or its
// Lame analogue, FP64 for flagged elements, exactly as the forward), forms
// row block a of A_e and adds its n / NC blocks into the row's slots in LDS;
// the slot of column vertex conn[e][b] is found by binary search in the row's
// sorted column list.  No other wave touches the rows, so the sums need no
// global atomics, and the adds of a wave execute in program order (one LDS
// atomic instruction per block entry and local vertex b).  The finished rows
// leave as one contiguous run of values.
//
// For P1 the reference tensor factors, K^{ab}_{mu nu} = g_a,mu g_b,nu (eq. 7
// with constant barycentric gradients g), so row block a is
//   w[nu][c][d]     = sum_mu g_a,mu T^{(mu c),(nu d)}
//   A_{(a,c),(b,d)} = sum_nu g_b,nu w[nu][c][d],
// where the runtime a selects among the compile-time rows of T (g_0 = -1...-1,
// g_{m+1} = e_m): no per-lane branch, whatever the lanes' local vertices.
#pragma once

#include "fwd_fma.h"

namespace fei {

// Rows and slots a wave owns at most (the host cuts chunks to fit).
constexpr int kAsmSlots = 256;
constexpr int kAsmRows = 256;

template <int FORM, int DIM>
struct AsmShape {
    using T = Traits<FORM, DIM>;
    static constexpr int NC = T::NC;
    static constexpr int BS2 = NC * NC;                    // floats per block
    static constexpr int ACC = kAsmSlots * BS2;            // accumulator floats
    static constexpr int WAVE_BYTES = 4 * (ACC + kAsmSlots + kAsmRows + 1 + 3);
    static constexpr int LDS_BYTES = 4 * WAVE_BYTES;
};

// Slot of column vertex v in a row's sorted columns col[b0 .. b1); -1 if absent.
__device__ __forceinline__ int find_slot(const int *col, int b0, int b1, int v)
{
    int lo = b0, hi = b1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return (lo < b1 && col[lo] == v) ? lo : -1;
}

template <int FORM, int DIM>
__global__ __launch_bounds__(256) void assemble_kernel(AsmParams p)
{
    using T = Traits<FORM, DIM>;
    using SH = AsmShape<FORM, DIM>;
    constexpr int NV = DIM + 1, NC = SH::NC, BS2 = SH::BS2;
    static_assert(FORM != LAP2, "fused assembly is for P1 forms");
    __shared__ __attribute__((aligned(16))) unsigned char smem[SH::LDS_BYTES];

    const int lane = threadIdx.x & 63, wave = wave_id();
    const int64_t chunk = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
    if (chunk >= p.n_chunks) return;               // wave-uniform; no workgroup barrier below
    float *acc = reinterpret_cast<float *>(smem + wave * SH::WAVE_BYTES);
    int *col = reinterpret_cast<int *>(acc + SH::ACC);
    int *rp = col + kAsmSlots;

    const int32_t r0 = p.chunks[chunk], r1 = p.chunks[chunk + 1];
    const int nrows = r1 - r0;
    const int32_t s0 = p.rowptr[r0], s1 = p.rowptr[r1];
    const int nslot = s1 - s0;
    for (int k = lane; k <= nrows; k += 64) rp[k] = p.rowptr[r0 + k] - s0;
    for (int k = lane; k < nslot; k += 64) col[k] = p.colidx[s0 + k];
    for (int k = lane; k < nslot * BS2; k += 64) acc[k] = 0.f;
    wave_sync();

    const float *__restrict__ mu = p.mu;
    const float *__restrict__ lam = p.lam;
    const int32_t j0 = p.ptr[r0], j1 = p.ptr[r1];
    for (int32_t jb = j0; jb < j1; jb += 64) {
        const int32_t j = jb + lane;
        const bool live = j < j1;
        const int32_t ent = p.inc[live ? j : j0];
        const int64_t e = ent / NV;
        const int a = ent - int(e) * NV;
        // plain loads: every element is read once per vertex, by neighbouring rows
        int v[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = p.m.conn[e * NV + m];
        float xv[NV][DIM];
        gather<DIM>(p.m, v, xv);
        float me = 0.f, le = 0.f;
        if constexpr (FORM == ELA1) {
            me = mu[e];
            le = lam[e];
        }
        float Gf[T::G];
        bool singular = false;
        const bool flag = geometry<FORM, DIM>(xv, me, le, p.tau2, Gf, singular);
        // each element counted once: at its incidence with local vertex 0
        count_flags(p.counters, live && a == 0 && flag, live && a == 0 && singular);

        // row of this incidence and the slots of the element's vertices in it
        int local = 0;
#pragma unroll
        for (int m = 0; m < NV; ++m) local = (a == m) ? v[m] - r0 : local;
        const bool in_rows = live && local >= 0 && local < nrows;
        const int b0 = in_rows ? rp[local] : 0, b1 = in_rows ? rp[local + 1] : 0;
        int slot[NV];
#pragma unroll
        for (int b = 0; b < NV; ++b) slot[b] = find_slot(col, b0, b1, v[b]);

        // w[nu][c][d] = sum_mu g_a,mu T^{(mu c),(nu d)} (runtime a, compile-time T index)
        float w[DIM][NC][NC];
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < NC; ++d) {
                    float s = 0.f;
#pragma unroll
                    for (int m = 0; m < DIM; ++m) s += Gf[sym_index(T::GD, m * NC + c, nu * NC + d)];
                    float r = -s;
#pragma unroll
                    for (int m = 0; m < DIM; ++m)
                        r = (a == m + 1) ? Gf[sym_index(T::GD, m * NC + c, nu * NC + d)] : r;
                    w[nu][c][d] = r;
                }
        // blocks (a, b) = sum_nu g_b,nu w[nu], added into the row's slots
#pragma unroll
        for (int b = 0; b < NV; ++b) {
            const bool put = in_rows && slot[b] >= 0;
            float *dst = acc + (put ? slot[b] : 0) * BS2;
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < NC; ++d) {
                    float blk;
                    if (b == 0) {
                        float s = 0.f;
#pragma unroll
                        for (int nu = 0; nu < DIM; ++nu) s += w[nu][c][d];
                        blk = -s;
                    } else {
                        blk = w[b - 1][c][d];
                    }
                    if (put)
                        __hip_atomic_fetch_add(dst + c * NC + d, blk, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
        }
    }
    wave_sync();
    // the chunk's rows are one contiguous run of values
    float *out = p.values + int64_t(s0) * BS2;
    for (int k = lane; k < nslot * BS2; k += 64) out[k] = acc[k];
}

}  // namespace fei

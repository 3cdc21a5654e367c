// Fused global assembly of P1 forms: the element matrices are summed straight
// into the values of the global sparse matrix (CSR over vertices, with
// NC x NC blocks: 1 x 1 for the Laplacian, dim x dim for elasticity), so the
// n x n element matrices are never written to memory.  This is the global
// portion of the computation that element integration feeds (Sec. 1), with
// the local portion, A_e = G_e : K (Sec. 3, eq. 1), computed on the fly.
//
// Rows are gathered, not scattered, and every row has owners: a wave takes a
// contiguous range of up to kAsmRows rows (a host-built chunk whose blocks
// fit the wave's LDS accumulator), and the kAsmLanes lanes r, r + kAsmRows, ..
// own row r of it.  They walk the row's vertex-to-element incidences (e, a),
// lane k of the row taking incidences k, k + kAsmLanes, .., recomputing
// element e's geometric tensor (eq. 8 or its Lame
// analogue, FP64 for flagged elements, exactly as the forward), forming row
// block a of A_e and adding its n / NC blocks into the row's slots in LDS; the
// slot of column vertex conn[e][b] is found by binary search in the row's
// sorted column list.  The lanes of one part of the wave own distinct rows,
// so their adds touch distinct slots: the parts add in turn with plain LDS
// read-modify-writes, no atomics (LDS float atomics, where the lanes of a row
// collide on its slots, measured 6x slower), and every sum runs in the order
// of the row's incidence list, so every run gives the same bits.  The
// finished rows leave as one contiguous run of values.
//
#pragma once

#include "fwd_fma.h"

namespace fei {

// Rows and slots a wave owns at most (the host cuts chunks to fit), and the
// lanes per row.  Four lanes per row: 16 rows (240 slots of 3 x 3 blocks, the
// 15 of a Kuhn vertex each) keep four 4-wave workgroups per CU, and a row's 24
// incidences take 6 steps.
constexpr int kAsmLanes = 4;
constexpr int kAsmRows = 64 / kAsmLanes;
constexpr int kAsmSlots = 240;

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

    // this lane's row and its share (every kAsmLanes-th incidence) of the row's list
    const int part = lane / kAsmRows, local = lane % kAsmRows;
    const bool has_row = local < nrows;
    const int32_t row = r0 + (has_row ? local : 0);
    const int32_t jb = has_row ? p.ptr[row] + part : 0;
    const int32_t je = has_row ? p.ptr[row + 1] : 0;
    const int b0 = has_row ? rp[local] : 0, b1 = has_row ? rp[local + 1] : 0;
    // the wave steps through the longest share of its rows (je - jb >= 1 - kAsmLanes)
    int steps = has_row ? (je - jb + kAsmLanes - 1) / kAsmLanes : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) steps = max(steps, __shfl_xor(steps, off));

    const float *__restrict__ mu = p.mu;
    const float *__restrict__ lam = p.lam;
    for (int it = 0; it < steps; ++it) {
        const int32_t j = jb + kAsmLanes * it;
        const bool live = has_row && j < je;
        const int32_t ent = p.inc[live ? j : 0];
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

        int slot[NV];
#pragma unroll
        for (int b = 0; b < NV; ++b) slot[b] = live ? find_slot(col, b0, b1, v[b]) : -1;

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
        // blocks (a, b) = sum_nu g_b,nu w[nu], added into the row's slots by
        // one part of the wave after the other (a part's rows are distinct)
#pragma unroll
        for (int h = 0; h < kAsmLanes; ++h) {
            if (part == h) {
#pragma unroll
                for (int b = 0; b < NV; ++b) {
                    if (slot[b] < 0) continue;
                    float *dst = acc + slot[b] * BS2;
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
                            dst[c * NC + d] += blk;
                        }
                }
            }
            wave_sync();
        }
    }
    wave_sync();
    // the chunk's rows are one contiguous run of values
    float *out = p.values + int64_t(s0) * BS2;
    for (int k = lane; k < nslot * BS2; k += 64) out[k] = acc[k];
}

}  // namespace fei

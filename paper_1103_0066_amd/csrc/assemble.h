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
// own row r of it.  They walk the row's vertex-to-element incidences (e, a) in
// the plan's schedule, lane k of the row taking entries k, k + kAsmLanes, ..,
// recomputing element e's geometry (J, adj J, det J and the quality test, FP64
// for flagged elements, exactly as the forward) and forming row block a of
// A_e = G_e : K.  The row block is contracted in factored form: P1's K is rank
// one per vertex pair, K^{ab}_{mu nu} = g_a,mu g_b,nu (reference gradients), and
// G_e is a sum of products of adj J entries (eq. 8; the Lame analogue for
// elasticity), so contracting g_a into adj J first (beta = g_a^T adj J) leaves
// 27 products for the 3 x 3 x 3 row block of 3D elasticity instead of the 45
// entries of G_e and their contraction.  The schedule puts a row's incidences
// in steps of kAsmLanes whose elements share no vertex but the row's, so the
// off-diagonal blocks of one step land on distinct slots and the whole wave
// adds them into LDS at once with plain read-modify-writes (no atomics); the
// diagonal block, which every incidence of the row touches, is summed in the
// lanes' registers and added by the row's lanes in turn at the end.  The slot
// of column vertex conn[e][b] in the row's sorted column list comes with the
// schedule entry (one byte per vertex, computed by the plan).  Every sum runs in an order fixed by the plan, so every run
// gives the same bits.  The finished rows leave as one contiguous run of values.
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
static_assert(kAsmSlots <= 256, "a row's slots are addressed by one byte in the plan");

template <int FORM, int DIM>
struct AsmShape {
    using T = Traits<FORM, DIM>;
    static constexpr int NC = T::NC;
    static constexpr int BS2 = NC * NC;                    // floats per block
    static constexpr int ACC = kAsmSlots * BS2;            // accumulator floats
    static constexpr int WAVE_BYTES = 4 * (ACC + kAsmSlots);      // accumulator, columns
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

// w[nu][c][d] = sum_mu g_a,mu G^{(mu c),(nu d)} of one element from adj J and
// the weights of G (gf_weights): with beta = g_a^T adj J and m_nu = (adj J
// beta)_nu, the Laplacian's row is wa m_nu and elasticity's is
// wa (delta_cd m_nu + beta_d adj_nu,c) + wb beta_c adj_nu,d.  g_0 = (-1, .., -1),
// g_a = e_{a-1} for a >= 1.  dg is the block (a, a) of A_e.
template <int FORM, int DIM, typename R>
__device__ __forceinline__ void row_of_g(const R (&adj)[DIM][DIM], R wa, R wb, int a,
                                         float (&w)[DIM][Traits<FORM, DIM>::NC]
                                                   [Traits<FORM, DIM>::NC],
                                         float (&dg)[Traits<FORM, DIM>::NC][Traits<FORM, DIM>::NC])
{
    R beta[DIM];
#pragma unroll
    for (int al = 0; al < DIM; ++al) {
        R s = adj[0][al];
#pragma unroll
        for (int m = 1; m < DIM; ++m) s += adj[m][al];
        R r = -s;
#pragma unroll
        for (int m = 0; m < DIM; ++m) r = (a == m + 1) ? adj[m][al] : r;
        beta[al] = r;
    }
#pragma unroll
    for (int nu = 0; nu < DIM; ++nu) {
        R mnu = adj[nu][0] * beta[0];
#pragma unroll
        for (int al = 1; al < DIM; ++al) mnu += adj[nu][al] * beta[al];
        if constexpr (FORM != ELA1) {
            w[nu][0][0] = float(wa * mnu);
        } else {
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    R t = wa * (beta[d] * adj[nu][c]) + wb * (beta[c] * adj[nu][d]);
                    if (c == d) t += wa * mnu;
                    w[nu][c][d] = float(t);
                }
        }
    }
    // the diagonal block (a, a): g_a contracted on both sides, beta . beta and
    // beta beta^T
    R bb = beta[0] * beta[0];
#pragma unroll
    for (int al = 1; al < DIM; ++al) bb += beta[al] * beta[al];
    if constexpr (FORM != ELA1) {
        dg[0][0] = float(wa * bb);
    } else {
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                R t = wa * (beta[d] * beta[c]) + wb * (beta[c] * beta[d]);
                if (c == d) t += wa * bb;
                dg[c][d] = float(t);
            }
    }
}

// The geometry of one element (FP32, or FP64 when the quality test flags it,
// as the forward) and its row a of G_e : K (row_of_g, in FP32).  Returns the
// flag; *singular reports det J == 0 on the path taken.
template <int FORM, int DIM>
__device__ __forceinline__ bool row_block(const float (&xv)[DIM + 1][DIM], float mu, float lam,
                                          float tau2, int a,
                                          float (&w)[DIM][Traits<FORM, DIM>::NC]
                                                    [Traits<FORM, DIM>::NC],
                                          float (&dg)[Traits<FORM, DIM>::NC]
                                                     [Traits<FORM, DIM>::NC],
                                          bool &singular)
{
    float J[DIM][DIM], adj[DIM][DIM];
    jacobian<DIM>(xv, J);
    const float det = adjugate(J, adj);
    const bool flag = needs_fp64<DIM>(J, adj, det, tau2);
    float wa, wb;
    singular = false;
    if (!flag) {
        gf_weights<FORM, DIM>(det, mu, lam, wa, wb);
    } else {
        // J, adj J, det J and the weights in FP64 (where FP32 loses the
        // element), rounded for the FP32 contraction, whose error is then
        // normwise FP32 as for every other element
        double Jd[DIM][DIM], adjd[DIM][DIM], wad, wbd;
        jacobian<DIM>(xv, Jd);
        const double detd = adjugate(Jd, adjd);
        singular = detd == 0.0;
        gf_weights<FORM, DIM>(detd, mu, lam, wad, wbd);
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) adj[m][n] = float(adjd[m][n]);
        wa = float(wad);
        wb = float(wbd);
    }
    row_of_g<FORM, DIM>(adj, wa, wb, a, w, dg);
    return flag;
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

    const int32_t r0 = p.chunks[chunk], r1 = p.chunks[chunk + 1];
    const int nrows = r1 - r0;
    const int32_t s0 = p.rowptr[r0], s1 = p.rowptr[r1];
    const int nslot = s1 - s0;

    // this lane's row and its share (every kAsmLanes-th incidence) of the row's
    // list; the per-row pointers are loaded together with the chunk's columns
    const int part = lane / kAsmRows, local = lane % kAsmRows;
    const bool has_row = local < nrows;
    const int32_t row = r0 + (has_row ? local : 0);                  // in range
    const int32_t i0 = p.ptr[row], i1 = p.ptr[row + 1];
    const int32_t c0 = p.rowptr[row], c1 = p.rowptr[row + 1];
    const int32_t jb = has_row ? i0 + part : 0, je = has_row ? i1 : 0;
    const int b0 = has_row ? c0 - s0 : 0, b1 = has_row ? c1 - s0 : 0;
    if (nslot > 0) {
        // all of the chunk's column loads in flight at once (indexes clamped into the chunk)
        constexpr int CL = (kAsmSlots + 63) / 64;
        int c[CL];
#pragma unroll
        for (int i = 0; i < CL; ++i) c[i] = p.colidx[s0 + min(lane + 64 * i, nslot - 1)];
#pragma unroll
        for (int i = 0; i < CL; ++i)
            if (lane + 64 * i < nslot) col[lane + 64 * i] = c[i];
    }
    // 16-byte zeroing: the accumulator is a whole number of 16-byte pieces
    static_assert(SH::ACC % 4 == 0 && SH::WAVE_BYTES % 16 == 0, "16-byte accumulator pieces");
    for (int k = 4 * lane; k < nslot * BS2; k += 256)
        *reinterpret_cast<float4 *>(acc + k) = make_float4(0.f, 0.f, 0.f, 0.f);
    wave_sync();

    // the wave steps through the longest share of its rows (je - jb >= 1 - kAsmLanes)
    int steps = has_row ? (je - jb + kAsmLanes - 1) / kAsmLanes : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) steps = max(steps, __shfl_xor(steps, off));

    const float *__restrict__ mu = p.mu;
    const float *__restrict__ lam = p.lam;
    // each lane's share of its row's diagonal block, added into LDS at the end
    float dsum[NC][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = 0; d < NC; ++d) dsum[c][d] = 0.f;
    // the schedule is empty when no row has a step: nothing may be read then
    if (steps > 0) {
        // Software pipeline over the steps: each step issues the coordinate
        // loads of its own element, the connectivity of the next step's element
        // and the schedule entry two steps ahead before its arithmetic, so of
        // the three dependent loads only the last is exposed.  Lanes past the
        // end of their row's schedule read entry 0, padding entries (-1) read
        // element 0; neither adds anything.
        auto entry_at = [&](int it, int32_t &ent, uint32_t &sl) {
            const int32_t j = jb + kAsmLanes * it;
            const int32_t jj = (has_row && j < je) ? j : 0;
            ent = p.inc[jj];
            sl = uint32_t(p.slots[jj]);
        };
        int32_t ent;
        uint32_t sl;
        entry_at(0, ent, sl);
        int v[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = p.m.conn[int64_t(max(ent, 0) / NV) * NV + m];
        int32_t ent1;
        uint32_t sl1;
        entry_at(1, ent1, sl1);
        for (int it = 0; it < steps; ++it) {
            const bool live = has_row && jb + kAsmLanes * it < je && ent >= 0;
            const int64_t e = max(ent, 0) / NV;
            const int a = max(ent, 0) - int(e) * NV;
            // plain loads: every element is read once per vertex, by neighbouring rows
            float xv[NV][DIM];
            gather<DIM>(p.m, v, xv);
            float me = 0.f, le = 0.f;
            if constexpr (FORM == ELA1) {
                me = mu[e];
                le = lam[e];
            }
            int v1[NV];
#pragma unroll
            for (int m = 0; m < NV; ++m) v1[m] = p.m.conn[int64_t(max(ent1, 0) / NV) * NV + m];
            int32_t ent2;
            uint32_t sl2;
            entry_at(it + 2, ent2, sl2);

            // w[nu][c][d] = sum_mu g_a,mu G^{(mu c),(nu d)}: row a of G_e : K before its
            // contraction with g_b; dg = block (a, a)
            float w[DIM][NC][NC], dg[NC][NC];
            bool singular = false;
            const bool flag = row_block<FORM, DIM>(xv, me, le, p.tau2, a, w, dg, singular);
            // each element counted once: at its incidence with local vertex 0
            count_flags(p.counters, live && a == 0 && flag, live && a == 0 && singular);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < NC; ++d) dsum[c][d] += live ? dg[c][d] : 0.f;

            // off-diagonal blocks (a, b), b != a: sum_nu g_b,nu w[nu] = w[b - 1]
            // for b >= 1, minus their sum for b = 0
            int slot[NV];
#pragma unroll
            for (int b = 0; b < NV; ++b)    // the plan's slot bytes, relative to the row's first
                slot[b] = (live && b != a) ? b0 + int((sl >> (8 * b)) & 255u) : -1;
            float w0[NC][NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < NC; ++d) {
                    float t = w[0][c][d];
#pragma unroll
                    for (int nu = 1; nu < DIM; ++nu) t += w[nu][c][d];
                    w0[c][d] = -t;
                }
            // The step's elements share no vertex but the row's (the plan's
            // schedule), and rows are distinct, so no two lanes touch one block:
            // the whole wave adds at once with plain read-modify-writes, a
            // lane's reads before its writes (its slots are distinct: an
            // element's vertices are; one that lists a vertex twice is singular,
            // and the entries it reaches are not finite either way).
            float old[NV][BS2];
#pragma unroll
            for (int b = 0; b < NV; ++b)
#pragma unroll
                for (int i = 0; i < BS2; ++i) old[b][i] = acc[max(slot[b], 0) * BS2 + i];
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                if (slot[b] < 0) continue;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int d = 0; d < NC; ++d)
                        acc[slot[b] * BS2 + c * NC + d] =
                            old[b][c * NC + d] + (b == 0 ? w0[c][d] : w[b - 1][c][d]);
            }
            wave_sync();
            ent = ent1;
            sl = sl1;
#pragma unroll
            for (int m = 0; m < NV; ++m) v[m] = v1[m];
            ent1 = ent2;
            sl1 = sl2;
        }
    }
    // the diagonal blocks: the kAsmLanes lanes of a row add their shares in turn
    {
        const int sd = has_row ? find_slot(col, b0, b1, row) : -1;
#pragma unroll
        for (int h = 0; h < kAsmLanes; ++h) {
            if (part == h && sd >= 0) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int d = 0; d < NC; ++d) acc[sd * BS2 + c * NC + d] += dsum[c][d];
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

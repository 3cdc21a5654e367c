// Adjoint of the element integration for L = sum_e <dA_e, A_e>.
//
// The forward chain is A = Gf : K (eq. 1), Gf from (B = J^-1, s = |det J|,
// mu, lambda) (eq. 8 and its Lame analogue), J from the vertex coordinates.
// Reverse, per element, one lane per element, recomputing the geometry:
//
//   U_g   = sum_IJ dA_IJ Kf[g][IJ]             (the folded K^T applied to dA)
//   S     = symmetric tensor with S_pp = U_pp, S_pq = S_qp = U_pq / 2
//   Laplacian forms, Gf = c s B B^T:
//     sbar = c <S, BB^T>,  Bbar = 2 c s S B
//   Elasticity, Gf = c s [mu P1(B) + lambda P2(B)]:
//     H_mn = sum_c S_(mc),(nc);  Z_kg = sum_cn S_(kc),(ng) B_nc;
//     Y_kg = sum_nd S_(kg),(nd) B_nd;
//     F1 = <H, BB^T> + sum_md B_md Z_md;  F2 = sum_mc B_mc Y_mc
//     mubar = c s F1,  lambar = c s F2,  sbar = c (mu F1 + lambda F2)
//     Bbar = c s (2 mu (H B + Z) + 2 lambda Y)
//   Jbar = sbar s B^T - B^T Bbar B^T        (d|det J| = s J^-T : dJ, dB = -B dJ B)
//   xbar_{m+1} += Jbar[:, m],  xbar_0 -= sum_m Jbar[:, m]   (FP32 atomics)
//
// dA is read through LDS: the wave loads R rows of its 64 elements' dA with
// consecutive lanes on consecutive 16-byte pieces, then every lane folds its
// own rows into U.  With R = n (whole matrices) the wave stages EC of its
// element matrices at a time (32 for the 12 x 12 and 10 x 10 matrices, 64 for
// the smaller ones): each chunk is one contiguous, line-aligned run of dA, the
// next chunk's loads are in flight while the lanes owning this chunk's
// elements fold it, and no line is fetched twice.
//
// Split-precision MFMA fold (PREC = FP16x2, BF16x2, BF16x3; whole-matrix
// staging): the fold of a staged chunk is the dense product
//   U^T[g][elements] = Kf[g][ij] . dA^T[ij][elements]
// on v_mfma_f32_16x16x32_{f16,bf16}, every lane of the wave taking part (16
// elements per MFMA column block).  dA is split into two or three 16-bit
// terms (FP16 with a power-of-two scale per element, undone exactly), each
// multiplied by the same integer Kf, which is exact in both formats; the
// products accumulate in FP32 and pass through LDS to the lane that owns the
// element.  The reverse geometry stays FP32 (FP64 for flagged elements, whose
// fold is FP64 as in the FP32 form).
//
// Elements flagged by the quality test run the reverse geometry in FP64, and
// their U is recomputed in FP64 too: for such a tet (kappa ~ 1e3) the FP32
// rounding of U alone is amplified to ~1e-4 in dL/dx.  That FP64 fold is done
// by the whole wave, one lane per unique entry g, from the sparse rows of Kf,
// so a flagged element costs a few instructions instead of a serial fold.
// FP64 coordinates run everything in FP64.
#pragma once

#include "fwd_mfma.h"

namespace fei {

template <int FORM, int DIM>
__device__ KSparse<FORM, DIM> g_ksparse;

// A fragments of the MFMA fold per (form, dim, 16-bit format); values
// generated at build time.
template <int FORM, int DIM, int PREC>
__device__ AdjFragTable<FORM, DIM, PREC> g_adj_frags;

// S accessors: from registers (U as accumulated) or from an LDS copy.
template <int FORM, int DIM, typename AccT>
struct SRegs {
    const AccT (&U)[Traits<FORM, DIM>::G];
    template <typename R>
    __device__ __forceinline__ R get(int p, int q) const
    {
        const R u = R(U[sym_index(Traits<FORM, DIM>::GD, p, q)]);
        return p == q ? u : R(0.5) * u;
    }
};

struct SLds {
    const double *u;
    int gd;
    template <typename R>
    __device__ __forceinline__ R get(int p, int q) const
    {
        const R v = R(u[sym_index(gd, p, q)]);
        return p == q ? v : R(0.5) * v;
    }
};

template <int FORM, int DIM, typename R, typename SAcc>
__device__ __forceinline__ void adjoint_chain(const R (&adj)[DIM][DIM], R det, float mu_f,
                                              float lam_f, const SAcc &S,
                                              float (&Jbar)[DIM][DIM], float &mubar,
                                              float &lambar)
{
    using T = Traits<FORM, DIM>;
    const R s = det < R(0) ? -det : det;
    const R c = R(T::SCALE);
    const R inv = R(1) / det;
    R B[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int a = 0; a < DIM; ++a) B[m][a] = adj[m][a] * inv;
    R M[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int n = 0; n < DIM; ++n) {
            R acc = R(0);
#pragma unroll
            for (int a = 0; a < DIM; ++a) acc += B[m][a] * B[n][a];
            M[m][n] = acc;
        }
    R sbar;
    R Bbar[DIM][DIM];
    if constexpr (FORM != ELA1) {
        R F = R(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) F += S.template get<R>(m, n) * M[m][n];
        sbar = c * F;
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                R acc = R(0);
#pragma unroll
                for (int n = 0; n < DIM; ++n) acc += S.template get<R>(k, n) * B[n][g];
                Bbar[k][g] = R(2) * c * s * acc;
            }
        mubar = 0.f;
        lambar = 0.f;
    } else {
        const R mu = R(mu_f), lam = R(lam_f);
        R H[DIM][DIM], Z[DIM][DIM], Y[DIM][DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) {
                R h = R(0);
#pragma unroll
                for (int cc = 0; cc < DIM; ++cc) h += S.template get<R>(m * DIM + cc, n * DIM + cc);
                H[m][n] = h;
            }
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                R z = R(0), y = R(0);
#pragma unroll
                for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
                    for (int n = 0; n < DIM; ++n) {
                        z += S.template get<R>(k * DIM + cc, n * DIM + g) * B[n][cc];
                        y += S.template get<R>(k * DIM + g, n * DIM + cc) * B[n][cc];
                    }
                Z[k][g] = z;
                Y[k][g] = y;
            }
        R F1 = R(0), F2 = R(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) {
                F1 += H[m][n] * M[m][n] + B[m][n] * Z[m][n];
                F2 += B[m][n] * Y[m][n];
            }
        mubar = float(c * s * F1);
        lambar = float(c * s * F2);
        sbar = c * (mu * F1 + lam * F2);
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                R hb = R(0);
#pragma unroll
                for (int n = 0; n < DIM; ++n) hb += H[k][n] * B[n][g];
                Bbar[k][g] = c * s * (R(2) * mu * (hb + Z[k][g]) + R(2) * lam * Y[k][g]);
            }
    }
    // Jbar[a][m] = sbar s B[m][a] - sum_kl B[k][a] Bbar[k][l] B[m][l]
    R W[DIM][DIM];  // W = Bbar B^T : W[k][m] = sum_l Bbar[k][l] B[m][l]
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            R acc = R(0);
#pragma unroll
            for (int l = 0; l < DIM; ++l) acc += Bbar[k][l] * B[m][l];
            W[k][m] = acc;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            R acc = sbar * s * B[m][a];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc -= B[k][a] * W[k][m];
            Jbar[a][m] = float(acc);
        }
}

// Fold one 4-float piece of dA (entries flat0..flat0+3) into U.
template <int FORM, int DIM, typename AccT>
__device__ __forceinline__ void fold_piece(AccT *uacc, int flat0, const float (&r)[4],
                                           int count)
{
    using T = Traits<FORM, DIM>;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= count) break;
        const int flat = flat0 + k;
        const int I = flat / T::N, J = flat % T::N;
        const int a = I / T::NC, cI = I % T::NC, b = J / T::NC, dJ = J % T::NC;
#pragma unroll
        for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
            for (int nu = 0; nu < DIM; ++nu) {
                const int g = sym_index(T::GD, mu * T::NC + cI, nu * T::NC + dJ);
                // Zero entries of K add no term (a select decided at compile
                // time, not a branch, so the loops still unroll fully).
                const float kv = kval<FORM, DIM>(a, b, mu, nu);
                const AccT sum = uacc[g] + AccT(kv) * AccT(r[k]);
                uacc[g] = (kv != 0.f) ? sum : uacc[g];
            }
    }
}

// Vertex scatter.  The wave's 64 elements reference (DIM+1)*64 vertices but,
// on any mesh with locality, far fewer distinct ones (~48 for consecutive Kuhn
// tets).  The wave first merges its contributions per vertex in an LDS
// open-addressing table (CAS on the key, LDS float atomics on the values),
// then issues one global FP32 atomic per distinct vertex and component.
// 256 slots: as many as the wave's vertex references (64 elements x 4), so
// the table never fills and every probe sequence ends; a mesh with locality
// fills under a fifth of it.  (512 slots cost 16 KB more LDS per workgroup,
// which left room for one workgroup per CU instead of two: measured 285 vs
// 250 us for the 3D elasticity adjoint, 216 vs 140 us for the 3D Laplacian.)
constexpr int kHashSlots = 256;

__device__ __forceinline__ int hash_slot(int v)
{
    return int((unsigned(v) * 2654435761u) >> (32 - 8));  // Knuth multiplicative, 8 bits
}

template <int DIM>
__device__ __forceinline__ void scatter_vertices(const AdjParams &p, const int (&v)[DIM + 1],
                                                 const float (&Jbar)[DIM][DIM], bool valid,
                                                 int *key, float *val, int lane)
{
    for (int i = lane; i < kHashSlots; i += 64) {
        key[i] = -1;
#pragma unroll
        for (int al = 0; al < DIM; ++al) val[i * DIM + al] = 0.f;
    }
    wave_sync();
    if (valid) {
#pragma unroll
        for (int a = 0; a <= DIM; ++a) {
            // contribution to vertex a: column a-1 of Jbar, or minus the row sums
            float c[DIM];
#pragma unroll
            for (int al = 0; al < DIM; ++al) {
                if (a > 0) {
                    c[al] = Jbar[al][a - 1];
                } else {
                    float s0 = 0.f;
#pragma unroll
                    for (int m = 0; m < DIM; ++m) s0 += Jbar[al][m];
                    c[al] = -s0;
                }
            }
            int h = hash_slot(v[a]);
            for (int probe = 0; probe < kHashSlots; ++probe) {
                const int old = atomicCAS(key + h, -1, v[a]);
                if (old == -1 || old == v[a]) break;
                h = (h + 1) & (kHashSlots - 1);
            }
#pragma unroll
            for (int al = 0; al < DIM; ++al) atomicAdd(val + h * DIM + al, c[al]);
        }
    }
    wave_sync();
    float *X[3] = {p.dx, p.dy, p.dz};
    for (int i = lane; i < kHashSlots; i += 64) {
        const int k = key[i];
        if (k >= 0) {
#pragma unroll
            for (int al = 0; al < DIM; ++al) unsafeAtomicAdd(X[al] + k, val[i * DIM + al]);
        }
    }
}

// GATHER: the tile always writes J-bar (AdjParams.jbar) and carries no vertex
// table; otherwise it scatters, or writes J-bar when jbar is set.  PREC other
// than P_FP32: the MFMA fold (whole-matrix staging, FP32 coordinates).
template <int FORM, int DIM, typename CT, int R, bool GATHER = false, int PREC = P_FP32>
struct AdjTile {
    using T = Traits<FORM, DIM>;
    using S = Stage<FORM, DIM, R>;
    using AccT = typename std::conditional<sizeof(CT) == 8, double, float>::type;
    static constexpr int NN = S::NN;
    static constexpr int GP = ((T::G + 1) / 2) * 2;
    // Whole-matrix staging (R = n, n*n a multiple of 4): EC elements per
    // chunk, NWC chunks per wave, WP 16-byte pieces per chunk (WNP per lane).
    static constexpr bool WHOLE = (R == T::N) && (NN % 4 == 0);
    static constexpr bool MF = PREC != P_FP32;
    static_assert(!MF || (WHOLE && sizeof(CT) == 4), "MFMA fold: whole matrices, FP32 coordinates");
    using MS = MfmaAdjShape<FORM, DIM>;
    // MFMA fold: A fragments in registers when they take at most 32 VGPRs,
    // else in LDS (one copy per workgroup); chunks of 16 matrices (one MFMA
    // column block) when 64 would not fit 20 KB
    static constexpr bool AFREG = MS::MT * MS::KS <= 8;
    static constexpr int EC = WHOLE ? ((64 * (NN + 4) * 4 <= 20 * 1024) ? 64 : (MF ? 16 : 32)) : 64;
    static constexpr int NWC = WHOLE ? 64 / EC : 0;
    static constexpr int WP = EC * NN / 4;
    static constexpr int WNP = (WP + 63) / 64;
    // Next chunk in flight while this one is folded, where registers allow it
    // (the 12 x 12 matrices' 18 KB chunk would hold 72 more registers next to
    // U and the FP64 chain: the waves resident beside this one cover the
    // latency instead).  The MFMA fold holds its accumulators (16 per M
    // tile) and the register-resident A fragments instead of U.
    static constexpr bool WPREFETCH = MF
        ? (8 * WNP + 16 * MS::MT + (AFREG ? 4 * MS::MT * MS::KS : 0) <= 140)
        : (WNP * 4 + T::G <= 100);
    static constexpr int SLOTS = GATHER ? 0 : kHashSlots;
    // U^T rows of the MFMA fold, transposed through LDS (row stride UST floats)
    static constexpr int UST = 16 * MS::MT + 4;
    // A whole-matrix chunk buffer is reused, once the fold is done, for the
    // FP64 fold of flagged elements (dA row + GP doubles), the vertex-merge
    // table, the J-bar staging and the MFMA fold's transpose; it must hold
    // each of them.
    static constexpr int WHOLE_SW0 = (EC * S::STR > 64 * DIM * DIM + 4)
        ? EC * S::STR : 64 * DIM * DIM + 4;
    static constexpr int WHOLE_SW = (MF && 64 * UST > WHOLE_SW0) ? 64 * UST : WHOLE_SW0;
    static constexpr int WHOLE_SW2 = (WHOLE_SW > SLOTS * (1 + DIM)) ? WHOLE_SW : SLOTS * (1 + DIM);
    // (whole staging: the FP64 fold of a flagged element runs while its chunk
    // is staged, from the chunk, into GP doubles past the chunk buffer)
    static constexpr int WHOLE_U64 = ((WHOLE_SW2 + 1) / 2) * 2;
    // FP64 folds of a wave's first NS64 flagged elements, kept until the
    // reverse pass (further flagged elements reread their dA there)
    static constexpr int NS64 = 2;
    static constexpr int SW = WHOLE ? WHOLE_U64 + 2 * GP * (1 + NS64)
                          : (R > 0) ? ((64 * S::STR > NN) ? 64 * S::STR : NN) : ((NN + 3) / 4) * 4;
    // Flagged elements of a wave whose dA is kept in LDS while it streams past
    // (further flagged elements of the same wave reload theirs from memory;
    // with whole-matrix staging all of them do).
    static constexpr int NSTASH = (R > 0 && !WHOLE && sizeof(CT) == 4) ? 2 : 0;
    // LDS: dA staging | FP64 fold of a flagged element | vertex-merge keys |
    // values | stashed dA of flagged elements (whole-matrix staging: the
    // staging buffer alone, reused)
    static constexpr int OFF_U64 = 4 * SW * 4;
    static constexpr int OFF_KEY = OFF_U64 + (WHOLE ? 0 : 4 * GP * 8);
    static constexpr int OFF_VAL = OFF_KEY + (WHOLE ? 0 : 4 * SLOTS * 4);
    static constexpr int OFF_STASH = OFF_VAL + (WHOLE ? 0 : 4 * SLOTS * DIM * 4);
    static constexpr int OFF_FRAG = OFF_STASH + 4 * NSTASH * NN * 4;
    static constexpr int LDS_BYTES = OFF_FRAG + ((MF && !AFREG) ? MS::NFRAG * 16 : 0);

    struct Lds {
        float *st;       // staging rows (SW floats)
        double *u64;     // FP64 fold (GP doubles)
        int *key;        // vertex-merge table
        float *val;
        float *stash;    // NSTASH whole dA matrices
    };
    __device__ static Lds lds(unsigned char *smem)
    {
        const int wave = wave_id();
        if constexpr (WHOLE) {
            float *b = reinterpret_cast<float *>(smem) + wave * SW;
            return {b, reinterpret_cast<double *>(b + WHOLE_U64), reinterpret_cast<int *>(b),
                    b + SLOTS, nullptr};
        }
        return {reinterpret_cast<float *>(smem) + wave * SW,
                reinterpret_cast<double *>(smem + OFF_U64) + wave * GP,
                reinterpret_cast<int *>(smem + OFF_KEY) + wave * SLOTS,
                reinterpret_cast<float *>(smem + OFF_VAL) + wave * SLOTS * DIM,
                reinterpret_cast<float *>(smem + OFF_STASH) + wave * NSTASH * NN};
    }

    struct In {          // connectivity of this lane's element
        int v[DIM + 1];
    };
    struct Xv {          // gathered vertex coordinates and coefficients
        CT x[DIM + 1][DIM];
        float mu, lam;
    };
    struct Chunk {       // the wave's 16-byte dA pieces of one staged chunk
        f32x4_t r[WHOLE ? WNP : (R > 0) ? S::NV4 : 1];
    };
    struct AFrags {      // MFMA fold: register-resident A fragments
        uint4 v[(MF && AFREG) ? MS::MT * MS::KS : 1];
    };
    static constexpr int TP = (PREC == P_FP16X2) ? P_FP16X2 : P_BF16X2;   // fragment encoding

    // A fragments into registers, or into LDS with a workgroup barrier; once
    // per workgroup, before the first tile.
    __device__ static void load_afrags(AFrags &a, unsigned char *smem)
    {
        if constexpr (MF) {
            const uint4 *gfr = reinterpret_cast<const uint4 *>(g_adj_frags<FORM, DIM, TP>.v);
            if constexpr (AFREG) {
                const int lane = threadIdx.x & 63;
#pragma unroll
                for (int i = 0; i < MS::MT * MS::KS; ++i) a.v[i] = gfr[i * 64 + lane];
            } else {
                uint4 *sf = reinterpret_cast<uint4 *>(smem + OFF_FRAG);
                for (int i = threadIdx.x; i < MS::NFRAG; i += 256) sf[i] = gfr[i];
                __syncthreads();
            }
        }
    }

    __device__ static uint4 afrag(const AFrags &a, const unsigned char *smem, int t, int s)
    {
        if constexpr (AFREG) return a.v[t * MS::KS + s];
        else return reinterpret_cast<const uint4 *>(smem + OFF_FRAG)[(t * MS::KS + s) * 64 +
                                                                    (threadIdx.x & 63)];
    }

    // Loads of lanes past the last element (and of tiles past the end) read
    // the last element; their results are never used.  No branch around a
    // load, so prefetched data is waited for only where it is consumed.
    __device__ static int64_t clamp(const AdjParams &p, int64_t e)
    {
        return e < p.m.n_elements ? e : p.m.n_elements - 1;
    }

    __device__ static In load(const AdjParams &p, int64_t blk)
    {
        In in;
        load_conn<DIM>(p.m.conn, clamp(p, blk * 256 + threadIdx.x), in.v);
        return in;
    }

    __device__ static Xv gather_xv(const AdjParams &p, int64_t blk, const In &in)
    {
        Xv g;
        gather<DIM>(p.m, in.v, g.x);
        g.mu = g.lam = 0.f;
        if constexpr (FORM == ELA1) {
            const int64_t e = clamp(p, blk * 256 + threadIdx.x);
            g.mu = __builtin_nontemporal_load(p.mu + e);
            g.lam = __builtin_nontemporal_load(p.lam + e);
        }
        return g;
    }

    // Quality test ahead of the fold, so flagged elements can be stashed.
    __device__ static bool flagged(const AdjParams &p, int64_t blk, const Xv &g)
    {
        if constexpr (sizeof(CT) == 8) {
            return false;
        } else {
            float J[DIM][DIM], adj[DIM][DIM];
            jacobian<DIM>(g.x, J);
            const float det = adjugate(J, adj);
            return blk * 256 + threadIdx.x < p.m.n_elements && needs_fp64<DIM>(J, adj, det, p.tau2);
        }
    }

    // Chunk c of the wave's dA: consecutive lanes on consecutive 16-byte pieces.
    // Plain (temporal) loads: a chunk boundary can fall inside a 128-byte
    // line, whose other part the next chunk reads, and a non-temporal load
    // lets L2 drop that line in between (measured 1.24x the algorithmic read
    // bytes with non-temporal loads, 1.06x with plain ones, single call).
    __device__ static Chunk load_chunk(const AdjParams &p, int64_t blk, int c)
    {
        Chunk ch;
        if constexpr (R > 0) {
            const int lane = threadIdx.x & 63;
            const int64_t e0 = blk * 256 + wave_id() * 64;
#pragma unroll
            for (int k = 0; k < S::NV4; ++k) {
                const int f = lane + 64 * k;
                const int el = f / S::NV4, part = f - el * S::NV4;
                ch.r[k] = *reinterpret_cast<const f32x4_t *>(
                    p.dA + clamp(p, e0 + el) * (int64_t)NN + c * S::CH + 4 * part);
            }
        }
        return ch;
    }

    // Stage chunk c through the wave's LDS rows, fold this lane's rows into U,
    // and copy the rows of (up to NSTASH) flagged elements into the stash.
    __device__ static void fold_chunk(const Lds &L, int c, const Chunk &ch, unsigned long long fm,
                                      AccT (&U)[T::G])
    {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int k = 0; k < S::NV4; ++k) {
            const int f = lane + 64 * k;
            const int el = f / S::NV4, part = f - el * S::NV4;
            *reinterpret_cast<f32x4_t *>(L.st + el * S::STR + 4 * part) = ch.r[k];
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < S::CH; k += 4) {
            const f32x4_t w = *reinterpret_cast<const f32x4_t *>(L.st + lane * S::STR + k);
            const float r[4] = {w[0], w[1], w[2], w[3]};
            fold_piece<FORM, DIM, AccT>(U, c * S::CH + k, r, 4);
        }
#pragma unroll
        for (int s = 0; s < NSTASH; ++s) {
            if (!fm) break;
            const int el = __ffsll(fm) - 1;
            fm &= fm - 1;
            for (int k = lane; k < S::CH; k += 64)
                L.stash[s * NN + c * S::CH + k] = L.st[el * S::STR + k];
        }
        wave_sync();
    }

    // Whole-matrix chunk c of the wave: elements e0 + c EC .. + EC as one
    // contiguous run, consecutive lanes on consecutive 16-byte pieces (pieces of
    // elements past the last one read the last element).
    __device__ static Chunk load_whole(const AdjParams &p, int64_t blk, int c)
    {
        Chunk ch;
        if constexpr (WHOLE) {
            const int lane = threadIdx.x & 63;
            const int64_t eb = blk * 256 + wave_id() * 64 + c * EC;
#pragma unroll
            for (int k = 0; k < WNP; ++k) {
                const int f = lane + 64 * k;
                if (WP % 64 == 0 || f < WP) {
                    const int el = f / S::NV4, part = f - el * S::NV4;
                    ch.r[k] = *reinterpret_cast<const f32x4_t *>(
                        p.dA + clamp(p, eb + el) * (int64_t)NN + 4 * part);
                }
            }
        }
        return ch;
    }

    __device__ static void stage_whole(const Lds &L, const Chunk &ch)
    {
        if constexpr (WHOLE) {
            const int lane = threadIdx.x & 63;
#pragma unroll
            for (int k = 0; k < WNP; ++k) {
                const int f = lane + 64 * k;
                if (WP % 64 == 0 || f < WP) {
                    const int el = f / S::NV4, part = f - el * S::NV4;
                    *reinterpret_cast<f32x4_t *>(L.st + el * S::STR + 4 * part) = ch.r[k];
                }
            }
        }
    }

    // The lanes whose elements are in staged chunk c fold them.
    __device__ static void fold_whole(const Lds &L, int c, AccT (&U)[T::G])
    {
        if constexpr (WHOLE) {
            const int lane = threadIdx.x & 63;
            if (lane / EC != c) return;
            const float *row = L.st + (lane % EC) * S::STR;
#pragma unroll
            for (int k = 0; k < NN; k += 4) {
                const f32x4_t w = *reinterpret_cast<const f32x4_t *>(row + k);
                const float r[4] = {w[0], w[1], w[2], w[3]};
                fold_piece<FORM, DIM, AccT>(U, k, r, 4);
            }
        }
    }

    // MFMA fold of staged chunk c (EC elements, EC / 16 column blocks): lane
    // (n, q) = (lane % 16, lane / 16) takes entries 32 s + 8 q .. + 8 of
    // element n of a block, splits them and multiplies them with the A
    // fragments; acc[b][t] then holds U^T rows 16 t + 4 q .. + 4 of the wave's
    // element 16 b + n.
    __device__ static void mfma_fold(const Lds &L, int c, const AFrags &af,
                                     const unsigned char *smem, floatx4_t (&acc)[4][MS::MT])
    {
        if constexpr (MF) {
            const int lane = threadIdx.x & 63, n = lane & 15, q = lane >> 4;
#pragma unroll
            for (int bl = 0; bl < EC / 16; ++bl) {
                const int b = c * (EC / 16) + bl;
                const float *row = L.st + (bl * 16 + n) * S::STR;
                float x[MS::KS][8];
#pragma unroll
                for (int s = 0; s < MS::KS; ++s)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int k0 = 32 * s + 8 * q + 4 * h;    // n*n is a multiple of 4
                        f32x4_t w = {0.f, 0.f, 0.f, 0.f};
                        if (k0 < NN) w = *reinterpret_cast<const f32x4_t *>(row + k0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) x[s][4 * h + i] = w[i];
                    }
                int E = 0;
                if constexpr (PREC == P_FP16X2) {
                    // the element's scale: its 4 lanes (q = 0..3) hold all its entries
                    float mx = 0.f;
#pragma unroll
                    for (int s = 0; s < MS::KS; ++s)
#pragma unroll
                        for (int j = 0; j < 8; ++j) mx = fmaxf(mx, fabsf(x[s][j]));
                    mx = fmaxf(mx, __shfl_xor(mx, 16));
                    mx = fmaxf(mx, __shfl_xor(mx, 32));
                    (void)frexpf(mx, &E);
                    if (!(mx < __builtin_huge_valf())) E = 0;  // Inf / NaN: leave unscaled
                }
#pragma unroll
                for (int s = 0; s < MS::KS; ++s) {
                    uint16_t hv[8], lv[8], l2[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        if constexpr (PREC == P_FP16X2) {
                            const float v = ldexpf(x[s][j], -E);
                            const _Float16 hi = (_Float16)v;
                            hv[j] = f16_bits(hi);
                            lv[j] = f16_bits((_Float16)(v - (float)hi));
                        } else {
                            const float v = x[s][j];
                            const __bf16 hi = (__bf16)v;
                            const float r1 = v - (float)hi;
                            const __bf16 mid = (__bf16)r1;
                            hv[j] = bf16_bits(hi);
                            lv[j] = bf16_bits(mid);
                            l2[j] = bf16_bits((__bf16)(r1 - (float)mid));
                        }
                    }
                    auto pack = [](const uint16_t (&h)[8]) {
                        uint4 w;
                        w.x = unsigned(h[0]) | (unsigned(h[1]) << 16);
                        w.y = unsigned(h[2]) | (unsigned(h[3]) << 16);
                        w.z = unsigned(h[4]) | (unsigned(h[5]) << 16);
                        w.w = unsigned(h[6]) | (unsigned(h[7]) << 16);
                        return w;
                    };
                    const uint4 bh = pack(hv), blo = pack(lv);
#pragma unroll
                    for (int t = 0; t < MS::MT; ++t) {
                        const uint4 a = afrag(af, smem, t, s);
                        acc[b][t] = mfma_step<PREC>(a, bh, acc[b][t]);
                        acc[b][t] = mfma_step<PREC>(a, blo, acc[b][t]);
                        if constexpr (PREC == P_BF16X3) acc[b][t] = mfma_step<PREC>(a, pack(l2), acc[b][t]);
                    }
                }
                if constexpr (PREC == P_FP16X2) {
#pragma unroll
                    for (int t = 0; t < MS::MT; ++t)
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[b][t][i] = ldexpf(acc[b][t][i], E);
                }
            }
        }
    }

    // The MFMA fold's accumulators to U of the owning lanes, through LDS.
    __device__ static void mfma_unfold(const Lds &L, const floatx4_t (&acc)[4][MS::MT],
                                       AccT (&U)[T::G])
    {
        if constexpr (MF) {
            const int lane = threadIdx.x & 63, n = lane & 15, q = lane >> 4;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int t = 0; t < MS::MT; ++t)
                    *reinterpret_cast<floatx4_t *>(L.st + (16 * b + n) * UST + 16 * t + 4 * q) =
                        acc[b][t];
            wave_sync();
#pragma unroll
            for (int g = 0; g < T::G; g += 4) {
                const floatx4_t w = *reinterpret_cast<const floatx4_t *>(L.st + lane * UST + g);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (g + i < T::G) U[g + i] = w[i];
            }
            wave_sync();
        }
    }

    // R == 0: every lane folds its own dA directly (plain loads: the lines a
    // lane touches are completed by its neighbours' reads through L2).
    __device__ static void fold_direct(const AdjParams &p, int64_t blk, AccT (&U)[T::G])
    {
        const float *__restrict__ dAe = p.dA + clamp(p, blk * 256 + threadIdx.x) * (int64_t)NN;
#pragma unroll
        for (int k = 0; k < NN; k += 4) {
            float r[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (k + i < NN) r[i] = dAe[k + i];
            fold_piece<FORM, DIM, AccT>(U, k, r, NN - k < 4 ? NN - k : 4);
        }
    }

    // Per-lane results of the reverse pass of one tile.
    struct Rev {
        float Jbar[DIM][DIM];
        float mubar, lambar;
        bool flag, singular;
    };

    // FP64 fold of one element whose dA (NN floats) is at src in LDS: the wave
    // folds U into u64 (one lane per unique entry g, sparse rows of K').
    __device__ static void fold_fp64(const float *src, double *u64)
    {
        const int lane = threadIdx.x & 63;
        if (lane < T::G) {
            constexpr int NZ = KSparseShape<FORM, DIM>::NNZ;
            const KSparse<FORM, DIM> &ks = g_ksparse<FORM, DIM>;
            double u = 0.0;
            for (int t = 0; t < NZ; ++t) u += double(ks.coef[lane][t]) * double(src[ks.ij[lane][t]]);
            u64[lane] = u;
        }
        wave_sync();
    }

    // FP64 chain of lane Lf's element from its FP64 fold u64.
    __device__ static void chain_fp64(int Lf, const Xv &g, const double *u64, Rev &o)
    {
        if ((threadIdx.x & 63) == Lf) {
            double Jd[DIM][DIM], adjd[DIM][DIM];
            jacobian<DIM>(g.x, Jd);
            const double detd = adjugate(Jd, adjd);
            o.singular = (detd == 0.0);
            adjoint_chain<FORM, DIM>(adjd, detd, g.mu, g.lam, SLds{u64, T::GD}, o.Jbar,
                                     o.mubar, o.lambar);
        }
        wave_sync();
    }

    // Flagged element of lane Lf whose dA (NN floats) is at src in LDS: the
    // wave folds U in FP64, then the owner runs the FP64 chain.
    __device__ static void flagged_fp64(const float *src, int Lf, const Xv &g, const Lds &L,
                                        Rev &o)
    {
        fold_fp64(src, L.u64);
        chain_fp64(Lf, g, L.u64, o);
    }

    // Reverse geometry of a tile whose U is folded.  fm: the wave's flagged
    // lanes, the first NSTASH of them with their dA in the stash.
    __device__ static Rev reverse(const AdjParams &p, int64_t blk, const Xv &g,
                                  const AccT (&U)[T::G], unsigned long long fm, const Lds &L)
    {
        const int lane = threadIdx.x & 63;
        const int64_t e0 = blk * 256 + wave_id() * 64;
        Rev o;
        o.mubar = o.lambar = 0.f;
        o.singular = false;
        o.flag = (fm >> lane) & 1;
        if constexpr (sizeof(CT) == 8) {
            double J[DIM][DIM], adj[DIM][DIM];
            jacobian<DIM>(g.x, J);
            const double det = adjugate(J, adj);
            o.singular = e0 + lane < p.m.n_elements && det == 0.0;
            adjoint_chain<FORM, DIM>(adj, det, g.mu, g.lam, SRegs<FORM, DIM, AccT>{U}, o.Jbar,
                                     o.mubar, o.lambar);
        } else {
            if (!o.flag) {
                float J[DIM][DIM], adj[DIM][DIM];
                jacobian<DIM>(g.x, J);
                const float det = adjugate(J, adj);
                adjoint_chain<FORM, DIM>(adj, det, g.mu, g.lam, SRegs<FORM, DIM, AccT>{U}, o.Jbar,
                                         o.mubar, o.lambar);
            }
            // flagged elements, one at a time: FP64 fold by the wave, FP64 chain by the owner
            int slot = 0;
            while (fm) {
                const int Lf = __ffsll(fm) - 1;
                fm &= fm - 1;
                const float *src = NSTASH > 0 ? L.stash + slot * NN : L.st;
                if (slot >= NSTASH) {
                    for (int k = lane; k < NN; k += 64)
                        L.st[k] = __builtin_nontemporal_load(p.dA + (e0 + Lf) * (int64_t)NN + k);
                    src = L.st;
                }
                ++slot;
                wave_sync();
                flagged_fp64(src, Lf, g, L, o);
            }
        }
        return o;
    }

    // Counters, coefficient gradients and the vertex scatter of a tile.
    __device__ static void emit(const AdjParams &p, int64_t blk, const In &in, const Rev &o,
                                const Lds &L)
    {
        const int lane = threadIdx.x & 63;
        const int64_t e = blk * 256 + threadIdx.x;
        const bool valid = e < p.m.n_elements;
        count_flags(p.counters, o.flag, o.singular);
        if constexpr (FORM == ELA1) {
            if (valid && p.dmu) p.dmu[e] = o.mubar;
            if (valid && p.dlam) p.dlam[e] = o.lambar;
        }
        if (GATHER || p.jbar) {
            // J-bar per element, gathered per vertex by a later kernel.  A full
            // wave's 64 blocks of DIM^2 floats are one contiguous run: staged
            // in LDS and stored as 16-byte pieces; otherwise lane by lane.
            constexpr int JN = DIM * DIM;
            const int64_t e0 = e - lane;
            if (SW >= 64 * JN && e0 + 64 <= p.m.n_elements) {
#pragma unroll
                for (int al = 0; al < DIM; ++al)
#pragma unroll
                    for (int m = 0; m < DIM; ++m) L.st[lane * JN + al * DIM + m] = o.Jbar[al][m];
                wave_sync();
                f32x4_t *dst = reinterpret_cast<f32x4_t *>(p.jbar + e0 * JN);
                const f32x4_t *src = reinterpret_cast<const f32x4_t *>(L.st);
#pragma unroll
                for (int f = lane; f < 16 * JN; f += 64) dst[f] = src[f];
                wave_sync();
            } else if (valid) {
                float *J = p.jbar + e * JN;
#pragma unroll
                for (int al = 0; al < DIM; ++al)
#pragma unroll
                    for (int m = 0; m < DIM; ++m) J[al * DIM + m] = o.Jbar[al][m];
            }
        } else if constexpr (!GATHER) {
            scatter_vertices<DIM>(p, in.v, o.Jbar, valid, L.key, L.val, lane);
        }
    }

    // One tile on its own (batch kernels): chunk c + 1 is loaded while chunk c
    // is folded, and chunk 0 travels with the connectivity and coordinates.
    __device__ __forceinline__ static void run(const AdjParams &p, int64_t blk, unsigned char *smem)
    {
        static_assert(!MF, "the MFMA fold takes its A fragments");
        run(p, blk, smem, AFrags{});
    }

    __device__ __forceinline__ static void run(const AdjParams &p, int64_t blk, unsigned char *smem,
                                               const AFrags &af)
    {
        const Lds L = lds(smem);
        if constexpr (WHOLE) {
            // coordinates first (their loads complete before dA's), then the
            // chunks: chunk c + 1 is in flight while chunk c is folded
            // Flagged elements: the FP64 fold of the wave's first NS64 of them
            // runs while their chunk is staged (no second read of their dA) and
            // is kept in LDS; the FP64 chains run after the FP32 ones, once U
            // is no longer live.
            const In in = load(p, blk);
            const Xv g = gather_xv(p, blk, in);
            Chunk ch = load_whole(p, blk, 0);
            const unsigned long long fm = __ballot(flagged(p, blk, g));
            const int lane = threadIdx.x & 63;
            Rev o;
            o.mubar = o.lambar = 0.f;
            o.singular = false;
            o.flag = (fm >> lane) & 1;
            AccT U[T::G];
#pragma unroll
            for (int k = 0; k < T::G; ++k) U[k] = AccT(0);
            floatx4_t acc[4][MS::MT];
            if constexpr (MF) {
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int t = 0; t < MS::MT; ++t) acc[b][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int c = 0; c < NWC; ++c) {
                if (!WPREFETCH && c > 0) ch = load_whole(p, blk, c);
                stage_whole(L, ch);
                if (WPREFETCH && c + 1 < NWC) ch = load_whole(p, blk, c + 1);
                wave_sync();
                if constexpr (MF) mfma_fold(L, c, af, smem, acc);
                else fold_whole(L, c, U);
                // flagged elements of this chunk among the wave's first NS64
                unsigned long long fc = fm;
                for (int sl = 0; sl < NS64 && fc; ++sl) {
                    const int Lf = __ffsll(fc) - 1;
                    fc &= fc - 1;
                    if (Lf / EC == c) fold_fp64(L.st + (Lf % EC) * S::STR, L.u64 + GP * (1 + sl));
                }
                wave_sync();
            }
            if constexpr (MF) mfma_unfold(L, acc, U);
            if constexpr (sizeof(CT) == 8) {
                o = reverse(p, blk, g, U, 0ull, L);
            } else {
                if (!o.flag) {
                    float J[DIM][DIM], adj[DIM][DIM];
                    jacobian<DIM>(g.x, J);
                    const float det = adjugate(J, adj);
                    adjoint_chain<FORM, DIM>(adj, det, g.mu, g.lam, SRegs<FORM, DIM, AccT>{U},
                                             o.Jbar, o.mubar, o.lambar);
                }
                const int64_t e0 = blk * 256 + wave_id() * 64;
                unsigned long long fc = fm;
                for (int sl = 0; fc; ++sl) {
                    const int Lf = __ffsll(fc) - 1;
                    fc &= fc - 1;
                    if (sl < NS64) {
                        chain_fp64(Lf, g, L.u64 + GP * (1 + sl), o);
                    } else {
                        // dA reread from memory into the (free) chunk buffer
                        for (int k = lane; k < NN; k += 64)
                            L.st[k] = __builtin_nontemporal_load(p.dA + (e0 + Lf) * (int64_t)NN + k);
                        wave_sync();
                        flagged_fp64(L.st, Lf, g, L, o);
                    }
                }
            }
            emit(p, blk, in, o, L);
        } else {
            const In in = load(p, blk);
            Chunk ch = load_chunk(p, blk, 0);
            const Xv g = gather_xv(p, blk, in);
            const unsigned long long fm = __ballot(flagged(p, blk, g));
            AccT U[T::G];
#pragma unroll
            for (int k = 0; k < T::G; ++k) U[k] = AccT(0);
            if constexpr (R > 0) {
#pragma unroll
                for (int c = 0; c < S::NCHUNK; ++c) {
                    Chunk nx;
                    if (c + 1 < S::NCHUNK) nx = load_chunk(p, blk, c + 1);
                    fold_chunk(L, c, ch, fm, U);
                    if (c + 1 < S::NCHUNK) ch = nx;
                }
            } else {
                fold_direct(p, blk, U);
            }
            emit(p, blk, in, reverse(p, blk, g, U, fm, L), L);
        }
    }
};

// Persistent, software-pipelined adjoint (tiles split over the XCDs as in
// the forward).  Loads run one step ahead of their use: chunk c + 1 of a tile
// is in flight while chunk c is staged and folded; the next tile's
// coordinates are gathered during the last chunk, and its chunk 0 is issued
// after the reverse pass, before this tile's atomics.  Vector-memory
// operations complete in issue order, so every prefetch is issued before the
// stores and atomics of the step it overlaps.
// Used for the scatter form, whose LDS vertex table leaves room for one
// workgroup per CU: the pipelining hides that low occupancy.
template <int FORM, int DIM, typename CT, int R>
__global__ __launch_bounds__(256) void adj_fma_kernel(AdjParams p, int64_t n_tiles)
{
    using Tile = AdjTile<FORM, DIM, CT, R, false>;
    using AccT = typename Tile::AccT;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Tile::LDS_BYTES];
    const PersistentTiles pt(n_tiles);
    if constexpr (R == 0 || Tile::WHOLE) {
        for (int64_t t = pt.begin; t < pt.end; t += pt.stride) Tile::run(p, t, smem);
    } else {
        constexpr int NCH = Stage<FORM, DIM, R>::NCHUNK;
        const typename Tile::Lds L = Tile::lds(smem);
        int64_t t = pt.begin;
        if (t >= pt.end) return;
        typename Tile::In cur = Tile::load(p, t);
        typename Tile::Xv g = Tile::gather_xv(p, t, cur);
        typename Tile::In nxt = Tile::load(p, t + pt.stride);
        typename Tile::Chunk ch = Tile::load_chunk(p, t, 0);
        for (;;) {
            const int64_t tn = t + pt.stride;
            const unsigned long long fm = __ballot(Tile::flagged(p, t, g));
            AccT U[Traits<FORM, DIM>::G];
#pragma unroll
            for (int k = 0; k < Traits<FORM, DIM>::G; ++k) U[k] = AccT(0);
            typename Tile::Xv gn;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                typename Tile::Chunk nx;
                if (c + 1 < NCH) nx = Tile::load_chunk(p, t, c + 1);
                if (c + 1 == NCH) gn = Tile::gather_xv(p, tn, nxt);
                Tile::fold_chunk(L, c, ch, fm, U);
                if (c + 1 < NCH) ch = nx;
            }
            const typename Tile::Rev o = Tile::reverse(p, t, g, U, fm, L);
            ch = Tile::load_chunk(p, tn, 0);
            Tile::emit(p, t, cur, o, L);
            if (tn >= pt.end) break;
            cur = nxt;
            nxt = Tile::load(p, tn + pt.stride);
            g = gn;
            t = tn;
        }
    }
}

// MFMA fold (split precision): persistent grid, tiles split per XCD; the A
// fragments are loaded once per workgroup.  Scatter or, with GATHER, J-bar.
template <int FORM, int DIM, int PREC, bool GATHER>
__global__ __launch_bounds__(256, 2) void adj_mfma_kernel(AdjParams p, int64_t n_tiles)
{
    using Tile = AdjTile<FORM, DIM, float, Traits<FORM, DIM>::N, GATHER, PREC>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Tile::LDS_BYTES];
    typename Tile::AFrags af;
    Tile::load_afrags(af, smem);
    const PersistentTiles pt(n_tiles);
    for (int64_t t = pt.begin; t < pt.end; t += pt.stride) Tile::run(p, t, smem, af);
}

// The gather form (no vertex table: 59 KB of LDS and under 200 registers for
// 3D elasticity, two workgroups per CU): one workgroup per tile, tiles
// remapped so that each XCD takes one contiguous range.  The hardware then
// overlaps the workgroups' memory streams; measured faster than the pipelined
// persistent loop for this form (3D elasticity plan: 255 vs 266 us).
template <int FORM, int DIM, typename CT, int R, bool GATHER>
__global__ __launch_bounds__(256) void adj_tile_kernel(AdjParams p)
{
    using Tile = AdjTile<FORM, DIM, CT, R, GATHER>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Tile::LDS_BYTES];
    Tile::run(p, xcd_block(blockIdx.x, gridDim.x), smem);
}

}  // namespace fei

// Forward element integration, FP32 fused multiply-add form.
//
// One lane per element (a wave integrates 64 elements).  The lane gathers its
// vertices, forms J, adj J, det J and the folded geometric tensor Gf in
// registers (Sec. 3, eq. 8), then produces its element matrix entry by entry:
//
//   A_{(a,c),(b,d)} = sum_{mu,nu} K^{ab}_{mu nu} G^{(mu c),(nu d)}     (eq. 6; eq. 14 block form)
//
// which is the paper's per-entry contraction of a d x d block of G with a
// d x d block of K (Sec. 4.3), executed sequentially by the lane for the
// n(n+1)/2 distinct entries of its (symmetric) element matrix.  K is the same
// for every lane of the grid and known when the library is built, so it is
// compiled into the instruction stream: no K traffic at all, only the
// nonzero terms of the contraction are executed, and LDS stays free for the
// output.
//
// Output (template R): with R = 0 every lane stores its own rows with 16-byte
// vector stores (a wave instruction then touches 64 lines, one 16-byte piece
// each).  With R > 0 the wave produces R rows of all its 64 element matrices
// at a time (the paper's interleaving of computation and stores, Sec. 4.3),
// writes them to LDS and stores them cooperatively: consecutive lanes write
// consecutive 16-byte pieces, so each store instruction covers contiguous
// runs of R*n*4 bytes.
#pragma once

#include "geometry.h"
#include "shapes.h"

namespace fei {

// Block reference tensors, one per (form, dim), as compile-time constants
// (the specializations holding the values are generated at build time).
// Every index is known after unrolling, so K is folded into the code: zero
// entries are skipped by a compile-time test (the compiler may not drop
// fma(0, x, a) by itself, since it is NaN for infinite x) and +-1 entries
// become adds.  For finite inputs the result is bit for bit that of the full
// multiply-add chain, since fma(0, x, a) = a and fma(+-1, x, a) = a +- x.
template <int FORM, int DIM>
struct KFold;

template <int FORM, int DIM>
__device__ __forceinline__ float kval(int i, int j, int mu, int nu)
{
    using T = Traits<FORM, DIM>;
    return KFold<FORM, DIM>::t.v[((i * T::NB + j) * DIM + mu) * DIM + nu];
}

// One entry of A from the folded geometric tensor (all indices compile-time
// after unrolling).
template <int FORM, int DIM>
__device__ __forceinline__ float contract_entry(const float (&Gf)[Traits<FORM, DIM>::G], int I,
                                                int J)
{
    using T = Traits<FORM, DIM>;
    const int a = I / T::NC, c = I % T::NC, b = J / T::NC, d = J % T::NC;
    float acc = 0.f;
#pragma unroll
    for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu) {
            // A zero entry of K contributes no term.  The test is decided at
            // compile time; without it the compiler must keep 0*G (IEEE: it
            // is NaN for an infinite G) as a multiply-add.
            const float k = kval<FORM, DIM>(a, b, mu, nu);
            if (k != 0.f) acc = fmaf(k, Gf[sym_index(T::GD, mu * T::NC + c, nu * T::NC + d)], acc);
        }
    return acc;
}

// The element matrix is symmetric (K^{ab}_{mu nu} = K^{ba}_{nu mu} and G is
// symmetric), so each lane contracts only the n(n+1)/2 entries I <= J and
// writes every entry from that set: half the multiply-adds, and A is
// symmetric to the bit.
template <int FORM, int DIM>
struct Unique {
    static constexpr int N = Traits<FORM, DIM>::N;
    static constexpr int NU = N * (N + 1) / 2;
};

template <int FORM, int DIM>
__device__ __forceinline__ void unique_entries(const float (&Gf)[Traits<FORM, DIM>::G],
                                               float (&Au)[Unique<FORM, DIM>::NU])
{
    constexpr int N = Traits<FORM, DIM>::N;
#pragma unroll
    for (int I = 0; I < N; ++I)
#pragma unroll
        for (int J = I; J < N; ++J) Au[sym_index(N, I, J)] = contract_entry<FORM, DIM>(Gf, I, J);
}

template <int VEC>
struct VecT;
template <> struct VecT<4> { using type = f32x4_t; };
template <> struct VecT<2> { using type = f32x2_t; };
template <> struct VecT<1> { using type = float; };

// Direct stores: the lane writes its element row by row.
template <int FORM, int DIM>
__device__ __forceinline__ void contract_store(const float (&Au)[Unique<FORM, DIM>::NU],
                                               float *__restrict__ Ae)
{
    using T = Traits<FORM, DIM>;
    constexpr int N = T::N;
    constexpr int VEC = (N % 4 == 0) ? 4 : (N % 2 == 0) ? 2 : 1;
    using V = typename VecT<VEC>::type;
#pragma unroll
    for (int I = 0; I < N; ++I) {
#pragma unroll
        for (int J0 = 0; J0 < N; J0 += VEC) {
            float r[VEC];
#pragma unroll
            for (int k = 0; k < VEC; ++k) r[k] = Au[sym_index(N, I, J0 + k)];
            V out;
            __builtin_memcpy(&out, r, sizeof(V));
            *reinterpret_cast<V *>(Ae + I * N + J0) = out;
        }
    }
}

// Staged layout: chunk of R rows = CH floats per element, LDS row stride STR
// floats (16-byte aligned, offset by 4 banks per lane for conflict-free
// 16-byte accesses).

template <int FORM, int DIM, int R>
struct Stage {
    static constexpr int N = Traits<FORM, DIM>::N;
    static constexpr int NN = N * N;
    static constexpr int CH = (R > 0) ? R * N : 4;
    static constexpr int STR = CH + 4;
    static constexpr int NV4 = CH / 4;        // 16-byte pieces per element chunk
    static constexpr int NCHUNK = (R > 0) ? N / R : 0;
    // R == N with n*n not a multiple of 4 (3x3): whole matrices, staged packed
    static_assert(R == 0 || R == N || (N % R == 0 && CH % 4 == 0), "bad chunk");
};

// Orders this wave's LDS accesses around a point (the LDS executes one
// wave's operations in issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup tile (256 elements, 4 waves) of the FP32 forward, in stages
// (load -> gather -> compute -> store; each wave owns 64 consecutive
// elements).  LDS comes from the caller (LDS_BYTES, 16-byte aligned), so one
// persistent kernel can also host the tiles of several forms.
template <int FORM, int DIM, typename CT, int R>
struct FwdFmaTile {
    using T = Traits<FORM, DIM>;
    using S = Stage<FORM, DIM, R>;
    using U = Unique<FORM, DIM>;
    // R == N stages whole matrices, EC elements of the wave at a time, so each
    // chunk leaves as one contiguous run of EC matrices; R < N stages R rows of
    // all 64 elements.  The 12 x 12 and 10 x 10 matrices go 32 at a time (76
    // and 53 KB of LDS per workgroup instead of 152 and 106 KB: two or three
    // resident workgroups per CU; measured faster than 64 or 16 at a time).
    static constexpr bool WHOLE = (R == T::N);
    // Whole matrices that are not a whole number of 16-byte pieces (the 3x3
    // matrices of the 2D P1 Laplacian): the wave's 64 matrices are staged
    // packed, exactly as they lie in A, and leave as one contiguous run.
    static constexpr bool PACKED = WHOLE && (S::NN % 4 != 0);
    static constexpr int EC = WHOLE ? (T::N >= 10 ? 32 : 64) : 64;
    static constexpr int NCH = WHOLE ? 64 / EC : S::NCHUNK;
    static constexpr int LDS_BYTES =
        PACKED ? 4 * 64 * S::NN * 4 : ((R > 0) ? 4 * EC * S::STR * 4 : 0);
    // Staged stores: non-temporal or plain per matrix size (nt_matrix_stores)
    static constexpr bool NT_STORES = nt_matrix_stores<T::N>();
    __device__ static void put(f32x4_t *dst, f32x4_t v)
    {
        if constexpr (NT_STORES) store_out(dst, v);
        else *dst = v;
    }

    struct In {             // connectivity of this lane's element
        int v[DIM + 1];
    };
    struct Xv {             // gathered vertex coordinates and coefficients
        CT x[DIM + 1][DIM];
        float mu, lam;
    };

    // Lanes past the last element (and whole tiles past the end) read the
    // last element and are masked in compute(): the loads carry no branch, so
    // the compiler need not wait for their data at a join, and a prefetch of
    // a tile that does not exist stays in bounds.
    //
    // Every stage takes e0, the first element of the wave's 64; lane l owns
    // element e0 + l.
    __device__ static int64_t clamp_elem(const FwdParams &p, int64_t e0)
    {
        const int64_t e = e0 + (threadIdx.x & 63), E = p.m.n_elements;
        return e < E ? e : E - 1;
    }

    __device__ static In load(const FwdParams &p, int64_t e0)
    {
        In in;
        load_conn<DIM>(p.m.conn, clamp_elem(p, e0), in.v);
        return in;
    }

    __device__ static Xv gather_xv(const FwdParams &p, int64_t e0, const In &in)
    {
        Xv g;
        gather<DIM>(p.m, in.v, g.x);
        g.mu = g.lam = 0.f;
        if constexpr (FORM == ELA1) {
            const int64_t ec = clamp_elem(p, e0);
            g.mu = __builtin_nontemporal_load(p.mu + ec);
            g.lam = __builtin_nontemporal_load(p.lam + ec);
        }
        return g;
    }

    __device__ static void compute(const FwdParams &p, int64_t e0, const Xv &g,
                                   float (&Au)[U::NU])
    {
        float Gf[T::G];
        bool flag = false, singular = false;
        if (e0 + (threadIdx.x & 63) < p.m.n_elements) {
            flag = geometry<FORM, DIM>(g.x, g.mu, g.lam, p.tau2, Gf, singular);
        } else {
#pragma unroll
            for (int k = 0; k < T::G; ++k) Gf[k] = 0.f;
        }
        count_flags(p.counters, flag, singular);
        unique_entries<FORM, DIM>(Gf, Au);
    }

    __device__ __forceinline__ static void store(const FwdParams &p, int64_t e0, const float (&Au)[U::NU],
                                 unsigned char *smem)
    {
        const int64_t E = p.m.n_elements;
        if constexpr (R == 0) {
            const int64_t e = e0 + (threadIdx.x & 63);
            if (e < E) contract_store<FORM, DIM>(Au, p.A + e * (int64_t)S::NN);
        } else if constexpr (PACKED) {
            // The wave's 64 matrices start at e0 * n * n floats, a multiple of
            // 64 * 9 * 4 bytes from the 16-byte aligned A: piece f of the run
            // is 16-byte aligned; pieces past the last element's end are
            // dropped, the one that straddles it is stored float by float.
            const int lane = threadIdx.x & 63, wave = wave_id();
            float *st = reinterpret_cast<float *>(smem) + wave * 64 * S::NN;
#pragma unroll
            for (int k = 0; k < S::NN; ++k) st[lane * S::NN + k] = Au[sym_index(S::N, k / S::N, k % S::N)];
            wave_sync();
            const int64_t left = E - e0;
            const int nvalid = left <= 0 ? 0 : (left >= 64 ? 64 * S::NN : int(left) * S::NN);
            constexpr int PIECES = 64 * S::NN / 4;
            float *dst = p.A + e0 * (int64_t)S::NN;
#pragma unroll
            for (int k = 0; k < (PIECES + 63) / 64; ++k) {
                const int f = lane + 64 * k;
                if (f < PIECES) {
                    if (4 * f + 4 <= nvalid) {
                        put(reinterpret_cast<f32x4_t *>(dst + 4 * f),
                            *reinterpret_cast<const f32x4_t *>(st + 4 * f));
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (4 * f + i < nvalid) dst[4 * f + i] = st[4 * f + i];
                    }
                }
            }
            wave_sync();
        } else {
            const int lane = threadIdx.x & 63, wave = wave_id();
            float *st = reinterpret_cast<float *>(smem) + wave * EC * S::STR;
            constexpr int PIECES = EC * S::NV4;     // 16-byte pieces per chunk
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int row0 = WHOLE ? 0 : c * S::CH;  // first flat entry of the chunk
                const int64_t eb = e0 + (WHOLE ? c * EC : 0);
                // this lane's chunk rows into its LDS row
                if (!WHOLE || lane / EC == c) {
                    float *row = st + (lane % EC) * S::STR;
#pragma unroll
                    for (int k = 0; k < S::CH; k += 4) {
                        f32x4_t r;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int flat = row0 + k + i;
                            r[i] = Au[sym_index(S::N, flat / S::N, flat % S::N)];
                        }
                        *reinterpret_cast<f32x4_t *>(row + k) = r;
                    }
                }
                wave_sync();
                // cooperative store of the chunk: piece f -> (element, part).
                // A whole-matrix chunk is one contiguous run, piece f at 4 f
                // floats from its start; a full chunk (wave-uniform test) reads
                // all its pieces first, then stores them without checks.
                float *dst = p.A + eb * (int64_t)S::NN + row0;
                constexpr int NP = (PIECES + 63) / 64;
                if (PIECES % 64 == 0 && eb + EC <= E) {
                    f32x4_t r[NP];
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const int f = lane + 64 * k;
                        const int el = f / S::NV4, part = f - el * S::NV4;
                        r[k] = *reinterpret_cast<const f32x4_t *>(st + el * S::STR + 4 * part);
                    }
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const int f = lane + 64 * k;
                        const int el = f / S::NV4, part = f - el * S::NV4;
                        put(reinterpret_cast<f32x4_t *>(dst + (WHOLE ? 4 * f : el * S::NN + 4 * part)),
                            r[k]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const int f = lane + 64 * k;
                        const int el = f / S::NV4, part = f - el * S::NV4;
                        if ((PIECES % 64 == 0 || f < PIECES) && eb + el < E) {
                            const f32x4_t r =
                                *reinterpret_cast<const f32x4_t *>(st + el * S::STR + 4 * part);
                            put(reinterpret_cast<f32x4_t *>(dst + el * S::NN + 4 * part), r);
                        }
                    }
                }
                wave_sync();
            }
        }
    }

    // The wave's 64 elements from e0 (LDS_BYTES / 4 bytes of smem per wave).
    __device__ __forceinline__ static void run_at(const FwdParams &p, int64_t e0, unsigned char *smem)
    {
        const Xv g = gather_xv(p, e0, load(p, e0));
        float Au[U::NU];
        compute(p, e0, g, Au);
        store(p, e0, Au, smem);
    }

    // The whole 256-element tile blk in order (batch kernels).
    __device__ __forceinline__ static void run(const FwdParams &p, int64_t blk, unsigned char *smem)
    {
        run_at(p, blk * 256 + wave_id() * 64, smem);
    }
};

// Tiles of a persistent workgroup: the tiles are split into contiguous
// ranges, one per XCD that has workgroups (workgroups are dispatched
// round-robin over the 8 XCDs), and the workgroups of an XCD stride through
// its range.  With G < 8 workgroups only XCDs 0..G-1 get a range.
struct PersistentTiles {
    int64_t begin, end, stride;
    __device__ PersistentTiles(int64_t n_tiles)
    {
        const int64_t G = gridDim.x, b = blockIdx.x;
        const int64_t X = G < 8 ? G : 8;
        const int64_t x = b % 8, i = b / 8;
        const int64_t cnt = G / 8 + (x < G % 8 ? 1 : 0);
        const int64_t r0 = x * n_tiles / X, r1 = (x + 1) * n_tiles / X;
        begin = r0 + i;
        end = r1;
        stride = cnt;
    }
};

// FP32 forward: one workgroup per 256-element tile, tiles remapped so that
// each XCD integrates one contiguous range of elements (its L2 then holds the
// shared vertices, and each XCD's stores sweep one region of A).  Several
// workgroups are resident per CU (the whole-matrix staging keeps LDS at or
// below 76 KB), so the hardware overlaps one workgroup's gathers and
// contraction with another's stores; measured faster on MI355X than a
// persistent, software-pipelined loop over tiles with one wave per SIMD.
//
// WAVES: waves per workgroup (64 WAVES elements per workgroup; the paper's
// element batch size, Sec. 4, a tuning axis: 4 by default).
template <int FORM, int DIM, typename CT, int R, int WAVES = 4>
__global__ __launch_bounds__(64 * WAVES) void fwd_fma_kernel(FwdParams p)
{
    using Tile = FwdFmaTile<FORM, DIM, CT, R>;
    constexpr int LDS = Tile::LDS_BYTES / 4 * WAVES;
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS > 0 ? LDS : 16];
    Tile::run_at(p, xcd_block(blockIdx.x, gridDim.x) * (64 * WAVES) + wave_id() * 64, smem);
}

}  // namespace fei

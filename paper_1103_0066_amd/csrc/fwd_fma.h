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
// for every lane of the grid, so it lives in a __constant__ table and reaches
// the lanes through the scalar data cache as SGPR operands of v_fma_f32: a
// wave-uniform broadcast is what the scalar unit exists for, and it leaves
// LDS free for the output.
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

// Block reference tensors, one per (form, dim), in mutable __constant__
// memory, so the kernels read K at run time rather than folding it into code.
// The specializations holding the values are generated at build time.
template <int FORM, int DIM>
__constant__ KBlockTable<FORM, DIM> c_kblock;

template <int FORM, int DIM>
__device__ __forceinline__ float kval(int i, int j, int mu, int nu)
{
    using T = Traits<FORM, DIM>;
    return c_kblock<FORM, DIM>.v[((i * T::NB + j) * DIM + mu) * DIM + nu];
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
        for (int nu = 0; nu < DIM; ++nu)
            acc = fmaf(kval<FORM, DIM>(a, b, mu, nu),
                       Gf[sym_index(T::GD, mu * T::NC + c, nu * T::NC + d)], acc);
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
    static_assert(R == 0 || (N % R == 0 && CH % 4 == 0), "bad chunk");
};

// Orders this wave's LDS accesses around a point (the LDS executes one
// wave's operations in issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup tile (256 elements, 4 waves) of the FP32 forward.  LDS comes
// from the caller (LDS_BYTES, 16-byte aligned), so one persistent kernel can
// host the tiles of several forms.
template <int FORM, int DIM, typename CT, int R>
struct FwdFmaTile {
    using T = Traits<FORM, DIM>;
    using S = Stage<FORM, DIM, R>;
    static constexpr int LDS_BYTES = (R > 0) ? 4 * 64 * S::STR * 4 : 0;

    __device__ static void run(const FwdParams &p, int64_t blk, unsigned char *smem)
    {
        const int64_t E = p.m.n_elements;
        const int64_t e = blk * 256 + threadIdx.x;
        if constexpr (R == 0) {
            if (e >= E) return;
        }
        const bool valid = e < E;
        float Gf[T::G];
        bool flag = false, singular = false;
        if (valid) {
            int v[DIM + 1];
            load_conn<DIM>(p.m.conn, e, v);
            CT xv[DIM + 1][DIM];
            gather<DIM>(p.m, v, xv);
            float mu = 0.f, lam = 0.f;
            if constexpr (FORM == ELA1) {
                mu = __builtin_nontemporal_load(p.mu + e);
                lam = __builtin_nontemporal_load(p.lam + e);
            }
            flag = geometry<FORM, DIM>(xv, mu, lam, p.tau2, Gf, singular);
        } else {
#pragma unroll
            for (int g = 0; g < T::G; ++g) Gf[g] = 0.f;
        }
        count_flags(p.counters, flag, singular);
        float Au[Unique<FORM, DIM>::NU];
        unique_entries<FORM, DIM>(Gf, Au);

        if constexpr (R == 0) {
            contract_store<FORM, DIM>(Au, p.A + e * (int64_t)S::NN);
        } else {
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            float *st = reinterpret_cast<float *>(smem) + wave * 64 * S::STR;
            const int64_t e0 = blk * 256 + wave * 64;
#pragma unroll
            for (int c = 0; c < S::NCHUNK; ++c) {
                // this lane's R rows into its LDS row
#pragma unroll
                for (int k = 0; k < S::CH; k += 4) {
                    f32x4_t r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int flat = c * S::CH + k + i;
                        r[i] = Au[sym_index(S::N, flat / S::N, flat % S::N)];
                    }
                    *reinterpret_cast<f32x4_t *>(st + lane * S::STR + k) = r;
                }
                wave_sync();
                // cooperative store of the wave's chunk: piece f -> (element, part)
#pragma unroll
                for (int k = 0; k < S::NV4; ++k) {
                    const int f = lane + 64 * k;
                    const int el = f / S::NV4, part = f - el * S::NV4;
                    const f32x4_t r =
                        *reinterpret_cast<const f32x4_t *>(st + el * S::STR + 4 * part);
                    if (e0 + el < E)
                        store_out(reinterpret_cast<f32x4_t *>(p.A + (e0 + el) * (int64_t)S::NN +
                                                              c * S::CH + 4 * part), r);
                }
                wave_sync();
            }
        }
    }
};

template <int FORM, int DIM, typename CT, int R>
__global__ __launch_bounds__(256) void fwd_fma_kernel(FwdParams p)
{
    using Tile = FwdFmaTile<FORM, DIM, CT, R>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Tile::LDS_BYTES > 0 ? Tile::LDS_BYTES : 16];
    Tile::run(p, xcd_block(blockIdx.x, gridDim.x), smem);
}

}  // namespace fei

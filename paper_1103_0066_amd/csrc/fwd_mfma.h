// Forward element integration, split-precision MFMA form.
//
// The contraction of eq. 1 over a batch of elements is a dense product
//   A^T[entries][elements] = Kf^T[entries][g] * Gf^T[g][elements],
// g the unique entries of the symmetric geometric tensor.  Gf is split into
// two (FP16 or BF16) or three (BF16) terms, concatenated along the reduction
// axis, and multiplied by the same integer K stacked two or three times:
//   [Gf_hi | Gf_lo (| Gf_lo2)] . [Kf; Kf (; Kf)]
// with v_mfma_f32_16x16x32_{f16,bf16} accumulating in FP32.  The integer Kf
// is exact in both 16-bit formats, so only G carries split error.  FP16 uses
// a per-element power-of-two scale (max |Gf * 2^-E| in [1/2, 1)) that is
// undone exactly on the FP32 result.
//
// Workgroup = 4 waves = 256 elements.  Phase 1 is the FP32 path's geometry,
// one lane per element, writing the split Gf row of its element into LDS.
// Phase 2: each wave multiplies its 64 elements as 4 groups of 16 MFMA
// columns.  The K fragments (the MFMA A operand) are precomputed at build
// time in lane order and held in registers (staged in LDS once per workgroup
// if they would not fit).  The MFMA output
// puts 4 consecutive entries of one element in each lane, which are stored
// as one 16-byte vector (64 contiguous bytes per element per M tile).
#pragma once

#include "fwd_fma.h"

namespace fei {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// K fragments per (form, dim, precision); values generated at build time.
template <int FORM, int DIM, int PREC>
__device__ FragTable<FORM, DIM, PREC> g_frags;

__device__ __forceinline__ uint16_t f16_bits(_Float16 h) { return __builtin_bit_cast(uint16_t, h); }
__device__ __forceinline__ uint16_t bf16_bits(__bf16 h) { return __builtin_bit_cast(uint16_t, h); }

template <int PREC>
__device__ __forceinline__ floatx4_t mfma_step(const uint4 &a, const uint4 &b, floatx4_t acc)
{
    if constexpr (PREC == P_FP16X2) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a),
                                                      __builtin_bit_cast(half8_t, b), acc, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), acc, 0, 0, 0);
    }
}

// Split one element's Gf into a register row of KT 16-bit values and copy it
// to the element's LDS row with 16-byte stores; returns the FP16 scale exponent.
template <int FORM, int DIM, int PREC>
__device__ __forceinline__ int split_gf(const float (&Gf)[Traits<FORM, DIM>::G],
                                        uint16_t *__restrict__ lds_row)
{
    using T = Traits<FORM, DIM>;
    using S = MfmaShape<FORM, DIM, PREC>;
    uint16_t row[S::KT];
    int E = 0;
    if constexpr (PREC == P_FP16X2) {
        float mx = 0.f;
#pragma unroll
        for (int g = 0; g < T::G; ++g) mx = fmaxf(mx, fabsf(Gf[g]));
        (void)frexpf(mx, &E);
        if (!(mx < __builtin_huge_valf())) E = 0;  // Inf / NaN: leave unscaled
#pragma unroll
        for (int g = 0; g < T::G; ++g) {
            const float x = ldexpf(Gf[g], -E);
            const _Float16 hi = (_Float16)x;
            const _Float16 lo = (_Float16)(x - (float)hi);
            row[g] = f16_bits(hi);
            row[T::G + g] = f16_bits(lo);
        }
    } else {
#pragma unroll
        for (int g = 0; g < T::G; ++g) {
            const float x = Gf[g];
            const __bf16 hi = (__bf16)x;
            const float r1 = x - (float)hi;
            const __bf16 mid = (__bf16)r1;
            row[g] = bf16_bits(hi);
            row[T::G + g] = bf16_bits(mid);
            if constexpr (PREC == P_BF16X3) row[2 * T::G + g] = bf16_bits((__bf16)(r1 - (float)mid));
        }
    }
#pragma unroll
    for (int k = T::G * S::NSPLIT; k < S::KT; ++k) row[k] = 0;
#pragma unroll
    for (int k = 0; k < S::KT; k += 8) {
        uint4 w;
        w.x = unsigned(row[k + 0]) | (unsigned(row[k + 1]) << 16);
        w.y = unsigned(row[k + 2]) | (unsigned(row[k + 3]) << 16);
        w.z = unsigned(row[k + 4]) | (unsigned(row[k + 5]) << 16);
        w.w = unsigned(row[k + 6]) | (unsigned(row[k + 7]) << 16);
        *reinterpret_cast<uint4 *>(lds_row + k) = w;
    }
    return E;
}

// LDS layout of the MFMA kernel: per wave, the split-Gf rows of its 64
// elements (B operand source), later reused to stage 16 elements' matrices.
template <int FORM, int DIM, int PREC>
struct MfmaLds {
    using S = MfmaShape<FORM, DIM, PREC>;
    static constexpr bool STAGED = (S::NN % 4 == 0);
    static constexpr int OSTR = S::NN + 4;                    // staged row stride (floats)
    static constexpr int BBYTES = 64 * S::BROW * 2;           // split-Gf rows of a wave
    static constexpr int OBYTES = STAGED ? 16 * OSTR * 4 : 0;  // 16 staged matrices
    static constexpr int WBYTES = ((BBYTES > OBYTES ? BBYTES : OBYTES) + 15) / 16 * 16;
    // K fragments live in registers when they take at most 192 VGPRs (all the
    // forms here; measured faster than LDS-staged fragments), else in LDS
    static constexpr bool AREG = S::MT * S::KS <= 48;
};

// One workgroup tile (256 elements, 4 waves) of the MFMA forward.  Waves only
// touch their own LDS rows, so the phases are ordered per wave, not per
// workgroup; the K fragments are loaded once per workgroup (load_frags) and
// reused for every tile it processes.
template <int FORM, int DIM, typename CT, int PREC, bool DIRECT>
struct MfmaTile {
    using T = Traits<FORM, DIM>;
    using S = MfmaShape<FORM, DIM, PREC>;
    using L = MfmaLds<FORM, DIM, PREC>;
    static constexpr int FRAG_BYTES = L::AREG ? 0 : S::NFRAG * 16;
    // non-temporal or plain stores per matrix size, as in the FP32 form
    __device__ static void put(f32x4_t *dst, f32x4_t v)
    {
        if constexpr (nt_matrix_stores<T::N>()) store_out(dst, v);
        else *dst = v;
    }
    static constexpr int LDS_BYTES = FRAG_BYTES + 4 * L::WBYTES + 256 * 4;

    struct Frags {
        uint4 v[L::AREG ? S::MT * S::KS : 1];
    };

    // K fragments into registers, or (too many for registers) into LDS with a
    // workgroup barrier; call once per workgroup before run().
    __device__ static void load_frags(Frags &a, unsigned char *smem)
    {
        const uint4 *gfr = reinterpret_cast<const uint4 *>(g_frags<FORM, DIM, PREC>.v);
        if constexpr (L::AREG) {
            const int lane = threadIdx.x & 63;
#pragma unroll
            for (int i = 0; i < S::MT * S::KS; ++i) a.v[i] = gfr[i * 64 + lane];
        } else {
            uint4 *s_frag = reinterpret_cast<uint4 *>(smem);
            for (int i = threadIdx.x; i < S::NFRAG; i += 256) s_frag[i] = gfr[i];
            __syncthreads();
        }
    }

    __device__ static uint4 frag(const Frags &a, const unsigned char *smem, int t, int s)
    {
        if constexpr (L::AREG) return a.v[t * S::KS + s];
        else return reinterpret_cast<const uint4 *>(smem)[(t * S::KS + s) * 64 + (threadIdx.x & 63)];
    }

    // LDS: [K fragments] | per-wave split-Gf rows / output staging | FP16 exponents
    __device__ __forceinline__ static void run(const FwdParams &p, int64_t blk, unsigned char *smem, const Frags &a)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        unsigned char *s_wave_w = smem + FRAG_BYTES + wave * L::WBYTES;
        uint16_t *s_b = reinterpret_cast<uint16_t *>(s_wave_w);
        int *s_exp = reinterpret_cast<int *>(smem + FRAG_BYTES + 4 * L::WBYTES) + wave * 64;
        const int64_t e0 = blk * 256 + wave * 64;
        const int64_t E = p.m.n_elements;

        // phase 1: geometry, one lane per element, split Gf into this wave's rows
        {
            const int64_t e = e0 + lane;
            float Gf[T::G];
            bool flag = false, singular = false;
            if (e < E) {
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
            s_exp[lane] = split_gf<FORM, DIM, PREC>(Gf, s_b + lane * S::BROW);
        }
        wave_sync();

        // phase 2: the wave's 64 elements as 4 MFMA column groups of 16
        const int n = lane & 15, q = lane >> 4;
        uint4 bf[4][S::KS];
        int ex[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int el = g * 16 + n;
#pragma unroll
            for (int s = 0; s < S::KS; ++s)
                bf[g][s] = *reinterpret_cast<const uint4 *>(s_b + el * S::BROW + 32 * s + 8 * q);
            ex[g] = s_exp[el];
        }
        wave_sync();  // the B fragments have been read; the rows may be reused
        if constexpr (DIRECT || !L::STAGED) {
            // each lane stores its 4 consecutive entries of one element per M tile
#pragma unroll
            for (int t = 0; t < S::MT; ++t) {
                floatx4_t acc[4];
#pragma unroll
                for (int g = 0; g < 4; ++g) acc[g] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < S::KS; ++s) {
                    const uint4 af = frag(a, smem, t, s);
#pragma unroll
                    for (int g = 0; g < 4; ++g) acc[g] = mfma_step<PREC>(af, bf[g][s], acc[g]);
                }
                const int m0 = 16 * t + 4 * q;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t e = e0 + g * 16 + n;
                    if (e >= E) continue;
                    floatx4_t r = acc[g];
                    if constexpr (PREC == P_FP16X2) {
                        r[0] = ldexpf(r[0], ex[g]); r[1] = ldexpf(r[1], ex[g]);
                        r[2] = ldexpf(r[2], ex[g]); r[3] = ldexpf(r[3], ex[g]);
                    }
                    float *Ae = p.A + e * (int64_t)S::NN;
                    if constexpr (S::NN % 4 == 0) {
                        if (m0 < S::NN)
                            put(reinterpret_cast<f32x4_t *>(Ae + m0), r);
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (m0 + i < S::NN) Ae[m0 + i] = r[i];
                    }
                }
            }
        } else {
            // per column group: all M tiles into LDS, then contiguous 16-byte stores
            float *so = reinterpret_cast<float *>(s_wave_w);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
#pragma unroll
                for (int t = 0; t < S::MT; ++t) {
                    floatx4_t acc = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < S::KS; ++s)
                        acc = mfma_step<PREC>(frag(a, smem, t, s), bf[g][s], acc);
                    const int m0 = 16 * t + 4 * q;
                    if constexpr (PREC == P_FP16X2) {
                        acc[0] = ldexpf(acc[0], ex[g]); acc[1] = ldexpf(acc[1], ex[g]);
                        acc[2] = ldexpf(acc[2], ex[g]); acc[3] = ldexpf(acc[3], ex[g]);
                    }
                    if (m0 < S::NN)
                        *reinterpret_cast<floatx4_t *>(so + n * L::OSTR + m0) = acc;
                }
                wave_sync();
                constexpr int NV4 = S::NN / 4;  // 16-byte pieces per element
                const int64_t eg = e0 + g * 16;
                float *dst = p.A + eg * (int64_t)S::NN;
#pragma unroll
                for (int k = 0; k < (16 * NV4 + 63) / 64; ++k) {
                    const int f = lane + 64 * k;
                    if (f >= 16 * NV4) break;
                    const int el = f / NV4, part = f - el * NV4;
                    const floatx4_t r =
                        *reinterpret_cast<const floatx4_t *>(so + el * L::OSTR + 4 * part);
                    if (eg + el < E) put(reinterpret_cast<f32x4_t *>(dst + 4 * f), r);
                }
                wave_sync();
            }
        }
    }

    // One tile without preloaded fragments (batch kernels).
    __device__ __forceinline__ static void run(const FwdParams &p, int64_t blk, unsigned char *smem)
    {
        Frags a;
        load_frags(a, smem);
        run(p, blk, smem, a);
    }
};

// PERSISTENT: a grid of resident workgroups loops over the tiles (split per
// XCD), loading the K fragments once; otherwise one workgroup per tile
// (tiles remapped per XCD).
template <int FORM, int DIM, typename CT, int PREC, bool DIRECT, bool PERSISTENT>
__global__ __launch_bounds__(256) void fwd_mfma_kernel(FwdParams p, int64_t n_tiles)
{
    using Tile = MfmaTile<FORM, DIM, CT, PREC, DIRECT>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Tile::LDS_BYTES];
    typename Tile::Frags a;
    Tile::load_frags(a, smem);
    if constexpr (PERSISTENT) {
        const PersistentTiles pt(n_tiles);
        for (int64_t t = pt.begin; t < pt.end; t += pt.stride) Tile::run(p, t, smem, a);
    } else {
        Tile::run(p, xcd_block(blockIdx.x, gridDim.x), smem, a);
    }
}

}  // namespace fei

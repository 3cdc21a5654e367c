// Compile-time shapes shared by the kernels and the table generator: MFMA
// tiling of the folded contraction, 16-bit encodings of small integers and
// the pair index of symmetric tensors.  Host and device.
#pragma once

#include "reftensor.h"

namespace fei {

enum Prec { P_FP32 = 0, P_FP16X2 = 1, P_BF16X2 = 2, P_BF16X3 = 3 };

// MFMA form of A^T[entries][elements] = Kf^T[entries][g] Gf^T[g][elements]
// with 16x16x32 tiles: M = entries (MT tiles), K = split Gf (KS steps of 32).
template <int FORM, int DIM, int PREC>
struct MfmaShape {
    using T = Traits<FORM, DIM>;
    static constexpr int NSPLIT = (PREC == P_BF16X3) ? 3 : 2;
    static constexpr int KT = ((T::G * NSPLIT + 31) / 32) * 32;  // padded reduction length
    static constexpr int KS = KT / 32;                           // MFMA k-steps
    static constexpr int NN = T::N * T::N;
    static constexpr int MT = (NN + 15) / 16;                    // M tiles of 16 entries
    static constexpr int NFRAG = MT * KS * 64;                   // 16-byte lane fragments
    static constexpr int BROW = KT + 8;                          // LDS row (halfs), padded
};

// MFMA form of the adjoint's fold U^T[g][elements] = Kf[g][ij] dA^T[ij][elements]
// with 16x16x32 tiles: M = unique pairs g (MT tiles), K = element-matrix
// entries ij (KS steps of 32).  The split terms of dA are separate products
// with the same A fragments.
template <int FORM, int DIM>
struct MfmaAdjShape {
    using T = Traits<FORM, DIM>;
    static constexpr int NN = T::N * T::N;
    static constexpr int MT = (T::G + 15) / 16;
    static constexpr int KS = (NN + 31) / 32;
    static constexpr int NFRAG = MT * KS * 64;
};

// Block reference tensor [NB][NB][DIM][DIM] (integer values, as float).
template <int FORM, int DIM>
struct KBlockTable {
    float v[Traits<FORM, DIM>::NB * Traits<FORM, DIM>::NB * DIM * DIM];
};

// K fragments of the MFMA A operand in lane order: fragment
// f = (t*KS + s)*64 + lane holds A[m][32 s + 8 (lane/16) + j], j = 0..7, with
// m = 16 t + lane % 16 and A[m][k] = Kf[k mod g][m] for k < g*NSPLIT, else 0.
template <int FORM, int DIM, int PREC>
struct FragTable {
    uint16_t v[MfmaShape<FORM, DIM, PREC>::NFRAG * 8];
};

// Adjoint fragments in lane order: fragment f = (t*KS + s)*64 + lane holds
// A[m][32 s + 8 (lane/16) + j], j = 0..7, with m = 16 t + lane % 16 and
// A[m][ij] = Kf[m][ij] for m < G and ij < n*n, else 0.  PREC is P_FP16X2 or
// P_BF16X2 (the encoding; BF16x3 uses the BF16 table).
template <int FORM, int DIM, int PREC>
struct AdjFragTable {
    uint16_t v[MfmaAdjShape<FORM, DIM>::NFRAG * 8];
};

// Sparse rows of the folded tensor: for every unique pair g the nonzero
// entries (flat element-matrix index, integer coefficient), padded with
// zero coefficients to NNZ.  U_g = sum_t coef[g][t] * dA[ij[g][t]] is the
// folded K^T applied to dA.
// Coefficient reference tensor [NB][NB][NV][DIM][DIM] (integer values, as float).
template <int FORM, int DIM>
struct KWTable {
    float v[Traits<FORM, DIM>::NB * Traits<FORM, DIM>::NB * (DIM + 1) * DIM * DIM];
};

template <int FORM, int DIM>
struct KSparseShape {
    static constexpr int NNZ = (FORM == LAP2) ? ((DIM == 3) ? 72 : 32) : 8;
};

template <int FORM, int DIM>
struct KSparse {
    int16_t ij[Traits<FORM, DIM>::G][KSparseShape<FORM, DIM>::NNZ];
    float coef[Traits<FORM, DIM>::G][KSparseShape<FORM, DIM>::NNZ];
};

// Isoparametric P2 Laplacian (Sec. 3.1, eqs. 16-19): quadratic geometry and
// basis (NB nodes), the inverse Jacobian projected on the NV vertex functions.
// G^{(k mu),(l nu)} pairs p = k DIM + mu (GD of them, G unique); unique entries
// (i <= j) of the NB x NB element matrix: NU.
template <int DIM>
struct IsoShape {
    static constexpr int NV = DIM + 1;
    static constexpr int NB = (DIM + 1) * (DIM + 2) / 2;
    static constexpr int GD = NV * DIM;
    static constexpr int G = GD * (GD + 1) / 2;
    static constexpr int NU = NB * (NB + 1) / 2;
};

// Folded arity-4 reference tensor: v[u * G + g] for unique entry u = (i <= j)
// and unique pair g = (p <= q), integers over a common denominator; the
// tensor is v * scale.
template <int DIM>
struct KIsoTable {
    float v[IsoShape<DIM>::NU * IsoShape<DIM>::G];
    double scale;
};

FEI_HD constexpr void sym_pair(int gd, int gamma, int &p, int &q)
{
    for (int i = 0; i < gd; ++i)
        for (int j = i; j < gd; ++j)
            if (sym_index(gd, i, j) == gamma) { p = i; q = j; return; }
    p = q = 0;
}

// 16-bit encodings of integers exactly representable in the format.
inline uint16_t f16_bits_of_int(int v)
{
    if (v == 0) return 0;
    unsigned s = v < 0 ? 1u : 0u;
    unsigned a = v < 0 ? unsigned(-v) : unsigned(v);
    int e = 0;
    while ((a >> (e + 1)) != 0) ++e;
    unsigned mant = (e <= 10) ? ((a << (10 - e)) & 0x3FFu) : ((a >> (e - 10)) & 0x3FFu);
    return uint16_t((s << 15) | (unsigned(e + 15) << 10) | mant);
}

inline uint16_t bf16_bits_of_int(int v)
{
    if (v == 0) return 0;
    unsigned s = v < 0 ? 1u : 0u;
    unsigned a = v < 0 ? unsigned(-v) : unsigned(v);
    int e = 0;
    while ((a >> (e + 1)) != 0) ++e;
    unsigned mant = (e <= 7) ? ((a << (7 - e)) & 0x7Fu) : ((a >> (e - 7)) & 0x7Fu);
    return uint16_t((s << 15) | (unsigned(e + 127) << 7) | mant);
}

}  // namespace fei

// Build-time generator of the reference-tensor tables compiled into the
// kernels: for every (form, dim) the block tensor K (eq. 7, integer-scaled),
// and for every MFMA precision the K fragments in lane order.  Writes C++
// source to stdout.  Uses only reftensor.h / shapes.h, so the host API
// (fei_reference_tensor) and the kernels see the same K.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "polyint.h"
#include "shapes.h"

using namespace fei;

static const char *sep(int n) { return n == 0 ? "\n    " : (n % 16 ? ", " : ",\n    "); }

template <int F, int D>
static void emit_block()
{
    using T = Traits<F, D>;
    std::printf("template <> struct KFold<%d, %d> {\n"
                "    static constexpr KBlockTable<%d, %d> t = {{", F, D, F, D);
    int n = 0;
    for (int i = 0; i < T::NB; ++i)
        for (int j = 0; j < T::NB; ++j)
            for (int mu = 0; mu < D; ++mu)
                for (int nu = 0; nu < D; ++nu) {
                    int v = kblock(F, D, i, j, mu, nu);
                    std::printf("%s%d.f", sep(n++), v);
                }
    std::printf("}};\n};\n");
}

template <int F, int D>
static void emit_coefficient()
{
    using T = Traits<F, D>;
    std::printf("template <> struct KWFold<%d, %d> {\n"
                "    static constexpr KWTable<%d, %d> t = {{", F, D, F, D);
    int n = 0;
    for (int i = 0; i < T::NB; ++i)
        for (int j = 0; j < T::NB; ++j)
            for (int m = 0; m <= D; ++m)
                for (int mu = 0; mu < D; ++mu)
                    for (int nu = 0; nu < D; ++nu)
                        std::printf("%s%d.f", sep(n++), kwblock(F, D, i, j, m, mu, nu));
    std::printf("}};\n};\n");
}

template <int F, int D, int P>
static void emit_frags()
{
    using T = Traits<F, D>;
    using S = MfmaShape<F, D, P>;
    int pp[T::G], qq[T::G];
    for (int g = 0; g < T::G; ++g) sym_pair(T::GD, g, pp[g], qq[g]);
    std::printf("template <> __device__ FragTable<%d, %d, %d> g_frags<%d, %d, %d> = {{",
                F, D, P, F, D, P);
    int n = 0;
    for (int t = 0; t < S::MT; ++t)
        for (int s = 0; s < S::KS; ++s)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int m = 16 * t + lane % 16;
                    const int k = 32 * s + 8 * (lane / 16) + j;
                    int val = 0;
                    if (m < S::NN && k < T::G * S::NSPLIT) {
                        const int g = k % T::G;
                        val = kfolded(F, D, pp[g], qq[g], m / T::N, m % T::N);
                    }
                    if ((P == P_FP16X2 && (val > 2048 || val < -2048)) ||
                        (P != P_FP16X2 && (val > 256 || val < -256))) {
                        std::fprintf(stderr, "K entry %d not exact in 16 bits\n", val);
                        std::exit(1);
                    }
                    const unsigned bits =
                        (P == P_FP16X2) ? f16_bits_of_int(val) : bf16_bits_of_int(val);
                    std::printf("%s0x%04x", sep(n++), bits);
                }
    std::printf("}};\n");
}

// A fragments of the adjoint's MFMA fold (the transpose of the forward's
// operand, without the split stacking).
template <int F, int D, int P>
static void emit_adj_frags()
{
    using T = Traits<F, D>;
    using S = MfmaAdjShape<F, D>;
    std::printf("template <> __device__ AdjFragTable<%d, %d, %d> g_adj_frags<%d, %d, %d> = {{",
                F, D, P, F, D, P);
    int n = 0;
    for (int t = 0; t < S::MT; ++t)
        for (int s = 0; s < S::KS; ++s)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int m = 16 * t + lane % 16;
                    const int k = 32 * s + 8 * (lane / 16) + j;
                    int val = 0;
                    if (m < T::G && k < S::NN) {
                        int p = 0, q = 0;
                        sym_pair(T::GD, m, p, q);
                        val = kfolded(F, D, p, q, k / T::N, k % T::N);
                    }
                    if ((P == P_FP16X2 && (val > 2048 || val < -2048)) ||
                        (P != P_FP16X2 && (val > 256 || val < -256))) {
                        std::fprintf(stderr, "K entry %d not exact in 16 bits\n", val);
                        std::exit(1);
                    }
                    const unsigned bits =
                        (P == P_FP16X2) ? f16_bits_of_int(val) : bf16_bits_of_int(val);
                    std::printf("%s0x%04x", sep(n++), bits);
                }
    std::printf("}};\n");
}

template <int F, int D>
static void emit_sparse()
{
    using T = Traits<F, D>;
    constexpr int NNZ = KSparseShape<F, D>::NNZ;
    std::vector<int> ij, cf;
    for (int g = 0; g < T::G; ++g) {
        int p = 0, q = 0;
        sym_pair(T::GD, g, p, q);
        int cnt = 0;
        for (int I = 0; I < T::N; ++I)
            for (int J = 0; J < T::N; ++J) {
                const int v = kfolded(F, D, p, q, I, J);
                if (v == 0) continue;
                if (cnt == NNZ) {
                    std::fprintf(stderr, "sparse row %d of form %d/%d exceeds %d\n", g, F, D, NNZ);
                    std::exit(1);
                }
                ij.push_back(I * T::N + J);
                cf.push_back(v);
                ++cnt;
            }
        for (; cnt < NNZ; ++cnt) {
            ij.push_back(0);
            cf.push_back(0);
        }
    }
    std::printf("template <> __device__ KSparse<%d, %d> g_ksparse<%d, %d> = {{", F, D, F, D);
    for (size_t i = 0; i < ij.size(); ++i)
        std::printf("%s%d", sep(int(i)), ij[i]);
    std::printf("}, {");
    for (size_t i = 0; i < cf.size(); ++i)
        std::printf("%s%d.f", sep(int(i)), cf[i]);
    std::printf("}};\n");
}

template <int F, int D>
static void emit_form()
{
    emit_block<F, D>();
    emit_sparse<F, D>();
    emit_frags<F, D, P_FP16X2>();
    emit_frags<F, D, P_BF16X2>();
    emit_frags<F, D, P_BF16X3>();
    emit_adj_frags<F, D, P_FP16X2>();
    emit_adj_frags<F, D, P_BF16X2>();
}

// Isoparametric P2 Laplacian: K^{ijkl}_{mu nu} = int_ref lambda_k dphi_i/dxi_mu
// lambda_l dphi_j/dxi_nu (eq. 18, the inverse Jacobian projected on the vertex
// functions lambda_k), exactly, folded over the symmetric pairs of G:
// Kf[(i,j)][(p,q)] = K_ij^{pq} + [p != q] K_ij^{qp}, as integers over their
// common denominator.
template <int D>
static void emit_iso()
{
    using S = IsoShape<D>;
    using namespace fei::poly;
    const std::vector<Poly> B = lagrange_basis(D, 2);
    std::vector<Poly> P(size_t(S::GD) * S::NB);           // [p = k D + mu][i]
    for (int k = 0; k < S::NV; ++k) {
        Poly lk;
        Mono m{};
        m[k] = 1;
        add_term(lk, m, Rat(1));
        for (int mu = 0; mu < D; ++mu)
            for (int i = 0; i < S::NB; ++i) P[size_t(k * D + mu) * S::NB + i] = mul(lk, dxi(B[i], mu));
    }
    auto K = [&](int i, int j, int p, int q) {
        return integrate_ref(mul(P[size_t(p) * S::NB + i], P[size_t(q) * S::NB + j]), D);
    };
    std::vector<Rat> Kf(size_t(S::NU) * S::G);
    int64_t lcd = 1;
    for (int i = 0; i < S::NB; ++i)
        for (int j = i; j < S::NB; ++j)
            for (int p = 0; p < S::GD; ++p)
                for (int q = p; q < S::GD; ++q) {
                    Rat v = K(i, j, p, q);
                    if (p != q) v = v + K(i, j, q, p);
                    Kf[size_t(sym_index(S::NB, i, j)) * S::G + sym_index(S::GD, p, q)] = v;
                    lcd = lcd / std::gcd(lcd, v.q) * v.q;
                }
    std::printf("template <> struct KIsoFold<%d> {\n"
                "    static constexpr KIsoTable<%d> t = {{", D, D);
    int n = 0;
    for (const Rat &v : Kf) {
        const int64_t iv = v.p * (lcd / v.q);
        if (iv >= (int64_t(1) << 24) || -iv >= (int64_t(1) << 24)) {
            std::fprintf(stderr, "isoparametric K entry %lld not exact in FP32\n", (long long)iv);
            std::exit(1);
        }
        std::printf("%s%lld.f", sep(n++), (long long)iv);
    }
    std::printf("}, %.17g};\n};\n", 1.0 / double(lcd));
}

int main()
{
    std::printf("// Generated by gen_tables.cpp at build time. Do not edit.\n");
    std::printf("namespace fei {\n");
    emit_form<LAP1, 2>();
    emit_form<LAP1, 3>();
    emit_form<ELA1, 2>();
    emit_form<ELA1, 3>();
    emit_form<LAP2, 2>();
    emit_form<LAP2, 3>();
    emit_coefficient<WLAP1, 2>();
    emit_coefficient<WLAP1, 3>();
    emit_coefficient<WLAP2, 2>();
    emit_coefficient<WLAP2, 3>();
    emit_iso<2>();
    emit_iso<3>();
    std::printf("}  // namespace fei\n");
    return 0;
}

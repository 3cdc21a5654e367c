// Element matrices of a general bilinear form of Lagrange elements, described
// at run time (the forms a form language describes, Sec. 3.2), as the
// contraction of Sec. 3, eq. 1 with a reference tensor over values and
// reference derivatives:
//
//   A_{(i,c),(j,d)} = sum_{p,q} G_{(p,c),(q,d)} Khat_ij^{pq},
//   Khat_ij^{pq}    = int_ref Dhat_p phi_i Dhat_q phi_j        (eq. 7, extended to values)
//   G               = |J| That^T C_e That,   C_e = W_0 + sum_k coef_k(e) W_k
//
// with Dhat_0 the value, Dhat_{1+mu} = d/dxi_mu, and That the map from
// physical to reference derivatives, block-diagonal over components:
// That[0][0] = 1, That[1+alpha][1+mu] = (J^-1)_{mu alpha} (eq. 8's
// J^-1 factors, one per derivative).  W (the form's operator tables, from the
// form front end) and Khat are the same for every element: the kernel reads
// them with uniform addresses known at compile time, so they arrive through
// the scalar cache as SGPR operands; C_e, J^-1 and |J| are per element.
//
// One lane per element.  Symmetric forms whose order n is that of a built-in
// form (3, 4, 6, 10, 12) form the n(n+1)/2 distinct entries and leave through
// the FP32 forward's whole-matrix staging (each staged chunk one contiguous
// run of matrices); the others produce rows RC at a time (RC*n floats in
// registers), staged in LDS for the wave's 64 elements and stored with
// consecutive lanes on consecutive 16-byte pieces.  Elements flagged by the
// quality test build G in FP64.
#pragma once

#include <utility>

#include "fwd_fma.h"

namespace fei {

// The form's tables (W, Khat) are the same for every element and never
// written by the kernel: read through the constant address space, so the
// uniform loads go through the scalar cache into SGPRs.
typedef const __attribute__((address_space(4))) float form_tab_t;

// Where a kernel reads the form's tables: the generic kernel reads them at
// run time (FormTabRuntime); a kernel generated for one form (fei_form_compile)
// has them as compile-time constants (CONST), so its zero entries drop out of
// the G build and the contraction and its coefficient count is fixed.
struct FormTabRuntime {
    static constexpr bool CONST = false;
    __device__ static float w(const FormParams &p, int i) { return ((form_tab_t *)p.W)[i]; }
    __device__ static float k(const FormParams &p, int i) { return ((form_tab_t *)p.K)[i]; }
    __device__ static int n_coef(const FormParams &p) { return p.n_coef; }
};

template <int DIM, int DEG, int NC, bool NOVAL = false>
struct FormShape {
    // operators kept in G and Khat: value + DIM derivatives, or (NOVAL: the
    // form has no value term) the DIM derivatives only
    static constexpr int ND = NOVAL ? DIM : DIM + 1;
    static constexpr int P0 = NOVAL ? 1 : 0;                                // first operator kept
    static constexpr int NB = (DEG == 1) ? DIM + 1 : (DIM + 1) * (DIM + 2) / 2;
    static constexpr int N = NC * NB;
    static constexpr int NN = N * N;
    static constexpr int M = ND * NC;                                       // rows of G
    // rows per staged chunk: the largest divisor of N with RC*N <= 64 floats
    // and whole 16-byte pieces; 0 = direct per-lane stores
    static constexpr int rc()
    {
        for (int r = N; r >= 1; --r)
            if (N % r == 0 && r * N <= 64 && (r * N) % 4 == 0) return r;
        return 0;
    }
    static constexpr int RC = rc();
    static constexpr int STR = RC * N + 4;
    static constexpr int LDS_BYTES = RC > 0 ? 4 * 64 * STR * 4 : 16;
};

// G (M x M) from B = J^-1 (rows mu, columns alpha), s = |det J| * kscale and
// the per-element operator C = W_0 + sum_k coef_k W_k (W uniform).  SYM: W
// is symmetric, so only the pairs p <= q of G are formed (sym_index).
template <int DIM, int DEG, int NC, bool SYM, bool NOVAL>
using FormG = float[SYM ? FormShape<DIM, DEG, NC, NOVAL>::M * (FormShape<DIM, DEG, NC, NOVAL>::M + 1) / 2
                        : FormShape<DIM, DEG, NC, NOVAL>::M * FormShape<DIM, DEG, NC, NOVAL>::M];

// G (M x M) from B = J^-1 (rows mu, columns alpha), s = |det J| * kscale and
// the per-element operator C = W_0 + sum_k coef_k W_k (W uniform), block by
// block over the component pair (c, d), using the structure of That:
//   G_{(0,c),(0,d)}         = s C_{(0,c),(0,d)}
//   G_{(0,c),(1+nu,d)}      = s sum_beta C_{(0,c),(1+beta,d)} B_{nu beta}
//   G_{(1+mu,c),(0,d)}      = s sum_alpha B_{mu alpha} C_{(1+alpha,c),(0,d)}
//   G_{(1+mu,c),(1+nu,d)}   = s sum_{alpha,beta} B_{mu alpha} C_{(1+alpha,c),(1+beta,d)} B_{nu beta}
// SYM: W is symmetric, so only the pairs I <= J of G are formed (sym_index).
template <int DIM, int DEG, int NC, bool SYM, bool NOVAL, typename TAB, typename R>
__device__ __forceinline__ void form_build_g(const FormParams &p, const R (&B)[DIM][DIM], R s,
                                             const float (&cf)[kFormMaxCoef + 1],
                                             FormG<DIM, DEG, NC, SYM, NOVAL> &G)
{
    using SH = FormShape<DIM, DEG, NC, NOVAL>;
    constexpr int M = SH::M, MW = (DIM + 1) * NC, ND = DIM + 1;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = 0; d < NC; ++d) {
            // C block (c, d): Cb[a][b] = sum_k cf[k] W_k[(a,c),(b,d)] (NOVAL: a, b >= 1)
            R Cb[ND][ND];
#pragma unroll
            for (int a = SH::P0; a < ND; ++a)
#pragma unroll
                for (int b = SH::P0; b < ND; ++b) {
                    R acc = R(0);
#pragma unroll
                    for (int k = 0; k <= kFormMaxCoef; ++k)
                        if (k <= TAB::n_coef(p)) {
                            const float wv = TAB::w(p, (k * MW + a * NC + c) * MW + b * NC + d);
                            if (!TAB::CONST || wv != 0.f) acc += R(cf[k]) * R(wv);
                        }
                    Cb[a][b] = acc;
                }
            // Z[alpha][nu] = sum_beta C_{(1+alpha),(1+beta)} B_{nu beta}
            R Z[DIM][DIM];
#pragma unroll
            for (int al = 0; al < DIM; ++al)
#pragma unroll
                for (int nu = 0; nu < DIM; ++nu) {
                    R acc = R(0);
#pragma unroll
                    for (int be = 0; be < DIM; ++be) acc += Cb[1 + al][1 + be] * B[nu][be];
                    Z[al][nu] = acc;
                }
            // operator p (0 value, 1 + mu derivative) and component c -> G row (p - P0) NC + c
            auto put = [&](int pp, int cc, int q, int dd, R val) {
                const int I = (pp - SH::P0) * NC + cc, J = (q - SH::P0) * NC + dd;
                if (SYM && I > J) return;
                G[SYM ? sym_index(M, I, J) : I * M + J] = float(s * val);
            };
            if constexpr (!NOVAL) {
                put(0, c, 0, d, Cb[0][0]);
#pragma unroll
                for (int nu = 0; nu < DIM; ++nu) {
                    R acc = R(0);
#pragma unroll
                    for (int be = 0; be < DIM; ++be) acc += Cb[0][1 + be] * B[nu][be];
                    put(0, c, 1 + nu, d, acc);
                }
#pragma unroll
                for (int mu = 0; mu < DIM; ++mu) {
                    R acc = R(0);
#pragma unroll
                    for (int al = 0; al < DIM; ++al) acc += B[mu][al] * Cb[1 + al][0];
                    put(1 + mu, c, 0, d, acc);
                }
            }
#pragma unroll
            for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
                for (int nu = 0; nu < DIM; ++nu) {
                    R acc = R(0);
#pragma unroll
                    for (int al = 0; al < DIM; ++al) acc += B[mu][al] * Z[al][nu];
                    put(1 + mu, c, 1 + nu, d, acc);
                }
        }
}

template <int DIM, int DEG, int NC, bool SYM, bool NOVAL>
__device__ __forceinline__ float form_g(const FormG<DIM, DEG, NC, SYM, NOVAL> &G, int I, int J)
{
    constexpr int M = FormShape<DIM, DEG, NC, NOVAL>::M;
    if constexpr (SYM) return I <= J ? G[sym_index(M, I, J)] : G[sym_index(M, J, I)];
    else return G[I * M + J];
}

// The FP32 forward tile whose whole-matrix store serves symmetric matrices of
// order N (its store depends on N alone).
template <int N>
struct FormStore {
    static constexpr bool OK = false;
    static constexpr int LDS_BYTES = 0;
};
template <int F, int D>
struct FormStoreOf {
    static constexpr bool OK = true;
    using Tile = FwdFmaTile<F, D, float, Traits<F, D>::N>;
    static constexpr int LDS_BYTES = Tile::LDS_BYTES;
};
template <> struct FormStore<3> : FormStoreOf<LAP1, 2> {};
template <> struct FormStore<4> : FormStoreOf<LAP1, 3> {};
template <> struct FormStore<6> : FormStoreOf<ELA1, 2> {};
template <> struct FormStore<10> : FormStoreOf<LAP2, 3> {};
template <> struct FormStore<12> : FormStoreOf<ELA1, 3> {};

constexpr int sym_first(int n, int u)
{
    int a = 0, b = 0;
    sym_pair(n, u, a, b);
    return a;
}
constexpr int sym_second(int n, int u)
{
    int a = 0, b = 0;
    sym_pair(n, u, a, b);
    return b;
}

// Au[u] = entry(I, J) for every distinct entry u = (I <= J) of an order-N
// symmetric matrix, one instantiation per entry (an index sequence), so every
// index is a constant and Au stays in registers.
template <int N, typename F, int... Us>
__device__ __forceinline__ void fill_sym(float (&Au)[N * (N + 1) / 2], const F &entry,
                                         std::integer_sequence<int, Us...>)
{
    ((Au[Us] = entry(std::integral_constant<int, sym_first(N, Us)>::value,
                     std::integral_constant<int, sym_second(N, Us)>::value)), ...);
}

template <int DIM, int DEG, int NC, bool SYM, bool NOVAL, typename TAB>
__device__ __forceinline__ void form_body(const FormParams &p)
{
    using SH = FormShape<DIM, DEG, NC, NOVAL>;
    constexpr int N = SH::N, NN = SH::NN, NB = SH::NB, ND = SH::ND, RC = SH::RC;
    constexpr int KD = DIM + 1;                     // operators per side of Khat
    constexpr bool WHOLE = SYM && FormStore<N>::OK;
    constexpr int LDS = (WHOLE && FormStore<N>::LDS_BYTES > SH::LDS_BYTES) ? FormStore<N>::LDS_BYTES
                                                                            : SH::LDS_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS];

    const int lane = threadIdx.x & 63, wave = wave_id();
    const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * 256 + wave * 64;
    const int64_t E = p.m.n_elements;
    const int64_t e = e0 + lane;
    const bool live = e < E;
    const int64_t ec = live ? e : E - 1;

    int v[DIM + 1];
    load_conn<DIM>(p.m.conn, ec, v);
    float xv[DIM + 1][DIM];
    gather<DIM>(p.m, v, xv);
    float cf[kFormMaxCoef + 1];
    cf[0] = 1.f;
#pragma unroll
    for (int k = 1; k <= kFormMaxCoef; ++k)
        cf[k] = (k <= p.n_coef) ? __builtin_nontemporal_load(p.coef + (k - 1) * E + ec) : 0.f;

    FormG<DIM, DEG, NC, SYM, NOVAL> G;
    float J[DIM][DIM], adj[DIM][DIM];
    jacobian<DIM>(xv, J);
    const float det = adjugate(J, adj);
    bool flag = false, singular = false;
    if (live) {
        flag = needs_fp64<DIM>(J, adj, det, p.tau2);
        if (!flag) {
            const float inv = 1.f / det;
            float B[DIM][DIM];
#pragma unroll
            for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
                for (int al = 0; al < DIM; ++al) B[mu][al] = adj[mu][al] * inv;
            form_build_g<DIM, DEG, NC, SYM, NOVAL, TAB, float>(p, B, fabsf(det) * p.kscale, cf, G);
        } else {
            double Jd[DIM][DIM], adjd[DIM][DIM], Bd[DIM][DIM];
            jacobian<DIM>(xv, Jd);
            const double detd = adjugate(Jd, adjd);
            singular = (detd == 0.0);
            const double inv = 1.0 / detd;
#pragma unroll
            for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
                for (int al = 0; al < DIM; ++al) Bd[mu][al] = adjd[mu][al] * inv;
            form_build_g<DIM, DEG, NC, SYM, NOVAL, TAB, double>(p, Bd, fabs(detd) * double(p.kscale), cf, G);
        }
    } else {
#pragma unroll
        for (int k = 0; k < int(sizeof(G) / sizeof(float)); ++k) G[k] = 0.f;
    }
    count_flags(p.counters, flag, singular);

    // entry (I, J) = ((i, c), (j, d)), I = NC i + c
    auto entry = [&](int I, int Jc) {
        const int i = I / NC, c = I % NC, j = Jc / NC, d = Jc % NC;
        float acc = 0.f;
#pragma unroll
        for (int pp = 0; pp < ND; ++pp)
#pragma unroll
            for (int q = 0; q < ND; ++q) {
                const float kv = TAB::k(p, ((i * NB + j) * KD + pp + SH::P0) * KD + q + SH::P0);
                if (!TAB::CONST || kv != 0.f)
                    acc = fmaf(form_g<DIM, DEG, NC, SYM, NOVAL>(G, pp * NC + c, q * NC + d), kv, acc);
            }
        return acc;
    };

    if constexpr (WHOLE) {
        // the distinct entries (I <= J), stored as the forward stores its matrices
        float Au[N * (N + 1) / 2];
        fill_sym<N>(Au, entry, std::make_integer_sequence<int, N * (N + 1) / 2>{});
        FwdParams fp{};
        fp.m = p.m;
        fp.A = p.A;
        FormStore<N>::Tile::store(fp, e0, Au, smem);
    } else if constexpr (RC == 0) {
        if (live) {
            float *Ae = p.A + e * (int64_t)NN;
#pragma unroll
            for (int I = 0; I < N; ++I)
#pragma unroll
                for (int Jc = 0; Jc < N; ++Jc) Ae[I * N + Jc] = entry(I, Jc);
        }
    } else {
        float *st = reinterpret_cast<float *>(smem) + wave * 64 * SH::STR;
        constexpr int CH = RC * N;                 // floats per element and chunk
        constexpr int NV4 = CH / 4;
        constexpr int PIECES = 64 * NV4;
        constexpr int NP = (PIECES + 63) / 64;
#pragma unroll
        for (int r0 = 0; r0 < N; r0 += RC) {
#pragma unroll
            for (int k = 0; k < CH; k += 4) {
                f32x4_t r;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int flat = k + u;
                    r[u] = entry(r0 + flat / N, flat % N);
                }
                *reinterpret_cast<f32x4_t *>(st + lane * SH::STR + k) = r;
            }
            wave_sync();
            float *dst = p.A + e0 * (int64_t)NN + r0 * N;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const int f = lane + 64 * k;
                const int el = f / NV4, part = f - el * NV4;
                if ((PIECES % 64 == 0 || f < PIECES) && e0 + el < E)
                    *reinterpret_cast<f32x4_t *>(dst + el * (int64_t)NN + 4 * part) =
                        *reinterpret_cast<const f32x4_t *>(st + el * SH::STR + 4 * part);
            }
            wave_sync();
        }
    }
}

template <int DIM, int DEG, int NC, bool SYM, bool NOVAL>
__global__ __launch_bounds__(256) void form_kernel(FormParams p)
{
    form_body<DIM, DEG, NC, SYM, NOVAL, FormTabRuntime>(p);
}

}  // namespace fei

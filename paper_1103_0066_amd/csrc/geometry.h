// Per-element geometry on the device: gather, Jacobian, adjugate, quality
// test and the folded geometric tensor Gf.
//
// Sec. 3, eq. 8: G^{mu nu} = J^-1_{mu alpha} J^-1_{nu alpha} |J|.  With
// adj J = det J * J^-1 this is adj adj^T / |det J|, which needs no division
// per entry.  For elasticity the geometric tensor is the d^2 x d^2 tensor
//   T^{(mu c),(nu d)} = |J| [mu_e (delta_cd (BB^T)_{mu nu} + B_{mu d} B_{nu c})
//                            + lambda_e B_{mu c} B_{nu d}],     B = J^-1,
// the Lame-form analogue of eq. 15 (eq. 15 as printed keeps only the
// delta_cd term); with the block reference tensor of eq. 7 it reproduces
// 2 mu eps:eps + lambda div div exactly.
#pragma once

#include "params.h"
#include "reftensor.h"

namespace fei {

typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// 16-byte store of output that this kernel does not read again: a
// non-temporal store (streaming write, no cache allocation), measured 4-12%
// faster than a plain store for the element-matrix streams.
__device__ __forceinline__ void store_out(f32x4_t *dst, f32x4_t v)
{
    __builtin_nontemporal_store(v, dst);
}

// Whether the staged element-matrix stores of n x n matrices are non-temporal,
// per size as measured on MI355X: yes for 3 x 3 (2D P1 Laplacian, 2.1 M
// triangles: 23.1 vs 25.4 us), 4 x 4 (3D P1 Laplacian: 32.3-33.0 vs 34.2-35.0
// us), 6 x 6 (2D elasticity: 65.1 vs 69.4 us) and 12 x 12 (3D elasticity: 177
// vs 182 us), no for 10 x 10 (3D P2 Laplacian: 121-124 vs 128-130 us, the L2
// combining their runs better).
template <int N>
constexpr bool nt_matrix_stores()
{
    return N != 10;
}

template <int DIM>
__device__ __forceinline__ void load_conn(const int32_t *__restrict__ conn, int64_t e,
                                          int (&v)[DIM + 1])
{
    if constexpr (DIM == 3) {
        const i32x4_t c = __builtin_nontemporal_load(reinterpret_cast<const i32x4_t *>(conn) + e);
        v[0] = c[0]; v[1] = c[1]; v[2] = c[2]; v[3] = c[3];
    } else {
        const int32_t *p = conn + 3 * e;
        v[0] = __builtin_nontemporal_load(p + 0);
        v[1] = __builtin_nontemporal_load(p + 1);
        v[2] = __builtin_nontemporal_load(p + 2);
    }
}

template <int DIM, typename CT>
__device__ __forceinline__ void gather(const MeshView &m, const int (&v)[DIM + 1],
                                       CT (&xv)[DIM + 1][DIM])
{
    const CT *__restrict__ X = static_cast<const CT *>(m.x);
    const CT *__restrict__ Y = static_cast<const CT *>(m.y);
    const CT *__restrict__ Z = static_cast<const CT *>(m.z);
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        xv[a][0] = X[v[a]];
        xv[a][1] = Y[v[a]];
        if constexpr (DIM == 3) xv[a][2] = Z[v[a]];
    }
}

// J[alpha][m] = x_{m+1}[alpha] - x_0[alpha]
template <int DIM, typename R, typename CT>
__device__ __forceinline__ void jacobian(const CT (&xv)[DIM + 1][DIM], R (&J)[DIM][DIM])
{
#pragma unroll
    for (int al = 0; al < DIM; ++al)
#pragma unroll
        for (int m = 0; m < DIM; ++m) J[al][m] = R(xv[m + 1][al]) - R(xv[0][al]);
}

// adj[m][alpha] = det(J) * (J^-1)[m][alpha]; returns det(J).
template <typename R>
__device__ __forceinline__ R adjugate(const R (&J)[3][3], R (&adj)[3][3])
{
    const R a = J[0][0], b = J[0][1], c = J[0][2];
    const R d = J[1][0], e = J[1][1], f = J[1][2];
    const R g = J[2][0], h = J[2][1], i = J[2][2];
    adj[0][0] = e * i - f * h; adj[0][1] = c * h - b * i; adj[0][2] = b * f - c * e;
    adj[1][0] = f * g - d * i; adj[1][1] = a * i - c * g; adj[1][2] = c * d - a * f;
    adj[2][0] = d * h - e * g; adj[2][1] = b * g - a * h; adj[2][2] = a * e - b * d;
    return a * adj[0][0] + b * adj[1][0] + c * adj[2][0];
}

template <typename R>
__device__ __forceinline__ R adjugate(const R (&J)[2][2], R (&adj)[2][2])
{
    adj[0][0] = J[1][1]; adj[0][1] = -J[0][1];
    adj[1][0] = -J[1][0]; adj[1][1] = J[0][0];
    return J[0][0] * J[1][1] - J[0][1] * J[1][0];
}

// Quality test: kappa_F = |J|_F |adj J|_F / |det J| > tau, evaluated as
// !(|J|^2 |adj|^2 <= tau^2 det^2) so that NaN and tau2 < 0 select the FP64
// path.  det == 0 selects it explicitly: when adj J vanishes too (collinear
// or coincident vertices) the product test reads 0 <= 0 and would pass.
template <int DIM>
__device__ __forceinline__ bool needs_fp64(const float (&J)[DIM][DIM],
                                           const float (&adj)[DIM][DIM], float det, float tau2)
{
    float nj = 0.f, na = 0.f;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            nj = fmaf(J[i][k], J[i][k], nj);
            na = fmaf(adj[i][k], adj[i][k], na);
        }
    return !(nj * na <= tau2 * (det * det)) || det == 0.f;
}

// Folded geometric tensor from adj J and the element's weights: wa = vol_ref
// / (KDEN |det J|) for the Laplacian forms; wa = that weight times mu and wb =
// times lam for elasticity.  Gf[sym_index(p, q)], p <= q, so that A = sum_g
// Gf[g] Kf[g] with the integer reference tensor.
template <int FORM, int DIM, typename R>
__device__ __forceinline__ void build_gf_weighted(const R (&adj)[DIM][DIM], R wa, R wb,
                                                  float (&Gf)[Traits<FORM, DIM>::G])
{
    using T = Traits<FORM, DIM>;
    R M[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int n = 0; n < DIM; ++n) {
            R acc = R(0);
#pragma unroll
            for (int al = 0; al < DIM; ++al) acc += adj[m][al] * adj[n][al];
            M[m][n] = acc;
        }
    if constexpr (FORM != ELA1) {
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = m; n < DIM; ++n) Gf[sym_index(DIM, m, n)] = float(wa * M[m][n]);
    } else {
#pragma unroll
        for (int p = 0; p < T::GD; ++p)
#pragma unroll
            for (int q = p; q < T::GD; ++q) {
                const int m = p / DIM, c = p % DIM, n = q / DIM, d = q % DIM;
                R t = wa * (adj[m][d] * adj[n][c]) + wb * (adj[m][c] * adj[n][d]);
                if (c == d) t += wa * M[m][n];
                Gf[sym_index(T::GD, p, q)] = float(t);
            }
    }
}

// The element's weights of build_gf_weighted.
template <int FORM, int DIM, typename R>
__device__ __forceinline__ void gf_weights(R det, float mu, float lam, R &wa, R &wb)
{
    const R s = det < R(0) ? -det : det;
    const R w = R(Traits<FORM, DIM>::SCALE) / s;
    wa = FORM == ELA1 ? w * R(mu) : w;
    wb = FORM == ELA1 ? w * R(lam) : R(0);
}

// Folded geometric tensor of the element (Sec. 3, eq. 8; the Lame analogue for
// elasticity), scaled by Traits::SCALE = vol_ref / KDEN.
template <int FORM, int DIM, typename R>
__device__ __forceinline__ void build_gf(const R (&adj)[DIM][DIM], R det, float mu, float lam,
                                         float (&Gf)[Traits<FORM, DIM>::G])
{
    R wa, wb;
    gf_weights<FORM, DIM>(det, mu, lam, wa, wb);
    build_gf_weighted<FORM, DIM>(adj, wa, wb, Gf);
}

// Whole geometry stage for one element (gather already done).  FP64
// coordinates always use FP64; FP32 coordinates use FP32 unless the quality
// test flags the element.  Returns true when the FP64 path was taken; *singular
// reports det J == 0 on the path taken.
template <int FORM, int DIM, typename CT>
__device__ __forceinline__ bool geometry(const CT (&xv)[DIM + 1][DIM], float mu, float lam,
                                         float tau2, float (&Gf)[Traits<FORM, DIM>::G],
                                         bool &singular)
{
    if constexpr (sizeof(CT) == 8) {
        double J[DIM][DIM], adj[DIM][DIM];
        jacobian<DIM>(xv, J);
        const double det = adjugate(J, adj);
        singular = (det == 0.0);
        build_gf<FORM, DIM>(adj, det, mu, lam, Gf);
        return false;
    } else {
        float J[DIM][DIM], adj[DIM][DIM];
        jacobian<DIM>(xv, J);
        const float det = adjugate(J, adj);
        const bool flag = needs_fp64<DIM>(J, adj, det, tau2);
        if (!flag) {
            singular = false;
            build_gf<FORM, DIM>(adj, det, mu, lam, Gf);
        } else {
            double Jd[DIM][DIM], adjd[DIM][DIM];
            jacobian<DIM>(xv, Jd);
            const double detd = adjugate(Jd, adjd);
            singular = (detd == 0.0);
            build_gf<FORM, DIM>(adjd, detd, mu, lam, Gf);
        }
        return flag;
    }
}

// Accumulate the FP64-path and singular counts of a wave with one atomic each.
__device__ __forceinline__ void count_flags(int32_t *counters, bool flag, bool singular)
{
    if (!counters) return;
    const unsigned long long fl = __ballot(flag);
    const unsigned long long sg = __ballot(singular);
    const unsigned long long active = __ballot(1);
    const int leader = __ffsll(active) - 1;
    if ((int)__lane_id() == leader) {
        if (fl) atomicAdd(&counters[0], (int)__popcll(fl));
        if (sg) atomicAdd(&counters[1], (int)__popcll(sg));
    }
}

// Index of this lane's wave in the workgroup, as a wave-uniform value (the
// compiler cannot see that threadIdx.x >> 6 is uniform; said explicitly,
// per-wave bases stay in SGPRs and per-wave conditions become scalar branches).
__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
}

// Workgroup index remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of elements; vertices
// shared by neighbouring elements are then gathered through the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t per = nb / 8, rem = nb % 8;
    const int64_t x = b % 8, i = b / 8;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

}  // namespace fei

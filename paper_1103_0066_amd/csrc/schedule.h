// The fused assembly's incidence schedule (host code, no device calls): each
// row's vertex-to-element incidences ordered into steps whose elements share
// no vertex but the row's, so that the lanes of a row can add one step's
// off-diagonal blocks without two of them touching the same block.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace fei {

// Orders the incidences list[0 .. n) of row v into steps of `lanes` entries
// (-1 pads a step) such that the elements of one step share no vertex but v:
// the lanes of a row then add a step's off-diagonal blocks at once, with no
// two of them on one block (each element's block on the diagonal goes to the
// lane's registers).  A depth-first search with a node budget looks for
// ceil(n / lanes) steps, then one more; first fit is the fallback.
inline void schedule_row(int32_t v, const int32_t *list, int n, const std::vector<int32_t> &conn,
                         int nv, int lanes, std::vector<int32_t> &out)
{
    const int no = nv - 1;                           // other vertices per element
    // an element that lists v more than once keeps v among its other vertices,
    // so two such incidences (whose blocks reach v's own slot through LDS)
    // never share a step
    std::vector<int32_t> nb(size_t(n) * no, v);
    for (int i = 0; i < n; ++i) {
        const int64_t e = list[i] / nv;
        int k = 0;
        for (int b = 0; b < nv; ++b) {
            const int32_t w = conn[size_t(e) * nv + b];
            if (w != v) nb[size_t(i) * no + k++] = w;
        }
    }
    std::vector<int> gsz, member;
    std::vector<int32_t> used;                       // per step: lanes * no vertices
    auto fits = [&](int i, int g) {
        if (gsz[g] >= lanes) return false;
        for (int k = 0; k < gsz[g] * no; ++k)
            for (int q = 0; q < no; ++q)
                if (used[size_t(g) * lanes * no + k] == nb[size_t(i) * no + q]) return false;
        return true;
    };
    auto put = [&](int i, int g) {
        for (int q = 0; q < no; ++q) used[size_t(g) * lanes * no + gsz[g] * no + q] = nb[size_t(i) * no + q];
        member[size_t(g) * lanes + gsz[g]++] = i;
    };
    auto emit = [&](int G) {
        for (int g = 0; g < G; ++g)
            for (int k = 0; k < lanes; ++k) out.push_back(k < gsz[g] ? list[member[size_t(g) * lanes + k]] : -1);
    };
    auto reset = [&](int G) {
        gsz.assign(G, 0);
        member.assign(size_t(G) * lanes, 0);
        used.assign(size_t(G) * lanes * no, -1);
    };
    const int lo = (n + lanes - 1) / lanes;
    for (int G = lo; G <= lo + 1 && n > 0; ++G) {
        reset(G);
        long budget = 4096;
        // steps are opened in order, so only the first empty step is tried
        std::function<bool(int)> dfs = [&](int i) -> bool {
            if (i == n) return true;
            if (--budget < 0) return false;
            for (int g = 0; g < G; ++g) {
                const bool empty = gsz[g] == 0;
                if (fits(i, g)) {
                    put(i, g);
                    if (dfs(i + 1)) return true;
                    --gsz[g];
                    if (budget < 0) return false;
                }
                if (empty) break;
            }
            return false;
        };
        if (dfs(0)) {
            emit(G);
            return;
        }
    }
    // first fit: always succeeds, with at most n steps
    reset(n);
    int G = 0;
    for (int i = 0; i < n; ++i) {
        int g = 0;
        while (g < G && !fits(i, g)) ++g;
        if (g == G) ++G;
        put(i, g);
    }
    emit(G);
}

}  // namespace fei

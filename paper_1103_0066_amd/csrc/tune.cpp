// Tune table and forward tuner (fei_tune_*): the forward's launch shape --
// elements per workgroup (the paper's element batch size, Sec. 4) and output
// staging (its interleaved stores, Sec. 4.3) -- chosen by timing candidates on
// the caller's data, kept per (form, dim, precision, coordinate type, size
// bucket) for the process and persisted as JSON lines.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fei.h"
#include "host.h"
#include "params.h"

using namespace fei;
using namespace fei::host;

namespace {

using Key = std::tuple<int, int, int, int, int>;   // form, dim, precision, coord, ebucket

std::mutex g_mutex;
std::map<Key, fei_tune_result> g_table;
bool g_env_loaded = false;

int ebucket(int64_t E)
{
    int b = 0;
    while (E > 1) {
        E >>= 1;
        ++b;
    }
    return b;
}

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return std::string();
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Value of "name": in a JSON line (numbers, or a string for "arch").
bool json_number(const std::string &line, const char *name, double &v)
{
    const std::string key = std::string("\"") + name + "\"";
    const size_t p = line.find(key);
    if (p == std::string::npos) return false;
    const size_t c = line.find(':', p + key.size());
    if (c == std::string::npos) return false;
    char *end = nullptr;
    v = std::strtod(line.c_str() + c + 1, &end);
    return end != line.c_str() + c + 1;
}

std::string json_string(const std::string &line, const char *name)
{
    const std::string key = std::string("\"") + name + "\"";
    const size_t p = line.find(key);
    if (p == std::string::npos) return std::string();
    const size_t q0 = line.find('"', line.find(':', p + key.size()) + 1);
    if (q0 == std::string::npos) return std::string();
    const size_t q1 = line.find('"', q0 + 1);
    return q1 == std::string::npos ? std::string() : line.substr(q0 + 1, q1 - q0 - 1);
}

int load_locked(const char *path)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(FEI_EINVAL, "cannot open tune file %s", path);
    int dev_count = 0;
    const std::string arch = (hipGetDeviceCount(&dev_count) == hipSuccess && dev_count > 0)
                                 ? device_arch() : std::string();
    char buf[1024];
    int bad = 0;
    while (std::fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        if (line.find('{') == std::string::npos) continue;
        double form, dim, prec, coord, eb, blk, rows, ms;
        if (!json_number(line, "form", form) || !json_number(line, "dim", dim) ||
            !json_number(line, "precision", prec) || !json_number(line, "coord", coord) ||
            !json_number(line, "ebucket", eb) || !json_number(line, "block_elements", blk) ||
            !json_number(line, "store_rows", rows)) {
            ++bad;
            continue;
        }
        if (!json_number(line, "ms", ms)) ms = 0.0;
        const std::string a = json_string(line, "arch");
        if (!arch.empty() && !a.empty() && a != arch) continue;
        fei_tune_result r;
        r.block_elements = int(blk);
        r.store_rows = int(rows);
        r.ms = float(ms);
        r.candidates = 0;
        g_table[Key{int(form), int(dim), int(prec), int(coord), int(eb)}] = r;
    }
    std::fclose(f);
    return bad ? fail(FEI_EINVAL, "%d malformed line(s) in %s", bad, path) : FEI_OK;
}

void load_env_locked()
{
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *path = std::getenv("FEI_TUNE_FILE");
    if (path && *path) (void)load_locked(path);
}

}  // namespace

namespace fei {
namespace host {

bool tune_find(int form, int dim, int precision, int coord_dtype, int64_t n_elements,
               fei_tune_result &out)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    load_env_locked();
    const auto it = g_table.find(Key{form, dim, precision, coord_dtype, ebucket(n_elements)});
    if (it == g_table.end()) return false;
    out = it->second;
    return true;
}

}  // namespace host
}  // namespace fei

extern "C" {

int fei_tune_lookup(int form, int dim, int precision, int coord_dtype, int64_t n_elements,
                    fei_tune_result *out)
{
    fei_tune_result r;
    if (!tune_find(form, dim, precision, coord_dtype, n_elements, r)) return 0;
    if (out) *out = r;
    return 1;
}

int fei_tune_save(const char *path)
{
    if (!path) return fail(FEI_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lock(g_mutex);
    load_env_locked();
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(FEI_EINVAL, "cannot write tune file %s", path);
    int dev_count = 0;
    const std::string arch = (hipGetDeviceCount(&dev_count) == hipSuccess && dev_count > 0)
                                 ? device_arch() : std::string("unknown");
    for (const auto &kv : g_table) {
        int form, dim, prec, coord, eb;
        std::tie(form, dim, prec, coord, eb) = kv.first;
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"form\": %d, \"dim\": %d, \"precision\": %d, "
                     "\"coord\": %d, \"ebucket\": %d, \"block_elements\": %d, "
                     "\"store_rows\": %d, \"ms\": %.6f}\n",
                     arch.c_str(), form, dim, prec, coord, eb, kv.second.block_elements,
                     kv.second.store_rows, double(kv.second.ms));
    }
    return std::fclose(f) == 0 ? FEI_OK : fail(FEI_EINVAL, "writing %s failed", path);
}

int fei_tune_load(const char *path)
{
    if (!path) return fail(FEI_EINVAL, "path is NULL");
    std::lock_guard<std::mutex> lock(g_mutex);
    load_env_locked();
    return load_locked(path);
}

int fei_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    g_env_loaded = true;     // an explicit clear also drops what the environment named
    g_table.clear();
    return FEI_OK;
}

int fei_tune_forward(const fei_mesh *m, int form, const float *mu, const float *lam, float *A,
                     const fei_options *opt, void *stream, fei_tune_result *out)
{
    if (!m) return fail(FEI_EINVAL, "mesh is NULL");
    fei_options base = opt ? *opt : defaults();
    int rc = check_options(base);
    if (rc) return rc;
    const int n = local_size(form, m->dim);
    if (n < 0) return fail(FEI_EINVAL, "bad form %d or dim %d", form, m->dim);
    if (m->n_elements == 0) return fail(FEI_EINVAL, "nothing to tune on (n_elements == 0)");
    // candidates: (block_elements, store_rows)
    std::vector<std::pair<int, int>> cand;
    if (base.precision == FEI_PREC_FP32) {
        if (m->coord_dtype == FEI_F32)
            for (int b : {64, 128, 256, 512}) cand.push_back({b, 0});
        else
            cand.push_back({256, 0});
        cand.push_back({256, -1});
        for (int r : {2, 4})
            if (n % r == 0 && (r * n) % 4 == 0 && r < n) cand.push_back({256, r});
    } else {
        cand.push_back({256, 0});
        cand.push_back({256, -1});
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    fei_tune_result best{0, 0, 0.f, 0};
    float best_ms = INFINITY;
    int tried = 0;
    for (const auto &c : cand) {
        fei_options o = base;
        o.block_elements = c.first;
        o.store_rows = c.second;
        // a candidate without a kernel is skipped; any other failure ends the tuning
        rc = fei_integrate(m, form, mu, lam, A, &o, stream);
        if (rc == FEI_EUNSUPPORTED) continue;
        if (rc) break;
        for (int w = 0; w < 2 && rc == FEI_OK; ++w) rc = fei_integrate(m, form, mu, lam, A, &o, stream);
        const int reps = 5;
        if (rc == FEI_OK && (e = hipEventRecord(e0, s)) != hipSuccess) rc = hip_fail(e, "event");
        for (int r = 0; r < reps && rc == FEI_OK; ++r) rc = fei_integrate(m, form, mu, lam, A, &o, stream);
        if (rc == FEI_OK && (e = hipEventRecord(e1, s)) != hipSuccess) rc = hip_fail(e, "event");
        if (rc == FEI_OK && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "event");
        float ms = 0.f;
        if (rc == FEI_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            rc = hip_fail(e, "event time");
        if (rc) break;
        ++tried;
        ms /= reps;
        if (ms < best_ms) {
            best_ms = ms;
            best.block_elements = c.first;
            best.store_rows = c.second;
            best.ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (tried == 0) return fail(FEI_EUNSUPPORTED, "no forward kernel for this variant");
    best.candidates = tried;
    // the default shape is stored as (0, 0), i.e. "use the built-in default"
    if (best.block_elements == 256 && best.store_rows == 0) best.block_elements = 0;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        load_env_locked();
        g_table[Key{form, m->dim, base.precision, m->coord_dtype, ebucket(m->n_elements)}] = best;
    }
    if (out) *out = best;
    return FEI_OK;
}

}  // extern "C"

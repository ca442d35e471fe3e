// Kernel-variant ("tile") table and autotuner.
//
// For a given (device architecture, Taylor order p, number of right-hand sides K,
// precision) the far and near fields can run as VALU kernels that take 1, 2 or 4
// right-hand sides per pass, or (FP32, several right-hand sides) run on the matrix
// cores; the far field can run every entry cluster major, and its group-major lists can
// be cut into up to four parts, a wave each.  stk_autotune times every candidate on a synthetic problem of the
// caller's shape (uniform points in the unit cube generated on the device) and records
// the fastest; evaluations look the table up and fall back to a fixed rule otherwise.
// The table can be written to and read from a text file.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "stk_internal.hpp"

namespace stk {
namespace {

using Key = std::tuple<std::string, int, int, int>;  // arch, p, K, precision

std::mutex g_mu;
std::map<Key, Tiles> g_table;

std::string arch_name() {
    int dev = 0;
    STK_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    STK_HIP(hipGetDeviceProperties(&prop, dev));
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// counter-based uniform in [0, 1): SplitMix64 of (seed, index)
__device__ inline double unif(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return double(z >> 11) * (1.0 / 9007199254740992.0);
}

__global__ void k_synth(int64_t n, int K, double *pos, double *f, double *h, double *nu) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < 3; ++a) pos[3 * i + a] = unif(1, 3 * i + a);
    double v[3], s = 0.0;
    for (int a = 0; a < 3; ++a) {
        v[a] = 2.0 * unif(2, 3 * i + a) - 1.0;
        s += v[a] * v[a];
    }
    s = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int a = 0; a < 3; ++a) nu[3 * i + a] = s > 0.0 ? v[a] * s : (a == 0 ? 1.0 : 0.0);
    for (int r = 0; r < K; ++r)
        for (int a = 0; a < 3; ++a) {
            f[(int64_t(r) * n + i) * 3 + a] = 2.0 * unif(3 + r, 3 * i + a) - 1.0;
            h[(int64_t(r) * n + i) * 3 + a] = 2.0 * unif(1000 + r, 3 * i + a) - 1.0;
        }
}

struct DevMem {
    void *p = nullptr;
    explicit DevMem(size_t bytes) { STK_HIP(hipMalloc(&p, bytes < 256 ? 256 : bytes)); }
    ~DevMem() { (void)hipFree(p); }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace

Tiles default_tiles(int K, stk_precision prec) {
    Tiles t;
    if (prec == STK_FP64) return t;
    t.far_kb = K % 4 == 0 ? 4 : (K % 2 == 0 ? 2 : 1);
    t.near_kb = t.far_kb;
    t.near_mfma = K >= 8;
    return t;
}

bool tiles_valid(const Tiles &t, int K, stk_precision prec) {
    auto kb_ok = [&](int kb) { return (kb == 1 || kb == 2 || kb == 4) && K % kb == 0; };
    if (!kb_ok(t.far_kb) || !kb_ok(t.near_kb)) return false;
    if (prec == STK_FP64 && (t.far_kb != 1 || t.near_kb != 1 || t.near_mfma || t.far_mfma)) return false;
    if (t.far_cm != FAR_CM_AUTO && t.far_cm != FAR_CM_ON && t.far_cm != FAR_CM_OFF) return false;
    if (t.far_cm == FAR_CM_ON && t.far_mfma) return false;  // the matrix-core far kernel has no cluster-major split
    if (t.far_split < 0 || t.far_split > FAR_SPLIT_MAX) return false;
    if (t.far_mfma && t.far_split > 1) return false;  // nor split group lists
    return true;
}

Tiles tiles_for(int p, int K, stk_precision prec) {
    const Key k{arch_name(), p, K, int(prec)};
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(k);
    return it != g_table.end() ? it->second : default_tiles(K, prec);
}

bool tiles_lookup(int p, int K, stk_precision prec, Tiles *out) {
    const Key k{arch_name(), p, K, int(prec)};
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(k);
    if (it == g_table.end()) return false;
    if (out) *out = it->second;
    return true;
}

void tiles_set(int p, int K, stk_precision prec, const Tiles *t) {
    const Key k{arch_name(), p, K, int(prec)};
    std::lock_guard<std::mutex> lk(g_mu);
    if (t)
        g_table[k] = *t;
    else
        g_table.erase(k);
}

void tiles_save(const char *path) {
    std::lock_guard<std::mutex> lk(g_mu);
    FILE *fp = std::fopen(path, "w");
    if (!fp) throw Error(STK_EINVAL, std::string("cannot write ") + path);
    std::fprintf(fp, "# arch p K precision far_kb near_kb near_mfma far_mfma far_cm far_split\n");
    for (const auto &e : g_table)
        std::fprintf(fp, "%s %d %d %d %d %d %d %d %d %d\n", std::get<0>(e.first).c_str(), std::get<1>(e.first),
                     std::get<2>(e.first), std::get<3>(e.first), e.second.far_kb, e.second.near_kb,
                     e.second.near_mfma ? 1 : 0, e.second.far_mfma ? 1 : 0, e.second.far_cm, e.second.far_split);
    std::fclose(fp);
}

int tiles_load(const char *path) {
    FILE *fp = std::fopen(path, "r");
    if (!fp) throw Error(STK_EINVAL, std::string("cannot read ") + path);
    std::vector<std::pair<Key, Tiles>> rows;
    char line[512];
    int lineno = 0;
    while (std::fgets(line, sizeof line, fp)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[128];
        int p, K, prec, fkb, nkb, nm, fm, fc, fs = 0;
        // far_split may be absent (tables written before it existed: automatic)
        const int got = std::sscanf(line, "%127s %d %d %d %d %d %d %d %d %d", arch, &p, &K, &prec, &fkb, &nkb, &nm,
                                    &fm, &fc, &fs);
        if ((got != 9 && got != 10) || (prec != STK_FP64 && prec != STK_MIXED)) {
            std::fclose(fp);
            throw Error(STK_EINVAL, std::string(path) + ": malformed line " + std::to_string(lineno));
        }
        Tiles t;
        t.far_kb = fkb;
        t.near_kb = nkb;
        t.near_mfma = nm != 0;
        t.far_mfma = fm != 0;
        t.far_cm = fc;
        t.far_split = got == 10 ? fs : 0;
        if (!tiles_valid(t, K, stk_precision(prec))) {
            std::fclose(fp);
            throw Error(STK_EINVAL, std::string(path) + ": invalid tiles on line " + std::to_string(lineno));
        }
        rows.push_back({Key{arch, p, K, prec}, t});
    }
    std::fclose(fp);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &r : rows) g_table[r.first] = r.second;
    return int(rows.size());
}

Tiles autotune(int p, int K, stk_precision prec, int64_t n, double theta, int32_t n0, double *best_ms,
               hipStream_t s) {
    DevMem pos(sizeof(double) * 3 * n), f(sizeof(double) * 3 * n * K), h(sizeof(double) * 3 * n * K),
        nu(sizeof(double) * 3 * n), u(sizeof(double) * 3 * n * K);
    hipLaunchKernelGGL(k_synth, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, K, pos.as<double>(),
                       f.as<double>(), h.as<double>(), nu.as<double>());
    STK_CHECK_LAUNCH();
    Tree tree;
    STK_HIP(hipGetDevice(&tree.device));
    build_tree(tree, pos.as<double>(), n, n0, s);
    compute_moments(tree, f.as<double>(), h.as<double>(), nu.as<double>(), K, p, prec, s);

    std::vector<Tiles> near_c, far_c;
    for (int kb : {1, 2, 4}) {
        Tiles t = default_tiles(K, prec);
        t.near_kb = kb;
        t.near_mfma = false;
        if (tiles_valid(t, K, prec)) near_c.push_back(t);
        t = default_tiles(K, prec);
        t.far_kb = kb;
        t.far_mfma = false;
        if (tiles_valid(t, K, prec)) far_c.push_back(t);
    }
    if (prec == STK_MIXED && K > 1) {
        Tiles t = default_tiles(K, prec);
        t.near_mfma = true;
        near_c.push_back(t);
        t = default_tiles(K, prec);
        t.far_mfma = true;
        far_c.push_back(t);
    }
    for (int32_t mode : {FAR_CM_ON, FAR_CM_OFF})
        for (int kb : {1, 2, 4}) {
            // every far entry cluster major (the group-major kernel then only writes the
            // sums), or never, with kb right-hand sides per recurrence
            Tiles t = default_tiles(K, prec);
            t.far_kb = kb;
            t.far_mfma = false;
            t.far_cm = mode;
            if (tiles_valid(t, K, prec)) far_c.push_back(t);
        }
    for (int split = 1; split <= FAR_SPLIT_MAX; ++split) {
        // group-major far lists cut into `split` parts, a wave each
        Tiles t = default_tiles(K, prec);
        t.far_mfma = false;
        t.far_cm = FAR_CM_OFF;
        t.far_split = split;
        if (tiles_valid(t, K, prec)) far_c.push_back(t);
    }
    hipEvent_t e0, e1;
    STK_HIP(hipEventCreate(&e0));
    STK_HIP(hipEventCreate(&e1));
    auto time_one = [&](const Tiles &t) {
        Plan pl;
        pl.forced = true;
        pl.force = t;
        evaluate(tree, pl, pos.as<double>(), n, theta, u.as<double>(), true, s);  // warm-up
        float best = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            STK_HIP(hipEventRecord(e0, s));
            evaluate(tree, pl, pos.as<double>(), n, theta, u.as<double>(), true, s);
            STK_HIP(hipEventRecord(e1, s));
            STK_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            STK_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = ms < best ? ms : best;
        }
        return double(best);
    };
    // near variant with the default far kernel, then the far block with that near variant
    Tiles best = default_tiles(K, prec);
    double bms = 1e300;
    for (const Tiles &t : near_c) {
        const double ms = time_one(t);
        if (ms < bms) {
            bms = ms;
            best = t;
        }
    }
    for (Tiles t : far_c) {
        t.near_kb = best.near_kb;
        t.near_mfma = best.near_mfma;
        const double ms = time_one(t);
        if (ms < bms) {
            bms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    STK_HIP(hipStreamSynchronize(s));
    tiles_set(p, K, prec, &best);
    if (best_ms) *best_ms = bms;
    return best;
}

}  // namespace stk

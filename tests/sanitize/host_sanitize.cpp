// Address / undefined-behaviour sanitizer run of the library's host code
// (test infrastructure): validation, host coarsening, plan sizing, the
// error paths of plan creation and the score plan sizing, on seeded random
// hypergraphs with isolated nodes, singleton hyperedges and tier-boundary
// rows.  Built with g++ -fsanitize=address,undefined together with
// csrc/hnv_host.cpp only (no device code); the few device-side functions the
// host code refers to are replaced below by stand-ins that report a device
// error, so every call that would reach the GPU takes its error path.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <set>
#include <vector>

#include "hnv_internal.h"

// --- stand-ins for the device side --------------------------------------
extern "C" hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t)
{
    return hipErrorNoDevice;
}
extern "C" hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorNoDevice; }
extern "C" const char *hipGetErrorString(hipError_t) { return "no device (sanitizer build)"; }
hnv_plan::~hnv_plan() {}
namespace hnv {
hnv_status dev_recompute_reciprocals(hnv_plan *, int, void *) { return fail(HNV_EDEVICE, "no device"); }
hnv_status dev_fill_inline_ids(hnv_plan *, int, hipStream_t)
{
    return fail(HNV_EDEVICE, "no device");
}
hnv_status dev_score(const ScorePlan &, const void *, hnv_dtype, int, int, float *, hipStream_t)
{
    return fail(HNV_EDEVICE, "no device");
}
}  // namespace hnv

// --- test harness: random hypergraphs through the host library -----------
struct Graph {
    int64_t n = 0, m = 0;
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> idx;
    std::vector<float> w;
};

static Graph random_graph(std::mt19937_64 &rng, int64_t n, int64_t m, int max_size, bool hub)
{
    Graph g;
    g.n = n;
    g.m = m;
    for (int64_t e = 0; e < m; ++e) {
        const int size = std::min<int64_t>(n, 1 + (int)(rng() % (uint64_t)max_size));
        std::set<int32_t> s;
        if (hub && e % 3 == 0)
            s.insert(0);
        while ((int)s.size() < size)
            s.insert((int32_t)(rng() % (uint64_t)n));
        g.idx.insert(g.idx.end(), s.begin(), s.end());
        g.ptr.push_back((int64_t)g.idx.size());
        g.w.push_back((float)(1 + rng() % 3));
    }
    return g;
}

static hnv_level level_of(const Graph &g)
{
    return hnv_level{g.n, g.m, (int64_t)g.idx.size(), g.ptr.data(), g.idx.empty() ? nullptr : g.idx.data(),
                     g.w.empty() ? nullptr : g.w.data()};
}

static int run_case(std::mt19937_64 &rng, int64_t n, int64_t m, int max_size, bool hub)
{
    std::vector<Graph> levels{random_graph(rng, n, m, max_size, hub)};
    std::vector<std::vector<int32_t>> nrep, erep;
    for (int step = 0; step < 3; ++step) {
        const Graph &f = levels.back();
        hnv_level lv = level_of(f);
        if (hnv_validate_level(&lv) != HNV_OK)
            return 1;
        Graph c;
        std::vector<int32_t> nr(f.n + 1), er(f.m + 1), cidx(f.idx.size() + 1);
        std::vector<int64_t> cptr(f.m + 1);
        std::vector<float> cw(f.m + 1);
        int64_t cn = 0, cm = 0, cz = 0;
        if (hnv_coarsen_level(&lv, nr.data(), er.data(), cptr.data(), cidx.data(), cw.data(), &cn, &cm, &cz) != HNV_OK)
            return 2;
        c.n = cn;
        c.m = cm;
        c.ptr.assign(cptr.begin(), cptr.begin() + cm + 1);
        c.idx.assign(cidx.begin(), cidx.begin() + cz);
        c.w.assign(cw.begin(), cw.begin() + cm);
        nr.resize(f.n);
        er.resize(f.m);
        nrep.push_back(nr);
        erep.push_back(er);
        levels.push_back(c);
    }
    std::vector<hnv_level> lv;
    for (auto &g : levels)
        lv.push_back(level_of(g));
    std::vector<hnv_map> maps;
    for (size_t l = 0; l + 1 < levels.size(); ++l)
        maps.push_back(hnv_map{nrep[l].data(), erep[l].data()});
    for (int small_max : {0, 3, 8})
        for (int chunk : {0, 5, 64}) {
            hnv_options o{0, small_max, chunk, 0};
            size_t bytes = 0;
            if (hnv_plan_workspace_bytes(lv.data(), maps.data(), (int)lv.size(), 16, HNV_BF16, &o, &bytes) != HNV_OK)
                return 3;
            // creation reaches the first device copy and must unwind cleanly
            std::vector<char> fake(bytes + 512);
            void *ws = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(fake.data()) + 255) & ~uintptr_t(255));
            hnv_plan *plan = nullptr;
            if (hnv_plan_create(lv.data(), maps.data(), (int)lv.size(), 16, HNV_BF16, &o, 1, ws, bytes, nullptr,
                                &plan) != HNV_EDEVICE || plan != nullptr)
                return 4;
        }
    // corrupted inputs give statuses, never a fault
    Graph bad = levels[0];
    if (!bad.idx.empty()) {
        bad.idx[0] = (int32_t)bad.n;
        hnv_level b = level_of(bad);
        if (hnv_validate_level(&b) != HNV_ERANGE)
            return 5;
    }
    std::vector<int32_t> badmap = nrep[0];
    if (!badmap.empty()) {
        badmap[0] = -7;
        hnv_map mp{badmap.data(), erep[0].data()};
        hnv_plan *plan = nullptr;
        std::vector<char> fake(4096);
        void *ws = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(fake.data()) + 255) & ~uintptr_t(255));
        if (hnv_plan_create(lv.data(), &mp, 2, 16, HNV_F32, nullptr, 1, ws, 1024, nullptr, &plan) != HNV_ERANGE)
            return 6;
    }
    // score plan sizing over the finest hyperedges as candidates
    size_t sb = 0;
    if (hnv_score_workspace_bytes(levels[0].ptr.data(), levels[0].m, 24, HNV_F32, &sb) != HNV_OK)
        return 7;
    return 0;
}

int main()
{
    std::mt19937_64 rng(20210317);
    const int64_t shapes[][3] = {{1, 1, 1}, {6, 4, 3}, {50, 30, 6}, {400, 300, 12}, {64, 500, 5}, {2000, 900, 70}};
    int i = 0;
    for (auto &s : shapes) {
        for (bool hub : {false, true}) {
            const int rc = run_case(rng, s[0], s[1], (int)s[2], hub);
            if (rc != 0) {
                std::fprintf(stderr, "case %d (hub %d) failed at check %d: %s\n", i, (int)hub, rc, hnv_last_error());
                return 1;
            }
        }
        ++i;
    }
    std::printf("host sanitizer run ok\n");
    return 0;
}

// Autotuner of the batched evaluate-and-stamp launch (cs_batch_tune).
//
// A sizing loop calls the simulator many times on the same batch of circuits
// (paper, Introduction), so the batched launch's schedule is chosen once per batch
// shape by measurement: every candidate (schedule, block size, evaluate-ahead mode,
// size below which a circuit is stamped inside one workgroup) is applied, one
// batched step is captured in a HIP graph, and the graph is replayed `reps` times
// between two events on the caller's stream.  The fastest candidate is applied and,
// when a cache file is given, recorded under a key made of the GPU architecture and
// the batch's signature (the sorted (devices, colours) pairs of its circuits); a
// later call with the same key applies the recorded choice without timing.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "colorstamp.h"
#include "internal.hpp"

using namespace cs;

namespace {

cs_status tfail(cs_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

// Candidates, in the order they are timed.
std::vector<cs_batch_config> candidates() {
    std::vector<cs_batch_config> v;
    for (int32_t block : {128, 256})
        for (int32_t local : {0, 64, 256, 1024, 4096})
            for (int32_t ea : {-1, 0}) v.push_back({CS_COLOR_PERSISTENT, block, ea, local, 0.0});
    for (int32_t block : {128, 192, 256}) v.push_back({CS_COLOR_REGION, block, -1, 0, 0.0});
    return v;
}

// FNV-1a over the sorted (devices, colours) pairs of the batch's circuits.
std::string signature(const cs_batch *B, const char *arch) {
    std::vector<std::pair<int64_t, int64_t>> sz;
    for (const cs_circuit *c : B->circ) sz.emplace_back(c->h.n_dev, c->h.n_colors);
    std::sort(sz.begin(), sz.end());
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t x) {
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((x >> (8 * k)) & 0xFF);
            h *= 1099511628211ull;
        }
    };
    mix((int64_t)sz.size());
    for (auto &p : sz) {
        mix(p.first);
        mix(p.second);
    }
    char buf[32];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    std::string a(arch);
    for (char &ch : a)
        if (ch == ' ') ch = '_';
    return a + ":" + buf;
}

// Cache lines: key schedule block eval_ahead local_max_dev ms
bool cache_lookup(const char *path, const std::string &key, cs_batch_config *cfg) {
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string k;
        cs_batch_config c{};
        if (ls >> k >> c.schedule >> c.block >> c.eval_ahead >> c.local_max_dev >> c.ms && k == key) {
            *cfg = c;   // the last line of a key wins
            found = true;
        }
    }
    return found;
}

cs_status apply(cs_batch *B, const cs_batch_config &c, const double *W, const double *L, const double *V,
                hipStream_t s) {
    cs_status st = cs_batch_set_launch(B, c.block, c.eval_ahead, c.local_max_dev);
    if (st == CS_OK) st = cs_batch_set_schedule(B, (cs_variant)c.schedule);
    if (st == CS_OK) st = cs_batch_set_params(B, W, L, V, s);
    return st;
}

// Mean milliseconds of one captured step over reps replays; false when the
// configuration does not run on this device.
bool time_config(cs_batch *B, const double *x, double ag0, double *A, double *b, int32_t reps, hipStream_t s,
                 double *ms) {
    // one ordinary call first: plans, uploads and allocations happen outside the capture
    if (cs_batch_eval_stamp(B, x, ag0, nullptr, A, b, s) != CS_OK) return false;
    if (cs_batch_check(B, s) != CS_OK) return false;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
    const cs_status st = cs_batch_eval_stamp(B, x, ag0, nullptr, A, b, s);
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (st != CS_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return false;
    }
    bool ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    ok = ok && hipGraphLaunch(ge, s) == hipSuccess;
    ok = ok && hipEventRecord(e0, s) == hipSuccess;
    for (int32_t r = 0; ok && r < reps; ++r) ok = hipGraphLaunch(ge, s) == hipSuccess;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float t = 0.0f;
    ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ge) (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    // a bounded barrier wait that expired marks the configuration unusable
    if (cs_batch_check(B, s) != CS_OK) return false;
    *ms = (double)t / reps;
    return ok;
}

}  // namespace

extern "C" cs_status cs_batch_tune(cs_batch *B, const double *W, const double *L, const double *VTH0,
                                   const double *x, double ag0, double *A, double *b_vec, int32_t reps,
                                   const char *cache_path, cs_batch_config *best, int32_t *n_tried,
                                   int32_t *cached, void *stream) {
    if (!B) return tfail(CS_EINVAL, "NULL batch");
    if (!W || !L || !VTH0 || !x || !A || !b_vec) return tfail(CS_EINVAL, "NULL argument");
    if (reps < 1 || reps > 100000) return tfail(CS_EINVAL, "reps must be in 1..100000");
    // the caller's stream may be the legacy default stream, which cannot be captured:
    // the tuner works on a stream of its own (default priority) once the caller's
    // stream has produced the inputs, and synchronises it before returning
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return tfail(CS_EHIP, "stream synchronise");
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return tfail(CS_EHIP, "stream create");
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    } guard{s};
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return tfail(CS_EHIP, "no HIP device");
    std::string key;
    try {
        key = signature(B, prop.gcnArchName);
    } catch (...) {
        return tfail(CS_ENOMEM, "host allocation");
    }
    if (n_tried) *n_tried = 0;
    if (cached) *cached = 0;
    cs_batch_config pick{};
    if (cache_path && cache_lookup(cache_path, key, &pick)) {
        cs_status st = apply(B, pick, W, L, VTH0, s);
        if (st != CS_OK) return st;
        if (best) *best = pick;
        if (cached) *cached = 1;
        return CS_OK;
    }
    bool have = false;
    int32_t tried = 0;
    for (const cs_batch_config &c : candidates()) {
        if (apply(B, c, W, L, VTH0, s) != CS_OK) continue;
        double ms = 0.0;
        if (!time_config(B, x, ag0, A, b_vec, reps, s, &ms)) continue;
        ++tried;
        if (!have || ms < pick.ms) {
            pick = c;
            pick.ms = ms;
            have = true;
        }
    }
    if (!have) return tfail(CS_ENOTSUP, "no candidate configuration runs on this device");
    cs_status st = apply(B, pick, W, L, VTH0, s);
    if (st != CS_OK) return st;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (!out) return tfail(CS_EINVAL, std::string("cannot write the tuning cache ") + cache_path);
        char line[256];
        std::snprintf(line, sizeof line, "%s %d %d %d %d %.6f\n", key.c_str(), pick.schedule, pick.block,
                      pick.eval_ahead, pick.local_max_dev, pick.ms);
        out << line;
    }
    if (best) *best = pick;
    if (n_tried) *n_tried = tried;
    return CS_OK;
}

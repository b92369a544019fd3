// Autotuner for the batched executor: per log2 size class, time fused
// launches of puts at each candidate (scope, work-group size, chunk) and keep
// the fastest.  Results can be saved and loaded as JSON keyed by device name.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace vshmem;

namespace {

struct Cand {
    int scope;
    int wg;
    uint64_t chunk;
};

// Median time (ms) of `reps` fused launches of `msgs` puts of `bytes` each.
int time_candidate(const Cand &c, uint64_t off, uint64_t span, uint64_t bytes, int msgs, int reps, hipStream_t s,
                   float *ms_out)
{
    const State &st_ = st();
    const int npes = st_.npes;
    // Messages go PE i -> i+1 at consecutive offsets of the scratch range;
    // source and destination halves do not overlap.
    const uint64_t half = span / 2;
    const uint64_t per = std::max<uint64_t>(1, half / std::max<uint64_t>(1, bytes));
    // Message m: PE m mod npes -> next PE, slot m / npes; (target, slot)
    // pairs are distinct while m < npes * per, so no two messages overlap.
    const uint64_t nmsg = std::min<uint64_t>((uint64_t)msgs, (uint64_t)npes * per);
    std::vector<shmemx_desc_t> d;
    for (uint64_t m = 0; m < nmsg; ++m) {
        shmemx_desc_t x{};
        x.op = SHMEMX_OP_PUT;
        x.scope = (uint8_t)c.scope;
        x.issuer_pe = (int32_t)(m % npes);
        x.target_pe = (int32_t)((m + 1) % npes);
        x.result_idx = SHMEMX_NO_RESULT;
        const uint64_t slot = m / npes;
        x.src = off + slot * bytes;
        x.dst = off + half + slot * bytes;
        x.nbytes = bytes;
        d.push_back(x);
    }
    shmemx_tune_t t;
    shmemx_tune_default(&t);
    t.wg_size = c.wg;
    for (int k = 0; k < SHMEMX_TUNE_CLASSES; ++k) t.chunk[k] = c.chunk;
    shmemx_plan_t *plan = nullptr;
    int rc = shmemx_plan_create(d.data(), d.size(), &t, &plan);
    if (rc) return rc;
    hipEvent_t e0, e1;
    VSHMEM_HIP(hipEventCreate(&e0));
    VSHMEM_HIP(hipEventCreate(&e1));
    std::vector<float> ts;
    for (int r = 0; r < reps + 1 && !rc; ++r) {
        (void)hipEventRecord(e0, s);
        rc = shmemx_plan_launch_fused(plan, nullptr, s);
        (void)hipEventRecord(e1, s);
        if (VSHMEM_HIP_FAILED(hipEventSynchronize(e1))) rc = SHMEMX_ERR_HIP;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) ts.push_back(ms);   // first launch is a warm-up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    shmemx_plan_destroy(plan);
    if (rc) return rc;
    std::sort(ts.begin(), ts.end());
    *ms_out = ts[ts.size() / 2];
    return SHMEMX_OK;
}

// Key of the current device in saved tables: its architecture name, or
// empty when no device is visible.
std::string device_key()
{
    hipDeviceProp_t prop{};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    return std::string(prop.gcnArchName);
}

}  // namespace

extern "C" {

int shmemx_autotune(uint64_t scratch_off, uint64_t scratch_bytes, uint64_t min_bytes, uint64_t max_bytes, int msgs,
                    int reps, shmemx_tune_t *tune, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!tune || msgs <= 0 || reps <= 0 || min_bytes == 0 || max_bytes < min_bytes ||
        !in_user_heap(scratch_off, scratch_bytes) || scratch_bytes < 2 * max_bytes || st().npes < 2)
        return SHMEMX_ERR_ARG;
    shmemx_tune_default(tune);
    hipStream_t s = (hipStream_t)stream;
    const int wgs[] = {64, 128, 256, 512, 1024};
    const uint64_t chunks[] = {0, 64ull << 10, 256ull << 10, 1ull << 20};
    for (uint64_t b = min_bytes; b <= max_bytes; b *= 2) {
        int cls = 0;
        while (cls + 1 < SHMEMX_TUNE_CLASSES && (2ull << cls) <= b) ++cls;
        float best = 1e30f;
        Cand pick{SHMEMX_SCOPE_WG, 256, 0};
        for (int sc = SHMEMX_SCOPE_THREAD; sc <= SHMEMX_SCOPE_WG; ++sc) {
            for (int wg : wgs) {
                for (uint64_t ch : chunks) {
                    if (sc != SHMEMX_SCOPE_WG && ch != 0) continue;
                    if (ch != 0 && ch >= b) continue;
                    Cand c{sc, wg, ch};
                    float ms = 0;
                    int rc = time_candidate(c, scratch_off, scratch_bytes, b, msgs, reps, s, &ms);
                    if (rc == SHMEMX_ERR_UNSUPPORTED) continue;   // this work-group size cannot be resident
                    if (rc) return rc;
                    if (ms < best) {
                        best = ms;
                        pick = c;
                    }
                }
            }
        }
        tune->scope[cls] = (uint8_t)pick.scope;
        tune->chunk[cls] = pick.chunk;
        // One work-group size serves the whole fused kernel: keep the one
        // that won the largest class.
        tune->wg_size = pick.wg;
        if (b > max_bytes / 2) break;
    }
    return SHMEMX_OK;
}

int shmemx_tune_save(const shmemx_tune_t *t, const char *path)
{
    if (!t || !path) return SHMEMX_ERR_ARG;
    const std::string key = device_key();
    FILE *f = fopen(path, "w");
    if (!f) return SHMEMX_ERR_ARG;
    fprintf(f, "{\n  \"device\": \"%s\",\n  \"wg_size\": %d,\n  \"grid_wgs\": %d,\n  \"classes\": [\n",
            key.c_str(), t->wg_size, t->grid_wgs);
    for (int c = 0; c < SHMEMX_TUNE_CLASSES; ++c)
        fprintf(f, "    {\"log2\": %d, \"scope\": %d, \"chunk\": %llu}%s\n", c, t->scope[c],
                (unsigned long long)t->chunk[c], c + 1 < SHMEMX_TUNE_CLASSES ? "," : "");
    fprintf(f, "  ]\n}\n");
    fclose(f);
    return SHMEMX_OK;
}

int shmemx_tune_load(shmemx_tune_t *out, const char *path)
{
    if (!out || !path) return SHMEMX_ERR_ARG;
    shmemx_tune_t *t = nullptr;
    FILE *f = fopen(path, "r");
    if (!f) return SHMEMX_ERR_ARG;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    fclose(f);
    // The table is only valid on the kind of device it was measured on.
    const std::string here = device_key();
    {
        const size_t k0 = s.find("\"device\"");
        const size_t q0 = k0 == std::string::npos ? k0 : s.find('"', s.find(':', k0));
        const size_t q1 = q0 == std::string::npos ? q0 : s.find('"', q0 + 1);
        const std::string saved = q1 == std::string::npos ? std::string() : s.substr(q0 + 1, q1 - q0 - 1);
        if (k0 == std::string::npos || saved != here) {
            set_error_detail(SHMEMX_ERR_ARG, "tune table %s was saved on device '%s', this is '%s'", path,
                             saved.c_str(), here.c_str());
            return SHMEMX_ERR_ARG;
        }
    }
    shmemx_tune_t tmp;
    shmemx_tune_default(&tmp);
    t = &tmp;
    auto num_after = [&](const std::string &key, size_t from, long long *v) -> size_t {
        size_t p = s.find(key, from);
        if (p == std::string::npos) return p;
        p = s.find(':', p);
        if (p == std::string::npos) return p;
        *v = strtoll(s.c_str() + p + 1, nullptr, 10);
        return p;
    };
    long long v = 0;
    if (num_after("\"wg_size\"", 0, &v) != std::string::npos) t->wg_size = (int)v;
    if (num_after("\"grid_wgs\"", 0, &v) != std::string::npos) t->grid_wgs = (int)v;
    size_t pos = s.find("\"classes\"");
    while (pos != std::string::npos) {
        long long lg = 0, sc = 0, ch = 0;
        size_t p1 = num_after("\"log2\"", pos, &lg);
        if (p1 == std::string::npos) break;
        size_t p2 = num_after("\"scope\"", p1, &sc);
        size_t p3 = p2 == std::string::npos ? p2 : num_after("\"chunk\"", p2, &ch);
        if (p3 == std::string::npos) break;
        if (lg >= 0 && lg < SHMEMX_TUNE_CLASSES) {
            t->scope[lg] = (uint8_t)sc;
            t->chunk[lg] = (uint64_t)ch;
        }
        pos = p3 + 1;
    }
    if (check_tune(tmp)) return SHMEMX_ERR_ARG;
    *out = tmp;
    return SHMEMX_OK;
}

}  // extern "C"

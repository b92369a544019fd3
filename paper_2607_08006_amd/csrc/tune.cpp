// Autotuner for the batched executor: per log2 size class, time fused
// launches of puts at each candidate (scope, work-group size, chunk) and keep
// the fastest.  Results can be saved and loaded as JSON keyed by device name.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "exec.hpp"
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

// Host-side SplitMix64 for the tuner's synthetic mix (input generation).
uint64_t mix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The served mix the candidates are scored on, shaped like the 4-PE mixed
// program: `msgs` put/get (half each) with sizes uniform in [min_bytes,
// max_bytes] between random PEs, in eight epochs separated by barriers of
// every PE; then one epoch of 10 * msgs thread-scope fetch_add(+1) on 64
// counters at the end of the range (contended: that program's 10^4 atomics
// to 1000 put/get).  Offsets are multiples of 8, as in that program, so that source
// and destination agree modulo 16 for about half of the messages.  Sources
// lie in the first half of the range, destinations in the second; the
// destinations of one epoch are disjoint (no conflicts), and the next epoch,
// after its barrier, uses the same space again.
std::vector<shmemx_desc_t> make_mix(uint64_t off, uint64_t span, uint64_t min_b, uint64_t max_b, int msgs)
{
    const int npes = st().npes;
    const uint64_t ctr = (off + span - 64 * 8) & ~7ull;   // 64 aligned counters
    const uint64_t half = (ctr - off) / 2;
    std::vector<shmemx_desc_t> d;
    const int epochs = 8;
    uint64_t k = 0;
    auto barrier = [&]() {
        for (int p = 0; p < npes; ++p) {
            shmemx_desc_t x{};
            x.op = SHMEMX_OP_BARRIER_ALL;
            x.issuer_pe = p;
            x.target_pe = p;
            x.result_idx = SHMEMX_NO_RESULT;
            d.push_back(x);
        }
    };
    for (int e = 0; e < epochs; ++e) {
        uint64_t used = 0;
        for (int m = e * msgs / epochs; m < (e + 1) * msgs / epochs; ++m) {
            const uint64_t n = min_b + mix64(0x7E57, k++) % (max_b - min_b + 1);
            const uint64_t n8 = (n + 7) & ~7ull;
            if (used + n8 > half) break;
            shmemx_desc_t x{};
            x.op = (mix64(0x7E57, k++) & 1) ? SHMEMX_OP_PUT : SHMEMX_OP_GET;
            x.scope = SHMEMX_SCOPE_AUTO;
            x.issuer_pe = (int32_t)(mix64(0x7E57, k++) % (uint64_t)npes);
            x.target_pe = (int32_t)(mix64(0x7E57, k++) % (uint64_t)npes);
            x.result_idx = SHMEMX_NO_RESULT;
            x.src = off + (mix64(0x7E57, k++) % ((half - n) / 8 + 1)) * 8;
            x.dst = off + half + used;
            x.nbytes = n;
            used += n8;
            d.push_back(x);
        }
        barrier();
    }
    for (int a = 0; a < 10 * msgs; ++a) {
        shmemx_desc_t x{};
        x.op = SHMEMX_OP_AMO_FETCH_ADD;
        x.scope = SHMEMX_SCOPE_THREAD;   // one lane per atomic, as the program issues them
        x.issuer_pe = (int32_t)(mix64(0x7E58, k++) % (uint64_t)npes);
        const uint64_t c = mix64(0x7E58, k++) % 64;
        x.target_pe = (int32_t)(c % (uint64_t)npes);
        x.result_idx = SHMEMX_NO_RESULT;
        x.src = ctr + 8 * c;
        x.nbytes = 8;
        x.value = 1;
        d.push_back(x);
    }
    barrier();
    return d;
}

// Median time (ms) of `reps` fused launches of the mix under `t`;
// SHMEMX_ERR_UNSUPPORTED when its work-groups cannot be resident.
int score_table(const std::vector<shmemx_desc_t> &mix, const shmemx_tune_t &t, int reps, hipStream_t s, float *ms)
{
    shmemx_plan_t *plan = nullptr;
    int rc = shmemx_plan_create(mix.data(), mix.size(), &t, &plan);
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
        float x = 0;
        (void)hipEventElapsedTime(&x, e0, e1);
        if (r > 0) ts.push_back(x);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    shmemx_plan_destroy(plan);
    if (rc) return rc;
    std::sort(ts.begin(), ts.end());
    *ms = ts[ts.size() / 2];
    return SHMEMX_OK;
}

}  // namespace

extern "C" {

int shmemx_autotune(uint64_t scratch_off, uint64_t scratch_bytes, uint64_t min_bytes, uint64_t max_bytes, int msgs,
                    int reps, shmemx_tune_t *tune, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!tune || msgs <= 0 || reps <= 0 || min_bytes == 0 || max_bytes < min_bytes ||
        !in_user_heap(scratch_off, scratch_bytes) || scratch_bytes < 2 * max_bytes + 1024 || st().npes < 2)
        return SHMEMX_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int wgs[] = {64, 128, 256, 512, 1024};
    const uint64_t chunks[] = {0, 64ull << 10, 256ull << 10, 1ull << 20};
    const std::vector<shmemx_desc_t> mix = make_mix(scratch_off, scratch_bytes, min_bytes, max_bytes, msgs);
    // Whole tables differ by a few percent on the mix, about as much as one
    // median moves from run to run: every table is scored once here, and
    // the best few again below, in turns.
    const int mix_reps = std::max(reps, 9);
    std::vector<std::pair<float, shmemx_tune_t>> scored;
    auto consider = [&](const shmemx_tune_t &t) -> int {
        float ms = 0;
        const int rc = score_table(mix, t, mix_reps, s, &ms);
        if (rc == SHMEMX_ERR_UNSUPPORTED) return SHMEMX_OK;   // not resident at this work-group size
        if (rc) return rc;
        scored.emplace_back(ms, t);
        return SHMEMX_OK;
    };
    for (int wg : wgs) {
        // Per size class, the fastest (scope, chunk) at THIS work-group size
        // on isolated puts of that class ...
        shmemx_tune_t t;
        shmemx_tune_default(&t);
        t.wg_size = wg;
        bool resident = true;
        for (uint64_t b = min_bytes; b <= max_bytes && resident; b *= 2) {
            const int cls = vshmem_exec::size_class(b);
            float cls_best = 1e30f;
            for (int sc = SHMEMX_SCOPE_THREAD; sc <= SHMEMX_SCOPE_WG; ++sc) {
                for (uint64_t ch : chunks) {
                    if (sc != SHMEMX_SCOPE_WG && ch != 0) continue;
                    if (ch != 0 && ch >= b) continue;
                    float ms = 0;
                    const int rc = time_candidate(Cand{sc, wg, ch}, scratch_off, scratch_bytes, b, msgs, reps, s, &ms);
                    if (rc == SHMEMX_ERR_UNSUPPORTED) {
                        resident = false;
                        break;
                    }
                    if (rc) return rc;
                    if (ms < cls_best) {
                        cls_best = ms;
                        t.scope[cls] = (uint8_t)sc;
                        t.chunk[cls] = ch;
                    }
                }
                if (!resident) break;
            }
            if (b > max_bytes / 2) break;
        }
        if (!resident) continue;
        // ... and the whole table, with the fixed tables of this size,
        // scored together on the mix: the work-group size is chosen with
        // the scopes it was tuned for.
        if (int rc = consider(t)) return rc;
        for (int sc = SHMEMX_SCOPE_THREAD; sc <= SHMEMX_SCOPE_WG; ++sc) {
            shmemx_tune_t u;
            shmemx_tune_default(&u);
            u.wg_size = wg;
            for (int c = 0; c < SHMEMX_TUNE_CLASSES; ++c) u.scope[c] = (uint8_t)sc;
            if (int rc = consider(u)) return rc;
        }
        shmemx_tune_t d;
        shmemx_tune_default(&d);
        d.wg_size = wg;
        if (int rc = consider(d)) return rc;
    }
    if (scored.empty()) {   // no work-group size was resident: the built-in table
        shmemx_tune_default(tune);
        return SHMEMX_OK;
    }
    // The finalists: the four best single scores, re-scored in five rounds
    // that visit each in turn (so that a drift of the device's speed during
    // tuning touches them alike); the lowest sum of round medians wins.
    std::stable_sort(scored.begin(), scored.end(),
                     [](const std::pair<float, shmemx_tune_t> &a, const std::pair<float, shmemx_tune_t> &b) {
                         return a.first < b.first;
                     });
    const size_t nf = std::min<size_t>(scored.size(), 4);
    std::vector<float> total(nf, 0.0f);
    for (int round = 0; round < 5; ++round) {
        for (size_t i = 0; i < nf; ++i) {
            float ms = 0;
            if (int rc = score_table(mix, scored[i].second, mix_reps, s, &ms)) return rc;
            total[i] += ms;
        }
    }
    size_t win = 0;
    for (size_t i = 1; i < nf; ++i)
        if (total[i] < total[win]) win = i;
    *tune = scored[win].second;
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

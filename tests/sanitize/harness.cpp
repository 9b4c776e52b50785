// Host-side sanitizer harness for the library's C ABI (CPU only, no GPU).
//
// Built by tests/test_host_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of capi.cpp and tune.hip (and
// this file), linked against the ordinary objects of the kernel sources.  It
// runs three groups of checks and exits non-zero on the first failure (the
// sanitizers abort on their own findings):
//   1. tuning-file parser fuzz: seed documents (one written by ca_tune_save
//      from a host-built context, and the packaged cache) are mutated by a
//      seeded generator (byte flips, insertions, deletions, truncation,
//      duplicated ranges, extreme numbers, deep nesting) and fed to
//      ca_tune_load; the status must be CA_OK or CA_ERR_INVALID_ARG, and a
//      refused file must leave the context's choices unchanged;
//   2. argument-validation fuzz: every entry point called with random counts,
//      sizes, option values and NULL / non-NULL pointers, on a NULL context,
//      a dummy handle and a host-built context; a call must return a status
//      (validation errors, or HIP errors where nothing can run on this host);
//   3. tuning knobs: ca_tune_set / ca_tune_get over random keys and values,
//      with ca_tune_save / ca_tune_load round trips.
// The host-built context has no device tables (no GPU here): argument checks,
// the parser and the tuning tables are host code and are exercised fully.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/curvealign.h"
#include "../../paper_2501_17779_amd/csrc/context.hpp"

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
// splitmix64 (Steele, Lea, Flood 2014)
uint64_t rnd() {
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
int rint_(int lo, int hi) { return lo + (int)(rnd() % (uint64_t)(hi - lo + 1)); }

int g_fail = 0;
#define CHECK(cond, ...)                                                   \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "CHECK failed at line %d: ", __LINE__);        \
            fprintf(stderr, __VA_ARGS__);                                  \
            fprintf(stderr, "\n");                                         \
            ++g_fail;                                                      \
        }                                                                  \
    } while (0)

std::string read_file(const std::string& p) {
    std::string s;
    FILE* f = fopen(p.c_str(), "rb");
    if (!f) return s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
    fclose(f);
    return s;
}
void write_file(const std::string& p, const std::string& s) {
    FILE* f = fopen(p.c_str(), "wb");
    if (!f) { perror("fopen"); exit(3); }
    fwrite(s.data(), 1, s.size(), f);
    fclose(f);
}

ca_context* host_context() {
    ca_context* c = new ca_context();
    c->device = 0;
    c->num_cus = 256;
    c->arch = "gfx950";
    return c;
}

std::string snapshot(ca_context* c, const std::string& dir) {
    const std::string p = dir + "/snap.json";
    const ca_status_t st = ca_tune_save(c, p.c_str());
    CHECK(st == CA_OK, "ca_tune_save: %d %s", st, ca_last_error());
    return read_file(p);
}

std::string mutate(const std::string& src) {
    std::string s = src;
    static const char alphabet[] = "{}[]\":,-+.eE0123456789 \t\nabcdefghijklmnopqrstuvwxyz\\/\x01\x7f\xff";
    const int rounds = rint_(1, 6);
    for (int r = 0; r < rounds; ++r) {
        const size_t n = s.size();
        switch (rint_(0, 8)) {
            case 0:   // flip a byte
                if (n) s[rnd() % n] = alphabet[rnd() % (sizeof(alphabet) - 1)];
                break;
            case 1: {  // insert characters
                const size_t at = n ? rnd() % (n + 1) : 0;
                std::string ins;
                for (int k = rint_(1, 8); k > 0; --k) ins.push_back(alphabet[rnd() % (sizeof(alphabet) - 1)]);
                s.insert(at, ins);
                break;
            }
            case 2:   // delete a range
                if (n) {
                    const size_t at = rnd() % n;
                    s.erase(at, (size_t)rint_(1, 40));
                }
                break;
            case 3:   // truncate
                if (n) s.resize(rnd() % n);
                break;
            case 4:   // duplicate a range
                if (n > 2) {
                    const size_t a = rnd() % n, len = 1 + rnd() % std::min<size_t>(200, n - a);
                    s.insert(rnd() % (n + 1), s.substr(a, len));
                }
                break;
            case 5: {  // replace a number by an extreme or odd one
                static const char* nums[] = {"1e308", "-1e308", "1e999", "2147483648", "-2147483649", "0.5",
                                             "-0", "1e-400", "9999999999999999999999", "16", "8192", "-1", "NaN"};
                for (size_t i = 0; i < s.size(); ++i)
                    if (s[i] >= '0' && s[i] <= '9' && (rnd() & 7) == 0) {
                        size_t j = i;
                        while (j < s.size() && ((s[j] >= '0' && s[j] <= '9') || s[j] == '.')) ++j;
                        s.replace(i, j - i, nums[rnd() % (sizeof(nums) / sizeof(nums[0]))]);
                        break;
                    }
                break;
            }
            case 6: {  // deep nesting
                const int d = rint_(10, 40);
                s = std::string(d, '[') + s + std::string(d, ']');
                break;
            }
            case 7:   // swap a knob name
                for (const char* k : {"team_grid", "allpairs_cols", "block_plan", "block_grid", "block_threads"}) {
                    const size_t at = s.find(k);
                    if (at != std::string::npos && (rnd() & 1)) {
                        static const char* other[] = {"team_grid", "block_plan", "nope", "", "block_threads"};
                        s.replace(at, strlen(k), other[rnd() % 5]);
                        break;
                    }
                }
                break;
            default: {  // escapes inside a string
                const size_t at = s.find('"');
                if (at != std::string::npos) s.insert(at + 1, (rnd() & 1) ? "\\\"" : "\\x");
                break;
            }
        }
    }
    return s;
}

void fuzz_parser(const std::string& dir, const std::vector<std::string>& seeds, int iters) {
    ca_context* c = host_context();
    std::string before = snapshot(c, dir);
    const std::string path = dir + "/fuzz.json";
    int accepted = 0, refused = 0;
    for (int i = 0; i < iters; ++i) {
        const std::string doc = mutate(seeds[rnd() % seeds.size()]);
        write_file(path, doc);
        int32_t applied = -1;
        const ca_status_t st = ca_tune_load(c, path.c_str(), &applied);
        CHECK(st == CA_OK || st == CA_ERR_INVALID_ARG, "ca_tune_load status %d", st);
        if (st == CA_OK) {
            ++accepted;
            CHECK(applied >= 0, "applied %d", applied);
            before = snapshot(c, dir);       // a valid file may change the choices
        } else {
            ++refused;
            CHECK(applied == 0, "refused file applied %d entries", applied);
            CHECK(strlen(ca_last_error()) > 0, "no error text");
            const std::string after = snapshot(c, dir);
            CHECK(after == before, "a refused file changed the context's choices");
        }
    }
    printf("parser fuzz: %d documents, %d accepted, %d refused\n", iters, accepted, refused);
    ca_destroy(c);
}

void* rptr() {
    switch (rnd() % 3) {
        case 0: return nullptr;
        case 1: return (void*)(uintptr_t)0x2000;
        default: return (void*)(uintptr_t)(0x10000 + 64 * (rnd() % 1024));
    }
}
int32_t rn() {
    static const int32_t v[] = {-5, -1, 0, 1, 2, 3, 11, 64, 96, 128, 256, 300, 512, 1000, 1009, 1024,
                                2048, 4093, 4096, 4097, 8192, 65536, 0x7fffffff, (int32_t)0x80000000};
    return v[rnd() % (sizeof(v) / sizeof(v[0]))];
}
int64_t rcount() {
    static const int64_t v[] = {-3, -1, 0, 1, 4, 1000, (int64_t)1 << 31, (int64_t)1 << 40};
    return v[rnd() % (sizeof(v) / sizeof(v[0]))];
}

void fuzz_arguments(int iters) {
    ca_context* hc = host_context();
    // every case: the call returns (any status); with a NULL or dummy
    // context only argument errors are possible
    int calls = 0;
    for (int i = 0; i < iters; ++i) {
        const int which_ctx = rint_(0, 2);
        ca_context_t c = which_ctx == 0 ? nullptr : which_ctx == 1 ? (ca_context_t)(uintptr_t)0x1000 : hc;
        // with a dummy handle, keep to calls whose validation must fail before the context is used
        const bool dummy = which_ctx == 1;
        ca_options_t o{rint_(-1, 3), rint_(-1, 2), rint_(0, 1), rint_(0, 8) == 0 ? 1 : 0};
        const ca_options_t* op = (rnd() & 1) ? &o : nullptr;
        ca_status_t st = CA_OK;
        switch (rint_(0, 7)) {
            case 0:
                if (dummy) { st = align_batch(c, nullptr, rptr(), nullptr, rn(), rcount(), (ca_result_t*)rptr(), op, nullptr); }
                else { st = align_batch(c, rptr(), rptr(), (const int64_t*)((rnd() & 3) ? nullptr : rptr()), rn(),
                                        rint_(0, 3) ? (rnd() & 1 ? -1 : 0) : rcount(), (ca_result_t*)rptr(), op, nullptr); }
                break;
            case 1:
                if (dummy) st = align_pair(c, rptr(), rptr(), rn() < 2 ? rn() : 0, nullptr, op, nullptr);
                else st = align_pair(c, rptr(), rptr(), rn(), (ca_result_t*)((rnd() & 3) ? nullptr : rptr()), op, nullptr);
                break;
            case 2: {
                const int32_t m = rn();
                if (dummy) st = align_all_pairs(c, nullptr, m < 2 ? 8 : m, rn(), nullptr, op, nullptr);
                else st = align_all_pairs(c, rptr(), m < 0 ? m : (m > 4096 ? m : (rnd() & 3 ? m : -1)), rn(),
                                          (ca_result_t*)rptr(), op, nullptr);
                break;
            }
            case 3: {
                const int32_t m = rn();
                if (dummy) st = align_all_pairs_noalloc(c, nullptr, m < 2 ? 8 : m, rn(), nullptr, op, nullptr);
                else st = align_all_pairs_noalloc(c, rptr(), m, rn(), (ca_result_t*)rptr(), op, nullptr);
                break;
            }
            case 4:
                st = resample_arclength(c, dummy ? nullptr : rptr(), (const int64_t*)rptr(),
                                        dummy ? (rnd() & 1 ? -1 : 4) : (rint_(0, 3) ? -1 : rcount()),
                                        (const int64_t*)rptr(), rptr(), (double*)rptr(), (uint32_t*)rptr(),
                                        rint_(-1, 2), nullptr);
                break;
            case 5:
                st = to_initializer(c, (const ca_result_t*)(dummy ? nullptr : rptr()), rn(),
                                    (const int64_t*)((rnd() & 1) ? rptr() : nullptr),
                                    dummy ? 4 : (rint_(0, 3) ? -1 : rcount()), (double*)rptr(), (double*)rptr(),
                                    nullptr);
                break;
            case 6:
                st = srv_transform(c, dummy ? nullptr : rptr(), (const int64_t*)((rnd() & 1) ? rptr() : nullptr),
                                   rn(), dummy ? 4 : (rint_(0, 3) ? -1 : rcount()), rptr(), nullptr);
                break;
            default: {
                int32_t vals[16];
                int32_t cnt = rint_(-1, 17);
                for (int k = 0; k < 16; ++k) vals[k] = rn();
                if (dummy) st = ca_tune_set(c, rint_(-2, 6), rn(), nullptr, cnt);
                else st = (rnd() & 1) ? ca_tune_set(c, rint_(-2, 6), rn(), vals, cnt)
                                      : ca_tune_get(c, rint_(-2, 6), rn(), vals, &cnt);
                break;
            }
        }
        if (c == nullptr || dummy) CHECK(st == CA_OK || st == CA_ERR_INVALID_ARG || st == CA_ERR_UNSUPPORTED_N ||
                                             st == CA_ERR_TOO_LARGE,
                                         "status %d on a %s context", st, c ? "dummy" : "NULL");
        CHECK(st <= 0 && st >= CA_ERR_TOO_LARGE, "status %d outside the enum", st);
        ++calls;
    }
    printf("argument fuzz: %d calls\n", calls);
    ca_destroy(hc);
}

void tune_round_trips(const std::string& dir, int iters) {
    ca_context* a = host_context();
    ca_context* b = host_context();
    const std::string p = dir + "/rt.json";
    for (int i = 0; i < iters; ++i) {
        const int knob = rint_(0, 4);
        int32_t key = 0, vals[16], cnt = 1;
        switch (knob) {
            case CA_TUNE_TEAM_GRID: key = 64 << rint_(0, 4); vals[0] = rint_(0, 8); break;
            case CA_TUNE_ALLPAIRS_COLS: key = 64 << rint_(0, 4); vals[0] = rint_(1, 256); break;
            case CA_TUNE_BLOCK_GRID: key = rint_(0, 4); vals[0] = rint_(0, 8); break;
            case CA_TUNE_BLOCK_THREADS: key = rint_(3, 4); vals[0] = (rnd() & 1) ? 256 : 512; break;
            default: {
                static const int sizes[] = {2, 6, 64, 300, 1000, 2187, 3000, 4096, 6000, 8192};
                key = sizes[rnd() % 10];
                int m = key;
                cnt = 0;
                for (int p2 : {8, 4, 2, 3, 5, 7})
                    while (m % p2 == 0 && cnt < 16) { vals[cnt++] = p2; m /= p2; }
                for (int k = cnt - 1; k > 0; --k) { const int j = rint_(0, k); std::swap(vals[k], vals[j]); }
            }
        }
        const ca_status_t st = ca_tune_set(a, knob, key, vals, cnt);
        CHECK(st == CA_OK, "tune_set knob %d key %d: %s", knob, key, ca_last_error());
        int32_t got[16], gc = 16;
        CHECK(ca_tune_get(a, knob, key, got, &gc) == CA_OK && gc == cnt && memcmp(got, vals, 4 * cnt) == 0,
              "tune_get after tune_set, knob %d key %d", knob, key);
    }
    CHECK(ca_tune_save(a, p.c_str()) == CA_OK, "save");
    int32_t applied = 0;
    CHECK(ca_tune_load(b, p.c_str(), &applied) == CA_OK, "load: %s", ca_last_error());
    CHECK(snapshot(a, dir) == snapshot(b, dir), "saved and reloaded choices differ");
    printf("tuning round trips: %d settings, %d entries reloaded\n", iters, applied);
    ca_destroy(a);
    ca_destroy(b);
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 3) {
        fprintf(stderr, "usage: harness <tmpdir> <packaged tune cache> [iterations]\n");
        return 2;
    }
    const std::string dir = argv[1];
    const int iters = argc > 3 ? atoi(argv[3]) : 3000;
    // seed documents: a file written by ca_tune_save, and the packaged cache
    std::vector<std::string> seeds;
    {
        ca_context* c = host_context();
        const int32_t v2[] = {2}, v4[] = {4}, v512[] = {512}, plan[] = {4, 8, 8, 3};
        ca_tune_set(c, CA_TUNE_TEAM_GRID, 1024, v2, 1);
        ca_tune_set(c, CA_TUNE_ALLPAIRS_COLS, 512, v4, 1);
        ca_tune_set(c, CA_TUNE_BLOCK_THREADS, 3, v512, 1);
        ca_tune_set(c, CA_TUNE_BLOCK_PLAN, 768, plan, 4);
        seeds.push_back(snapshot(c, dir));
        ca_destroy(c);
        const std::string pkg = read_file(argv[2]);
        if (!pkg.empty()) seeds.push_back(pkg);
        seeds.push_back("{}");
        seeds.push_back("{\"format\": \"curvealign-tune/1\", \"arch\": \"gfx950\", \"num_cus\": 256, \"entries\": []}");
    }
    // status strings and the size predicate over the whole range
    for (int s = -10; s <= 2; ++s) CHECK(ca_status_string(s) != nullptr, "status string %d", s);
    for (int n = -10; n <= 9000; ++n) {
        const int32_t k = ca_n_supported(n);
        CHECK(k >= 0 && k <= 2, "ca_n_supported(%d) = %d", n, k);
    }
    fuzz_parser(dir, seeds, iters);
    fuzz_arguments(iters);
    tune_round_trips(dir, iters / 10 + 1);
    if (g_fail) {
        fprintf(stderr, "%d check(s) failed\n", g_fail);
        return 1;
    }
    printf("all host checks passed\n");
    return 0;
}

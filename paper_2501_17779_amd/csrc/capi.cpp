// C ABI of the library (declared in include/curvealign.h): contexts, plan and
// twiddle tables, argument validation and kernel dispatch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/curvealign.h"
#include "fft_engines.hpp"
#include "context.hpp"

namespace ca {
int64_t resample_slot_bytes();
int resample_max_raw();
}

using ca::Plan;

namespace {
thread_local std::string g_err;
// context whose ca_graph_begin capture is open on this thread: an entry point
// that fails meanwhile marks the capture as failed
thread_local ca_context* g_capturing = nullptr;

// Scratch of align_all_pairs_noalloc: per-curve spectra, then FP64 norms.
// Every device the library runs on holds its own copy at its own address, so
// host code never passes the array's name to a kernel; it uses the device
// address hipGetSymbolAddress returned for that device (noalloc_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[CA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Byte offset of the norms in the scratch and the total size a gallery needs.
int64_t noalloc_norms_offset(int64_t m, int64_t n) { return (m * n * 8 + 255) / 256 * 256; }
int64_t noalloc_bytes(int64_t m, int64_t n) { return noalloc_norms_offset(m, n) + m * 8; }
}  // namespace

namespace ca {
namespace host {

ca_status_t fail(ca_status_t st, const std::string& msg) {
    g_err = msg;
    if (g_capturing) g_capturing->capture_failed = true;
    return st;
}
ca_status_t hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    if (g_capturing) g_capturing->capture_failed = true;
    return CA_ERR_HIP;
}

bool smooth7_size(int m) {
    if (m < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (m % p == 0) m /= p;
    return m == 1;
}

bool smooth7(int n) { return n >= 2 && n <= CA_MAX_N && smooth7_size(n); }

// Transform size of the block engine for n in [2, CA_MAX_N]: n itself when it
// is 7-smooth, else the smallest 7-smooth M >= 2n (zero-padded correlation).
int transform_size(int n) {
    if (smooth7(n)) return n;
    int m = 2 * n;
    while (!smooth7_size(m)) ++m;
    return m;
}

// Default radix schedule of the block engine: eights, then a four or two,
// then the odd primes.
std::vector<int> default_radices(int n) {
    std::vector<int> r;
    if (n < 2) return r;   // no schedule (and no endless division of 0 by 8)
    int m = n;
    while (m % 8 == 0) { r.push_back(8); m /= 8; }
    if (m % 4 == 0) { r.push_back(4); m /= 4; }
    if (m % 2 == 0) { r.push_back(2); m /= 2; }
    for (int p : {3, 5, 7})
        while (m % p == 0) { r.push_back(p); m /= p; }
    return r;
}

bool valid_radices(int m, const std::vector<int>& r) {
    if (r.empty() || r.size() > 16) return false;
    int64_t prod = 1;
    for (int x : r) {
        if (x != 2 && x != 3 && x != 4 && x != 5 && x != 7 && x != 8 && x != 16) return false;
        if (x == 16 && m <= kBlkR16Min / 2) return false;   // only the large classes compile it
        prod *= x;
        if (prod > m) return false;
    }
    return prod == m;
}

Plan plan_from(int n, const std::vector<int>& r) {
    Plan p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.npass = (int32_t)r.size();
    for (size_t i = 0; i < r.size(); ++i) p.radix[i] = r[i];
    return p;
}

std::vector<int> radices_for(const ca_context* c, int m) {
    auto it = c->tune.blk_plan.find(m);
    return it != c->tune.blk_plan.end() ? it->second : default_radices(m);
}

}  // namespace host
}  // namespace ca

using namespace ca::host;

namespace {

// Per-pass twiddles of the block-engine plan p (layout in fft_engines.hpp):
// pass i, radix R, stride ns: w_{ns R}^{r k} = w_n^{r k n / (ns R)}.
void plan_twiddles(const Plan& p, const std::vector<double>& re, const std::vector<double>& im,
                   std::vector<double>& pre, std::vector<double>& pim) {
    pre.clear();
    pim.clear();
    int ns = 1;
    for (int i = 0; i < p.npass; ++i) {
        const int R = p.radix[i];
        const int stride = p.n / (ns * R);
        for (int r = 1; r < R; ++r)
            for (int k = 0; k < ns; ++k) {
                pre.push_back(re[(size_t)r * k * stride]);
                pim.push_back(im[(size_t)r * k * stride]);
            }
        ns *= R;
    }
}

// w_n^m = exp(-2 pi i m / n), computed in long double and rounded once.
void twiddles(int n, std::vector<double>& re, std::vector<double>& im) {
    re.resize(n);
    im.resize(n);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int m = 0; m < n; ++m) {
        const long double a = two_pi * (long double)m / (long double)n;
        long double c = cosl(a), s = -sinl(a);
        if (fabsl(c) < 1e-18L) c = 0.0L;
        if (fabsl(s) < 1e-18L) s = 0.0L;
        re[m] = (double)c;
        im[m] = (double)s;
    }
}

}  // namespace

namespace ca {
namespace host {

// Per-pass twiddles of transform size m under the context's radix schedule.
void block_twiddles(const ca_context* c, int m, std::vector<double>& pre, std::vector<double>& pim) {
    std::vector<double> re, im;
    twiddles(m, re, im);
    plan_twiddles(plan_from(m, radices_for(c, m)), re, im, pre, pim);
}

// Plans for every n and the twiddle arenas (one segment of m - 1 entries per
// 7-smooth transform size m; the segment length does not depend on the radix
// schedule, so the offsets are fixed).
ca_status_t ensure_tables(ca_context* c, bool need64) {
    if (!c->d_plans) {
        c->h_plans.assign(CA_MAX_N + 1, Plan{});
        c->tw_off.assign(kMaxM + 1, -1);
        std::vector<float> arena32;
        int64_t off = 0;
        std::vector<double> pre, pim;
        for (int m = 2; m <= kMaxM; ++m) {
            if (!smooth7_size(m)) continue;
            c->tw_off[m] = off;
            block_twiddles(c, m, pre, pim);
            for (size_t k = 0; k < pre.size(); ++k) {
                arena32.push_back((float)pre[k]);
                arena32.push_back((float)pim[k]);
            }
            off += (int64_t)pre.size();
        }
        for (int n = 2; n <= CA_MAX_N; ++n) {
            const int M = transform_size(n);
            c->h_plans[n] = plan_from(M, radices_for(c, M));
            c->h_plans[n].tw_off = c->tw_off[M];
        }
        hipError_t e;
        if ((e = hipMalloc(&c->d_plans, sizeof(Plan) * (CA_MAX_N + 1))) != hipSuccess)
            return fail(CA_ERR_OOM, "plan table allocation failed");
        if ((e = hipMemcpy(c->d_plans, c->h_plans.data(), sizeof(Plan) * (CA_MAX_N + 1),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "plan upload");
        if ((e = hipMalloc(&c->d_tw32, arena32.size() * sizeof(float))) != hipSuccess)
            return fail(CA_ERR_OOM, "twiddle arena allocation failed");
        if ((e = hipMemcpy(c->d_tw32, arena32.data(), arena32.size() * sizeof(float),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "twiddle upload");
    }
    if (need64 && !c->d_tw64) {
        std::vector<double> arena64, pre, pim;
        for (int m = 2; m <= kMaxM; ++m) {      // same order and offsets as the FP32 arena
            if (!smooth7_size(m)) continue;
            block_twiddles(c, m, pre, pim);
            for (size_t k = 0; k < pre.size(); ++k) {
                arena64.push_back(pre[k]);
                arena64.push_back(pim[k]);
            }
        }
        hipError_t e;
        if ((e = hipMalloc(&c->d_tw64, arena64.size() * sizeof(double))) != hipSuccess)
            return fail(CA_ERR_OOM, "FP64 twiddle arena allocation failed");
        if ((e = hipMemcpy(c->d_tw64, arena64.data(), arena64.size() * sizeof(double),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "FP64 twiddle upload");
    }
    return CA_OK;
}

ca_status_t upload_block_plans(ca_context* c, const std::vector<int>& sizes) {
    if (!c->d_plans || sizes.empty()) return CA_OK;   // tables not built yet: built later with the new schedules
    hipError_t e = hipDeviceSynchronize();            // no kernel may read the tables while they change
    if (e != hipSuccess) return hip_fail(e, "synchronise before the plan update");
    for (int n = 2; n <= CA_MAX_N; ++n) {
        const int m = c->h_plans[n].n;
        if (std::find(sizes.begin(), sizes.end(), m) == sizes.end()) continue;
        const int64_t off = c->h_plans[n].tw_off;
        c->h_plans[n] = plan_from(m, radices_for(c, m));
        c->h_plans[n].tw_off = off;
    }
    if ((e = hipMemcpy(c->d_plans, c->h_plans.data(), sizeof(Plan) * (CA_MAX_N + 1),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "plan upload");
    std::vector<double> pre, pim;
    for (int m : sizes) {
        block_twiddles(c, m, pre, pim);
        const size_t cnt = pre.size();
        std::vector<float> t32(2 * cnt);
        std::vector<double> t64(2 * cnt);
        for (size_t k = 0; k < cnt; ++k) {
            t32[2 * k] = (float)pre[k];
            t32[2 * k + 1] = (float)pim[k];
            t64[2 * k] = pre[k];
            t64[2 * k + 1] = pim[k];
        }
        const int64_t off = c->tw_off[m];
        if ((e = hipMemcpy((float*)c->d_tw32 + 2 * off, t32.data(), t32.size() * sizeof(float),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "twiddle upload");
        if (c->d_tw64 && (e = hipMemcpy((double*)c->d_tw64 + 2 * off, t64.data(),
                                        t64.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "FP64 twiddle upload");
    }
    return CA_OK;
}

// Team-engine twiddles per pass after the first: (radix RP, stride NS, table offset).
struct TeamPass { int rp, ns, off; };
std::vector<TeamPass> team_passes(int n) {
    switch (n) {
        case 64: return {{8, 8, 0}};
        case 128: return {{8, 16, 0}};
        case 256: return {{16, 16, 0}};
        case 512: return {{16, 16, 0}, {2, 256, 240}};
        case 1024: return {{16, 16, 0}, {4, 256, 240}};
        default: return {};
    }
}

ca_status_t ensure_team_tables(ca_context* c) {
    if (c->d_team_tw[6]) return CA_OK;
    for (int n : {64, 128, 256, 512, 1024}) {
        int lg = 0;
        while ((1 << lg) < n) ++lg;
        std::vector<float> tab(2 * (size_t)ca::team_twiddle_count(n), 0.0f);
        std::vector<double> re, im;
        for (const TeamPass& p : team_passes(n)) {
            const int M = p.ns * p.rp;
            twiddles(M, re, im);
            for (int r = 1; r < p.rp; ++r)
                for (int k = 0; k < p.ns; ++k) {
                    const size_t e = (size_t)p.off + (size_t)(r - 1) * p.ns + k;
                    tab[2 * e] = (float)re[(r * k) % M];
                    tab[2 * e + 1] = (float)im[(r * k) % M];
                }
        }
        void* d = nullptr;
        if (hipMalloc(&d, tab.size() * sizeof(float)) != hipSuccess)
            return fail(CA_ERR_OOM, "team twiddle table");
        hipError_t e = hipMemcpy(d, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "team twiddle upload");
        c->d_team_tw[lg] = d;
    }
    return CA_OK;
}

// BF16 round-to-nearest-even of a float; the split of w into hi + lo.
uint16_t bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}
void split_bf16(double w, uint16_t& hi, uint16_t& lo) {
    hi = bf16_rne((float)w);
    lo = bf16_rne((float)(w - bf16_value(hi)));
}

// Per-lane operands of the n = 128 split-BF16 kernel (layout of Bf16Lane):
// for lane l = 16 g + c and element e (part e / 4, index i = e % 4), the
// 16-point DFT matrix at (4 g + i, c) and the 8-point one at
// (4 (g % 2) + i, c % 8) when pair g / 2 equals pair c / 8 (else 0), each as
// the real-GEMM entry of output part ob (Re, Im) in BF16 hi and lo; then the
// twiddles w_128^{(4 (g % 2) + r) c} and w_128^{(4 g + r) (c % 8)}.
ca_status_t ensure_bf16_tables(ca_context* c) {
    if (c->d_bf16) return CA_OK;
    struct Lane {
        uint16_t k1[2][2][8];
        uint16_t k2[2][2][8];
        float twf[4][2];
        float twt[4][2];
    };
    static_assert(sizeof(Lane) == 192, "lane block");
    std::vector<Lane> lanes(64);
    const long double tp = 6.283185307179586476925286766559005768L;
    // real-GEMM entry of W_M^{n k} for input part `part` and output part ob
    auto wentry = [&](int M, int n, int k, int part, int ob) {
        const long double a = tp * (long double)((n * k) % M) / (long double)M;
        const double re = (double)cosl(a), im = (double)-sinl(a);
        if (part == 0) return ob == 0 ? re : im;
        return ob == 0 ? -im : re;
    };
    for (int l = 0; l < 64; ++l) {
        const int g = l / 16, col = l % 16;
        for (int ob = 0; ob < 2; ++ob)
            for (int e = 0; e < 8; ++e) {
                const int part = e / 4, i = e % 4;
                uint16_t hi, lo;
                split_bf16(wentry(16, 4 * g + i, col, part, ob), hi, lo);
                lanes[l].k1[ob][0][e] = hi;
                lanes[l].k1[ob][1][e] = lo;
                const bool same_pair = (g / 2) == (col / 8);
                split_bf16(same_pair ? wentry(8, 4 * (g % 2) + i, col % 8, part, ob) : 0.0, hi, lo);
                lanes[l].k2[ob][0][e] = hi;
                lanes[l].k2[ob][1][e] = lo;
            }
        for (int r = 0; r < 4; ++r) {
            const long double af = tp * (long double)(((4 * (g % 2) + r) * col) % 128) / 128.0L;
            const long double at = tp * (long double)(((4 * g + r) * (col % 8)) % 128) / 128.0L;
            lanes[l].twf[r][0] = (float)cosl(af);
            lanes[l].twf[r][1] = (float)-sinl(af);
            lanes[l].twt[r][0] = (float)cosl(at);
            lanes[l].twt[r][1] = (float)-sinl(at);
        }
    }
    if (hipMalloc(&c->d_bf16, sizeof(Lane) * 64) != hipSuccess) return fail(CA_ERR_OOM, "BF16 constants");
    hipError_t e = hipMemcpy(c->d_bf16, lanes.data(), sizeof(Lane) * 64, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "BF16 constants upload");
    return CA_OK;
}

// Device address of the scratch array on `device`, looked up once per device
// (the caller has made `device` current).
ca_status_t noalloc_scratch_ptr(int device, void** ptr) {
    if (device < 0 || device >= kMaxDevices) return fail(CA_ERR_NO_DEVICE, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(CA_ERR_INTERNAL, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return CA_OK;
}

// Per-lane operands of the n = 1024 split-BF16 kernel: for lane l = 32 h + c,
// K-half q and element e, the entries of the 32-point DFT matrix at row
// j = 16 q + 8 (e / 4) + 4 h + e % 4 and column c (Re, Im, -Im, each as BF16
// hi and lo), then the twiddles w_1024^{row(g, h) c}, row(g, h) =
// 8 (g / 4) + 4 h + g % 4, as float4 pairs (g = 2 i, 2 i + 1) at [i][l].
ca_status_t ensure_bf16_1k_tables(ca_context* c) {
    if (c->d_bf16_1k) return CA_OK;
    std::vector<unsigned char> buf(ca::kBf16Tables1kBytes, 0);
    uint16_t* kk = reinterpret_cast<uint16_t*>(buf.data());
    const long double tp = 6.283185307179586476925286766559005768L;
    for (int l = 0; l < 64; ++l) {
        const int h = l / 32, col = l % 32;
        for (int q = 0; q < 2; ++q)
            for (int e = 0; e < 8; ++e) {
                const int j = 16 * q + 8 * (e / 4) + 4 * h + (e % 4);
                const long double a = tp * (long double)((j * col) % 32) / 32.0L;
                const double re = (double)cosl(a), im = (double)-sinl(a);
                const double v[3] = {re, im, -im};
                for (int cls = 0; cls < 3; ++cls) {
                    uint16_t hi, lo;
                    split_bf16(v[cls], hi, lo);
                    // lane block: k[q][cls][hl][e], 96 halves per lane
                    kk[l * 96 + ((q * 3 + cls) * 2 + 0) * 8 + e] = hi;
                    kk[l * 96 + ((q * 3 + cls) * 2 + 1) * 8 + e] = lo;
                }
            }
    }
    float* tw = reinterpret_cast<float*>(buf.data() + 64 * 192);
    for (int i = 0; i < 8; ++i)
        for (int l = 0; l < 64; ++l)
            for (int u = 0; u < 2; ++u) {
                const int g = 2 * i + u, h = l / 32, col = l % 32;
                const int row = 8 * (g / 4) + 4 * h + (g % 4);
                const long double a = tp * (long double)((row * col) % 1024) / 1024.0L;
                tw[(i * 64 + l) * 4 + 2 * u] = (float)cosl(a);
                tw[(i * 64 + l) * 4 + 2 * u + 1] = (float)-sinl(a);
            }
    if (hipMalloc(&c->d_bf16_1k, buf.size()) != hipSuccess) return fail(CA_ERR_OOM, "BF16 n = 1024 constants");
    hipError_t e = hipMemcpy(c->d_bf16_1k, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "BF16 n = 1024 constants upload");
    return CA_OK;
}

// Grows a context-owned workspace buffer to at least `need` bytes.  The
// outgrown buffer is retired, not freed: a HIP graph captured earlier may
// still hold its address, so it stays allocated until ca_destroy.
ca_status_t grow(ca_context* c, void** p, size_t* cap, size_t need, const char* what) {
    if (need <= *cap && *p) return CA_OK;
    void* q = nullptr;
    if (hipMalloc(&q, need) != hipSuccess) return fail(CA_ERR_OOM, std::string(what) + " allocation failed");
    if (*p) c->retired.push_back(*p);
    *p = q;
    *cap = need;
    return CA_OK;
}

const void* team_tw_for(ca_context* c, int n) {
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    return c->d_team_tw[lg];
}

ca_status_t parse_opts(const ca_options_t* opt, ca_options_t& o) {
    o = ca_options_t{CA_PREC_FP32, CA_RESCORE_TOP2, 0, 0};
    if (!opt) return CA_OK;
    o = *opt;
    if (o.precision != CA_PREC_FP32 && o.precision != CA_PREC_SPLIT_BF16 && o.precision != CA_PREC_FP64)
        return fail(CA_ERR_INVALID_ARG, "options.precision must be CA_PREC_FP32, _SPLIT_BF16 or _FP64");
    if (o.rescore != CA_RESCORE_TOP2 && o.rescore != CA_RESCORE_WINDOW)
        return fail(CA_ERR_INVALID_ARG, "options.rescore must be CA_RESCORE_TOP2 or _WINDOW");
    if (o.reserved != 0) return fail(CA_ERR_INVALID_ARG, "options.reserved must be 0");
    return CA_OK;
}

}  // namespace host
}  // namespace ca

extern "C" {

const char* ca_status_string(ca_status_t s) {
    switch (s) {
        case CA_OK: return "ok";
        case CA_ERR_INVALID_ARG: return "invalid argument";
        case CA_ERR_UNSUPPORTED_N: return "unsupported curve size";
        case CA_ERR_HIP: return "HIP runtime error";
        case CA_ERR_OOM: return "out of device memory";
        case CA_ERR_NO_DEVICE: return "no gfx950 device";
        case CA_ERR_INTERNAL: return "internal error";
        case CA_ERR_TOO_LARGE: return "input exceeds the static scratch";
        default: return "unknown status";
    }
}

const char* ca_last_error(void) { return g_err.c_str(); }

int32_t ca_n_supported(int32_t n) {
    if (smooth7(n)) return 1;
    return (n >= 2 && n <= CA_MAX_N) ? 2 : 0;
}

ca_status_t ca_create(ca_context_t* ctx, int device, const char* tune_cache_path) {
    if (!ctx) return fail(CA_ERR_INVALID_ARG, "ctx is NULL");
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(CA_ERR_NO_DEVICE, "no HIP device visible");
    if (device < 0 || device >= count) return fail(CA_ERR_NO_DEVICE, "device index out of range");
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CA_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", gfx950 required");
    ca_context* c = new ca_context();
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->arch = prop.gcnArchName;
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);
    DeviceGuard g(device);
    ca_status_t st = ensure_tables(c, false);
    // team tables and the scratch address now, so that the allocation-free
    // entry point never needs to allocate or look anything up
    if (st == CA_OK) st = ensure_team_tables(c);
    if (st == CA_OK) st = noalloc_scratch_ptr(device, &c->noalloc_scratch);
    if (st == CA_OK && tune_cache_path) st = ca_tune_load(c, tune_cache_path, nullptr);
    if (st != CA_OK) {
        const std::string msg = g_err;
        ca_destroy(c);
        g_err = msg;
        return st;
    }
    *ctx = c;
    return CA_OK;
}

ca_status_t ca_destroy(ca_context_t c) {
    if (!c) return CA_OK;
    {
        DeviceGuard g(c->device);
        if (c->capturing) {
            hipGraph_t gr = nullptr;
            if (hipStreamEndCapture(c->cap_stream, &gr) == hipSuccess && gr) (void)hipGraphDestroy(gr);
            if (g_capturing == c) g_capturing = nullptr;
        }
        (void)hipDeviceSynchronize();
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->d_plans) (void)hipFree(c->d_plans);
        if (c->d_tw32) (void)hipFree(c->d_tw32);
        if (c->d_tw64) (void)hipFree(c->d_tw64);
        for (void* p : c->d_team_tw)
            if (p) (void)hipFree(p);
        if (c->d_bf16) (void)hipFree(c->d_bf16);
        if (c->d_bf16_1k) (void)hipFree(c->d_bf16_1k);
        if (c->d_rs) (void)hipFree(c->d_rs);
        if (c->d_slow) (void)hipFree(c->d_slow);
        if (c->d_bins) (void)hipFree(c->d_bins);
        if (c->d_spec) (void)hipFree(c->d_spec);
        if (c->d_norms) (void)hipFree(c->d_norms);
        for (void* p : c->retired) (void)hipFree(p);
    }
    delete c;
    return CA_OK;
}

ca_status_t ca_graph_begin(ca_context_t c, void** capture_stream) {
    if (!c || !capture_stream) return fail(CA_ERR_INVALID_ARG, "context and capture_stream must be non-NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->capturing) return fail(CA_ERR_INVALID_ARG, "a capture is already open on this context");
    DeviceGuard g(c->device);
    hipError_t e;
    if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "capture stream");
    if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    c->capturing = true;
    c->capture_failed = false;
    g_capturing = c;
    *capture_stream = (void*)c->cap_stream;
    return CA_OK;
}

ca_status_t ca_graph_end(ca_context_t c, ca_graph_t* graph) {
    if (!c || !graph) return fail(CA_ERR_INVALID_ARG, "context and graph must be non-NULL");
    *graph = nullptr;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->capturing) return fail(CA_ERR_INVALID_ARG, "no capture is open on this context");
    DeviceGuard g(c->device);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
    c->capturing = false;
    if (g_capturing == c) g_capturing = nullptr;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    if (c->capture_failed) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(CA_ERR_INVALID_ARG, "a call failed during the capture; the capture was discarded");
    }
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, gr, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return hip_fail(e, "hipGraphInstantiate");
    }
    ca_graph* h = new ca_graph();
    h->device = c->device;
    h->graph = gr;
    h->exec = x;
    *graph = h;
    return CA_OK;
}

ca_status_t ca_graph_launch(ca_graph_t h, void* stream) {
    if (!h) return fail(CA_ERR_INVALID_ARG, "graph is NULL");
    DeviceGuard g(h->device);
    const hipError_t e = hipGraphLaunch(h->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return CA_OK;
}

ca_status_t ca_graph_destroy(ca_graph_t h) {
    if (!h) return CA_OK;
    {
        DeviceGuard g(h->device);
        if (h->exec) (void)hipGraphExecDestroy(h->exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
    }
    delete h;
    return CA_OK;
}

ca_status_t align_batch(ca_context_t c, const void* z1, const void* z2, const int64_t* offsets,
                        int32_t n, int64_t num_pairs, ca_result_t* out, const ca_options_t* opt,
                        void* stream) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (num_pairs < 0) return fail(CA_ERR_INVALID_ARG, "num_pairs < 0");
    ca_options_t o;
    ca_status_t st = parse_opts(opt, o);
    if (st != CA_OK) return st;
    if (num_pairs == 0) return CA_OK;
    if (!z1 || !z2 || !out) return fail(CA_ERR_INVALID_ARG, "z1, z2 and out must be non-NULL");
    if (num_pairs > 0x7fffffffLL) return fail(CA_ERR_INVALID_ARG, "num_pairs exceeds 2^31 - 1");
    if (!offsets && (n < 2 || n > CA_MAX_N)) return fail(CA_ERR_UNSUPPORTED_N, "n must be in [2, 4096]");
    if (!offsets && o.precision == CA_PREC_FP64 && transform_size(n) > kFp64MaxM)
        return fail(CA_ERR_UNSUPPORTED_N, "FP64 precision takes n with prime factors above 7 only up to 2048");
    if (o.precision == CA_PREC_SPLIT_BF16 && (offsets || (n != 128 && n != 1024)))
        return fail(CA_ERR_UNSUPPORTED_N, "split-BF16 precision needs a uniform batch with n = 128 or 1024");
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    st = ensure_tables(c, o.precision == CA_PREC_FP64);
    if (st != CA_OK) return st;
    hipError_t e;
    if (o.precision == CA_PREC_SPLIT_BF16 && n == 1024) {
        st = ensure_bf16_1k_tables(c);
        if (st != CA_OK) return st;
        e = ca::launch_align_bf16_1k(z1, z2, num_pairs, out, c->d_bf16_1k, o.theta_fp64, c->num_cus, s);
    } else if (o.precision == CA_PREC_SPLIT_BF16) {
        st = ensure_bf16_tables(c);
        if (st != CA_OK) return st;
        e = ca::launch_align_bf16(z1, z2, num_pairs, out, c->d_bf16, o.theta_fp64, c->num_cus, s);
    } else if (o.precision == CA_PREC_FP32 && !offsets && ca::team_supported(n)) {
        st = ensure_team_tables(c);
        if (st != CA_OK) return st;
        e = ca::launch_align_team(z1, z2, n, num_pairs, out, team_tw_for(c, n), o.rescore, o.theta_fp64,
                                  c->num_cus, c->tune.team_grid[team_key(n)], s);
    } else {
        ca::BlkArgs a;
        a.z1 = z1;
        a.z2 = z2;
        a.offsets = offsets;
        a.n_uniform = offsets ? 0 : n;
        a.m_uniform = offsets ? 0 : transform_size(n);
        a.m_cap = o.precision == CA_PREC_FP64 ? kFp64MaxM : kMaxM;
        a.num_pairs = num_pairs;
        a.out = out;
        a.plans = c->d_plans;
        a.rescore = o.rescore;
        a.theta64 = o.theta_fp64;
        a.num_cus = c->num_cus;
        for (int k = 0; k < ca::kBlkClasses; ++k) {
            a.grid_mult[k] = c->tune.blk_grid[k];
            a.threads[k] = c->tune.blk_threads[k];
        }
        a.bins = nullptr;
        if (offsets) {
            st = grow(c, (void**)&c->d_bins, &c->bins_bytes, (size_t)ca::blk_bin_ints(num_pairs) * sizeof(int),
                      "size-class lists");
            if (st != CA_OK) return st;
            a.bins = c->d_bins;
        }
        if (o.precision == CA_PREC_FP64) {
            a.tw_arena = c->d_tw64;
            e = ca::launch_align_blk_f64(a, s);
        } else {
            a.tw_arena = c->d_tw32;
            e = ca::launch_align_blk_f32(a, s);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "align kernel launch");
    return CA_OK;
}

ca_status_t align_pair(ca_context_t c, const void* z1, const void* z2, int32_t n, ca_result_t* out,
                       const ca_options_t* opt, void* stream) {
    return align_batch(c, z1, z2, nullptr, n, 1, out, opt, stream);
}

}  // extern "C"

namespace {

// Host validation shared by both all-pairs entry points (nothing is touched
// on the context before it passes).
ca_status_t check_all_pairs(ca_context_t c, const void* curves, int32_t m, int32_t n,
                            const ca_result_t* out_upper, const ca_options_t* opt, ca_options_t& o,
                            bool& nothing) {
    nothing = false;
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    ca_status_t st = parse_opts(opt, o);
    if (st != CA_OK) return st;
    if (m < 0) return fail(CA_ERR_INVALID_ARG, "m < 0");
    if (m < 2) {
        nothing = true;
        return CA_OK;
    }
    if (!curves || !out_upper) return fail(CA_ERR_INVALID_ARG, "curves and out_upper must be non-NULL");
    if (o.precision != CA_PREC_FP32) return fail(CA_ERR_INVALID_ARG, "align_all_pairs is FP32 only");
    if (!ca::allpairs_supported(n))
        return fail(CA_ERR_UNSUPPORTED_N, "align_all_pairs supports n in {64, 128, 256, 512, 1024}");
    const int64_t npairs = (int64_t)m * (m - 1) / 2;
    if (npairs > 0x7fffffffLL) return fail(CA_ERR_INVALID_ARG, "m*(m-1)/2 exceeds 2^31 - 1");
    return CA_OK;
}

// Spectra and norms into (spec, norms), then the upper-triangle tiles.
ca_status_t run_all_pairs(ca_context_t c, const void* curves, int32_t m, int32_t n, ca_result_t* out_upper,
                          const ca_options_t& o, void* spec, double* norms, hipStream_t s) {
    hipError_t e = ca::launch_spectra(curves, m, n, spec, norms, team_tw_for(c, n), s);
    if (e != hipSuccess) return hip_fail(e, "spectra kernel launch");
    e = ca::launch_allpairs(curves, spec, norms, m, n, out_upper, team_tw_for(c, n), o.rescore, o.theta_fp64,
                            c->tune.allpairs_cols[team_key(n)], c->num_cus, s);
    if (e != hipSuccess) return hip_fail(e, "all-pairs kernel launch");
    return CA_OK;
}

}  // namespace

extern "C" {

ca_status_t align_all_pairs(ca_context_t c, const void* curves, int32_t m, int32_t n,
                            ca_result_t* out_upper, const ca_options_t* opt, void* stream) {
    ca_options_t o;
    bool nothing;
    ca_status_t st = check_all_pairs(c, curves, m, n, out_upper, opt, o, nothing);
    if (st != CA_OK || nothing) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    st = ensure_tables(c, false);
    if (st != CA_OK) return st;
    st = ensure_team_tables(c);
    if (st != CA_OK) return st;
    st = grow(c, &c->d_spec, &c->spec_bytes, (size_t)m * n * 2 * sizeof(float), "spectra workspace");
    if (st != CA_OK) return st;
    st = grow(c, (void**)&c->d_norms, &c->norms_bytes, (size_t)m * sizeof(double), "norms workspace");
    if (st != CA_OK) return st;
    return run_all_pairs(c, curves, m, n, out_upper, o, c->d_spec, c->d_norms, (hipStream_t)stream);
}

ca_status_t align_all_pairs_noalloc(ca_context_t c, const void* curves, int32_t m, int32_t n,
                                    ca_result_t* out_upper, const ca_options_t* opt, void* stream) {
    ca_options_t o;
    bool nothing;
    ca_status_t st = check_all_pairs(c, curves, m, n, out_upper, opt, o, nothing);
    if (st != CA_OK || nothing) return st;
    const int64_t need = noalloc_bytes(m, n);
    if (need > (int64_t)CA_NOALLOC_SCRATCH_BYTES)
        return fail(CA_ERR_TOO_LARGE, "align_all_pairs_noalloc: a gallery of " + std::to_string(m) + " x " +
                                          std::to_string(n) + " needs " + std::to_string(need) +
                                          " bytes of scratch, above CA_NOALLOC_SCRATCH_BYTES = " +
                                          std::to_string((long long)CA_NOALLOC_SCRATCH_BYTES));
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    // ca_create built the tables and looked the scratch up; nothing to allocate here
    if (!c->noalloc_scratch || !team_tw_for(c, n))
        return fail(CA_ERR_INTERNAL, "context set-up incomplete (team tables or scratch address missing)");
    unsigned char* base = (unsigned char*)c->noalloc_scratch;
    return run_all_pairs(c, curves, m, n, out_upper, o, base,
                         (double*)(base + noalloc_norms_offset(m, n)), (hipStream_t)stream);
}

ca_status_t resample_arclength(ca_context_t c, const void* raw, const int64_t* raw_offsets,
                               int64_t num_curves, const int64_t* out_offsets, void* out,
                               double* norms_out, uint32_t* flags_out, int32_t mode, void* stream) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (num_curves < 0) return fail(CA_ERR_INVALID_ARG, "num_curves < 0");
    if (mode != CA_RESAMPLE_SPLINE && mode != CA_RESAMPLE_LINEAR)
        return fail(CA_ERR_INVALID_ARG, "mode must be CA_RESAMPLE_SPLINE or CA_RESAMPLE_LINEAR");
    if (num_curves == 0) return CA_OK;
    if (!raw || !raw_offsets || !out_offsets || !out)
        return fail(CA_ERR_INVALID_ARG, "raw, raw_offsets, out_offsets and out must be non-NULL");
    if (num_curves > 0x7fffffffLL) return fail(CA_ERR_INVALID_ARG, "num_curves exceeds 2^31 - 1");
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!c->d_rs) {
        const int64_t slots = 2 * (int64_t)c->num_cus;
        if (hipMalloc(&c->d_rs, (size_t)(slots * ca::resample_slot_bytes())) != hipSuccess)
            return fail(CA_ERR_OOM, "resampler scratch");
        c->rs_slots = slots;
    }
    ca_status_t st = grow(c, (void**)&c->d_slow, &c->slow_bytes, (size_t)(num_curves + 1) * sizeof(int),
                          "resampler curve list");
    if (st != CA_OK) return st;
    hipError_t e = ca::launch_resample(raw, raw_offsets, num_curves, out_offsets, out, norms_out,
                                       flags_out, mode, c->d_rs, ca::resample_slot_bytes(),
                                       c->rs_slots, c->d_slow, c->d_slow + 1, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "resample kernel launch");
    return CA_OK;
}

ca_status_t to_initializer(ca_context_t c, const ca_result_t* results, int32_t n, const int64_t* offsets,
                           int64_t count, double* t0_out, double* rot_out, void* stream) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (count < 0) return fail(CA_ERR_INVALID_ARG, "count < 0");
    if (!offsets && n < 1) return fail(CA_ERR_INVALID_ARG, "n must be >= 1 without offsets");
    if (offsets && n != 0) return fail(CA_ERR_INVALID_ARG, "n must be 0 when offsets are given");
    if (count == 0) return CA_OK;
    if (!results || !t0_out || !rot_out)
        return fail(CA_ERR_INVALID_ARG, "results, t0_out and rot_out must be non-NULL");
    DeviceGuard g(c->device);
    const hipError_t e =
        ca::launch_initializer(results, n, offsets, count, t0_out, rot_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "initializer kernel launch");
    return CA_OK;
}

ca_status_t srv_transform(ca_context_t c, const void* curves, const int64_t* offsets, int32_t n,
                          int64_t count, void* q_out, void* stream) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (count < 0) return fail(CA_ERR_INVALID_ARG, "count < 0");
    if (!offsets && n < 2) return fail(CA_ERR_INVALID_ARG, "n must be >= 2 without offsets");
    if (offsets && n != 0) return fail(CA_ERR_INVALID_ARG, "n must be 0 when offsets are given");
    if (count == 0) return CA_OK;
    if (!curves || !q_out) return fail(CA_ERR_INVALID_ARG, "curves and q_out must be non-NULL");
    DeviceGuard g(c->device);
    const hipError_t e = ca::launch_srv(curves, offsets, n, count, q_out, c->num_cus, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "SRV kernel launch");
    return CA_OK;
}

}  // extern "C"

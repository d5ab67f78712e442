// context.hip -- parameter validation, precomputed tables, scratch memory,
// limb transforms and coefficient-domain import/export.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "fhe_internal.h"

typedef unsigned __int128 u128;

namespace {
thread_local std::string g_err;

uint64_t hmul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t hpow(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    for (; e; e >>= 1, a = hmul(a, a, m))
        if (e & 1) r = hmul(r, a, m);
    return r;
}
uint64_t hinv(uint64_t a, uint64_t m) { return hpow(a % m, m - 2, m); }

bool miller_rabin(uint64_t n)
{
    if (n < 2) return false;
    static const uint64_t w[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : w)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (uint64_t a : w) {
        uint64_t x = hpow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int i = 1; i < s && composite; ++i) {
            x = hmul(x, x, n);
            if (x == n - 1) composite = false;
        }
        if (composite) return false;
    }
    return true;
}

// Any element of order exactly 2N (N a power of two): w = g^((q-1)/2N) with w^N = -1.
uint64_t root_2n(uint64_t q, uint32_t N)
{
    for (uint64_t g = 2; g < 1000000; ++g) {
        uint64_t w = hpow(g, (q - 1) / (2ull * N), q);
        if (hpow(w, N, q) == q - 1) return w;
    }
    return 0;
}
uint32_t brv(uint32_t x, uint32_t bits)
{
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; ++i, x >>= 1) r = (r << 1) | (x & 1);
    return r;
}
template <typename T>
fhe_status dev_alloc(fhe_ctx *c, T **p, size_t count)
{
    size_t bytes = count * sizeof(T);
    if (c->used + bytes > c->budget) return fhe_fail(FHE_ENOMEM, "context tables exceed the HBM budget");
    HIPCHK(hipMalloc((void **)p, bytes ? bytes : 8));
    c->used += bytes;
    return FHE_OK;
}
template <typename T>
fhe_status upload(fhe_ctx *c, T **p, const std::vector<T> &v)
{
    fhe_status s = dev_alloc(c, p, v.size());
    if (s) return s;
    HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return FHE_OK;
}
}  // namespace

fhe_status fhe_fail(fhe_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}
fhe_status scale_room_error(const char *what)
{
    return fhe_fail(FHE_ESCALE, std::string(what) + ": the output scale leaves fewer than " +
                                    std::to_string(FHE_SCALE_ROOM_BITS) + " bits below Q/2 (lower an input scale)");
}
fhe_status fhe_hip_check(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();   // a refused allocation must not resurface at a later launch check
    return FHE_EDEVICE;
}

extern "C" const char *fhe_last_error(void) { return g_err.c_str(); }

struct Prof {
    std::string cat;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<std::pair<int, std::string>> live;   // recorded (slot, category)
    std::map<std::string, std::pair<double, uint64_t>> acc;
};

int prof_begin(fhe_ctx *c, const char *cat)
{
    Prof *p = c->prof;
    if (!p || (p->cat != "*" && p->cat != cat)) return -1;
    int slot = -1;
    for (size_t i = 0; i < p->pool.size() && slot < 0; ++i) {
        bool used = false;
        for (auto &l : p->live) used |= l.first == (int)i;
        if (!used) slot = (int)i;
    }
    if (slot < 0) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
        p->pool.push_back({a, b});
        slot = (int)p->pool.size() - 1;
    }
    p->live.push_back({slot, cat});
    (void)hipEventRecord(p->pool[slot].first, c->stream);
    return slot;
}
void prof_end(fhe_ctx *c, int slot) { (void)hipEventRecord(c->prof->pool[slot].second, c->stream); }

static void prof_collect(fhe_ctx *c)
{
    Prof *p = c->prof;
    if (!p) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &l : p->live) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->pool[l.first].first, p->pool[l.first].second) == hipSuccess) {
            auto &e = p->acc[l.second];
            e.first += ms;
            e.second += 1;
        }
    }
    p->live.clear();
}

extern "C" fhe_status fhe_profile_enable(fhe_ctx *c, const char *category)
{
    if (c && c->capturing && category) return fhe_fail(FHE_EINVAL, "fhe_profile_enable: context is capturing");
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if (!category) {
        if (c->prof) {
            prof_collect(c);
            for (auto &e : c->prof->pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
            delete c->prof;
            c->prof = nullptr;
        }
        return FHE_OK;
    }
    if (!c->prof) c->prof = new Prof();
    prof_collect(c);
    c->prof->cat = category;
    c->prof->acc.clear();
    return FHE_OK;
}
extern "C" fhe_status fhe_profile_read(fhe_ctx *c, const char *category, double *total_ms, uint64_t *count)
{
    if (!c || !category || !total_ms || !count) return fhe_fail(FHE_EINVAL, "fhe_profile_read: null argument");
    *total_ms = 0.0;
    *count = 0;
    if (!c->prof) return FHE_OK;
    prof_collect(c);
    auto it = c->prof->acc.find(category);
    if (it != c->prof->acc.end()) {
        *total_ms = it->second.first;
        *count = it->second.second;
    }
    return FHE_OK;
}

static void ctx_free_all(fhe_ctx *c)
{
    if (c->prof) (void)fhe_profile_enable(c, nullptr);
    if (c->alloc_fn) {   // the growable buffers came from the caller's allocator
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        if (c->scratch) c->free_fn(c->scratch, c->alloc_user);
        if (c->wksp) c->free_fn(c->wksp, c->alloc_user);
        c->scratch = c->wksp = nullptr;
    }
    void *ptrs[] = {c->d_mod, c->d_tw, c->d_itw, c->d_ninv, c->d_cdt, c->d_cos, c->d_sin, c->d_g5,
                    c->d_bconv, c->d_pinv, c->d_phalf, c->d_pmod, c->d_qlinv, c->scratch, c->wksp, c->tbl_dev, c->d_big};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->tbl_host) (void)hipHostFree(c->tbl_host);
    for (auto &a : c->tbl_live) (void)hipEventDestroy(a.ev);
    for (hipEvent_t e : c->tbl_pool) (void)hipEventDestroy(e);
    c->tbl_live.clear();
    c->tbl_pool.clear();
    delete[] c->modup;
    delete[] c->moddown;
    delete c;
}

// Scratch of fhe_keyswitch_batch_static: one array per GPU, in the code object's
// device globals.  Host code must not use its name as an address (it names a host-side
// stand-in); static_scratch_ptr() resolves this device's address once.
static __device__ __align__(256) uint8_t scratch[FHE_STATIC_SCRATCH_BYTES];

static fhe_status static_scratch_ptr(int device, uint8_t **out)
{
    static std::mutex mu;
    static std::map<int, uint8_t *> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void *ptr = nullptr;   // the caller has made `device` current
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        it = addr.emplace(device, (uint8_t *)ptr).first;
    }
    *out = it->second;
    return FHE_OK;
}

extern "C" fhe_status fhe_ctx_create(const fhe_params *pp, void *hip_stream, uint64_t hbm_budget, fhe_ctx **out)
{
    if (!pp || !out || !pp->q || (pp->n_p && !pp->p) || (pp->n_cdt && !pp->cdt))
        return fhe_fail(FHE_EINVAL, "fhe_ctx_create: null argument");
    *out = nullptr;
    const uint32_t logN = pp->log_n, L = pp->n_q, K = pp->n_p;
    if (logN < 10 || logN > 16) return fhe_fail(FHE_EPARAM, "log_n must be in [10, 16]");
    if (L < 1 || L + K > FHE_MAXMOD || pp->dnum < 1 || pp->dnum > L)
        return fhe_fail(FHE_EPARAM, "need 1 <= n_q, n_q + n_p <= 64, 1 <= dnum <= n_q");
    const uint32_t N = 1u << logN;
    fhe_ctx *c = new fhe_ctx();   // value-initialised: plain fields zero, containers constructed
    c->tune_row_wg = 128;
    c->tune_fuse_row_inner = 1;
    c->tune_ks_nt = 1;

    c->logN = logN; c->N = N; c->L = L; c->K = K; c->dnum = pp->dnum;
    c->alpha = (L + pp->dnum - 1) / pp->dnum;
    c->stream = (hipStream_t)hip_stream;
    c->budget = hbm_budget ? hbm_budget : ~0ull;
    for (uint32_t i = 0; i < L; ++i) c->mod[i] = pp->q[i];
    for (uint32_t j = 0; j < K; ++j) c->mod[L + j] = pp->p[j];
    const uint32_t M = L + K;
    for (uint32_t i = 0; i < M; ++i) {
        uint64_t q = c->mod[i];
        bool bad = q >= (1ull << 50) || q < 3 || (q - 1) % (2ull * N) != 0 || !miller_rabin(q);
        for (uint32_t j = 0; j < i; ++j) bad |= c->mod[j] == q;
        if (bad) {
            delete c;
            return fhe_fail(FHE_EPARAM, "modulus " + std::to_string(i) +
                                            " is not a distinct prime below 2^50 congruent to 1 mod 2N");
        }
    }
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return fhe_fail(FHE_EDEVICE, "no HIP device"); }
    if (fhe_status e = static_scratch_ptr(c->device, &c->static_scr)) {
        delete c;
        return e;
    }

    fhe_status st = FHE_OK;
    // per-modulus constants and twiddles
    std::vector<ModQ> mq(M);
    std::vector<double> tw((size_t)M * N), itw((size_t)M * N), ninv(M), phalf(M);
    uint64_t Pm[FHE_MAXMOD];
    for (uint32_t i = 0; i < M; ++i) {
        uint64_t q = c->mod[i];
        mq[i].q = (double)q;
        mq[i].qinv = 1.0 / (double)q;
        uint64_t psi = root_2n(q, N), ipsi = hinv(psi, q);
        std::vector<uint64_t> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (uint32_t e = 1; e < N; ++e) {
            pw[e] = hmul(pw[e - 1], psi, q);
            ipw[e] = hmul(ipw[e - 1], ipsi, q);
        }
        for (uint32_t k = 0; k < N; ++k) {
            uint32_t e = brv(k, logN);
            tw[(size_t)i * N + k] = (double)pw[e];
            itw[(size_t)i * N + k] = (double)ipw[e];
        }
        ninv[i] = (double)hinv(N % q, q);
        uint64_t pm = 1;
        for (uint32_t j = 0; j < K; ++j) pm = hmul(pm, c->mod[L + j] % q, q);
        Pm[i] = pm;
        phalf[i] = (double)hmul((pm + q - 1) % q, hinv(2, q), q);    // (P-1)/2 mod q
    }
    std::vector<double> pinv(L), pmod(L), qlinv((size_t)L * L, 0.0);
    for (uint32_t i = 0; i < L; ++i) {
        pinv[i] = (double)hinv(Pm[i], c->mod[i]);
        pmod[i] = (double)Pm[i];
    }
    for (uint32_t l = 1; l < L; ++l)            // dropping limb l
        for (uint32_t i = 0; i < l; ++i) qlinv[(size_t)l * L + i] = (double)hinv(c->mod[l] % c->mod[i], c->mod[i]);

    // basis conversion tables
    std::vector<double> bc;
    auto make_bconv = [&](BconvTab &t, const std::vector<uint32_t> &src, const std::vector<uint32_t> &dst) {
        t.nsrc = (uint32_t)src.size();
        t.ndst = (uint32_t)dst.size();
        t.off = (uint32_t)bc.size();
        for (uint32_t a = 0; a < t.nsrc; ++a) t.src[a] = (uint8_t)src[a];
        for (uint32_t a = 0; a < t.ndst; ++a) t.dst[a] = (uint8_t)dst[a];
        for (uint32_t a = 0; a < t.nsrc; ++a) {
            uint64_t bi = c->mod[src[a]], h = 1;
            for (uint32_t o = 0; o < t.nsrc; ++o)
                if (o != a) h = hmul(h, c->mod[src[o]] % bi, bi);
            bc.push_back((double)hinv(h, bi));
        }
        for (uint32_t a = 0; a < t.nsrc; ++a) bc.push_back((double)c->mod[src[a]]);
        for (uint32_t a = 0; a < t.nsrc; ++a) bc.push_back(1.0 / (double)c->mod[src[a]]);
        for (uint32_t d = 0; d < t.ndst; ++d) bc.push_back((double)c->mod[dst[d]]);
        for (uint32_t d = 0; d < t.ndst; ++d) bc.push_back(1.0 / (double)c->mod[dst[d]]);
        for (uint32_t d = 0; d < t.ndst; ++d)
            for (uint32_t a = 0; a < t.nsrc; ++a) {
                uint64_t cm = c->mod[dst[d]], h = 1;
                for (uint32_t o = 0; o < t.nsrc; ++o)
                    if (o != a) h = hmul(h, c->mod[src[o]] % cm, cm);
                bc.push_back((double)h);
            }
    };
    c->modup = new BconvTab[(size_t)(L + 1) * c->dnum];
    c->moddown = new BconvTab[L + 1];
    std::memset((void *)c->modup, 0, sizeof(BconvTab) * (L + 1) * c->dnum);
    std::memset((void *)c->moddown, 0, sizeof(BconvTab) * (L + 1));
    for (uint32_t l = 1; l <= L; ++l) {
        uint32_t nd = (l + c->alpha - 1) / c->alpha;
        for (uint32_t j = 0; j < nd; ++j) {
            uint32_t lo = j * c->alpha, hi = std::min(lo + c->alpha, l);
            std::vector<uint32_t> src, dst;
            for (uint32_t i = lo; i < hi; ++i) src.push_back(i);
            for (uint32_t i = 0; i < l; ++i)
                if (i < lo || i >= hi) dst.push_back(i);
            for (uint32_t k = 0; k < K; ++k) dst.push_back(L + k);
            make_bconv(c->modup[(size_t)l * c->dnum + j], src, dst);
        }
        if (K) {
            std::vector<uint32_t> src, dst;
            for (uint32_t k = 0; k < K; ++k) src.push_back(L + k);
            for (uint32_t i = 0; i < l; ++i) dst.push_back(i);
            make_bconv(c->moddown[l], src, dst);
        }
    }
    // encoding tables
    std::vector<double> cs(2 * N), sn(2 * N);
    for (uint32_t e = 0; e < 2 * N; ++e) {
        double ang = M_PI * (double)e / (double)N;
        cs[e] = std::cos(ang);
        sn[e] = std::sin(ang);
    }
    std::vector<uint32_t> g5(N / 2);
    {
        uint64_t g = 1;
        for (uint32_t j = 0; j < N / 2; ++j) { g5[j] = (uint32_t)g; g = g * 5 % (2ull * N); }
    }
    std::vector<uint64_t> cdt(pp->cdt, pp->cdt + pp->n_cdt);
    c->ncdt = pp->n_cdt;

    if ((st = upload(c, &c->d_mod, mq)) || (st = upload(c, &c->d_tw, tw)) || (st = upload(c, &c->d_itw, itw)) ||
        (st = upload(c, &c->d_ninv, ninv)) || (st = upload(c, &c->d_phalf, phalf)) ||
        (st = upload(c, &c->d_pinv, pinv)) || (st = upload(c, &c->d_pmod, pmod)) ||
        (st = upload(c, &c->d_qlinv, qlinv)) || (st = upload(c, &c->d_bconv, bc)) ||
        (st = upload(c, &c->d_cos, cs)) || (st = upload(c, &c->d_sin, sn)) || (st = upload(c, &c->d_g5, g5)) ||
        (st = upload(c, &c->d_cdt, cdt.empty() ? std::vector<uint64_t>{0} : cdt))) {
        ctx_free_all(c);
        return st;
    }
    // the pointer-table ring and a few of its events are made here, so that calls that
    // may not allocate (fhe_keyswitch_batch_static) find them
    if (hipMalloc((void **)&c->tbl_dev, TBL_ARENA_BYTES) != hipSuccess ||
        hipHostMalloc((void **)&c->tbl_host, TBL_ARENA_BYTES) != hipSuccess) {
        (void)hipGetLastError();
        ctx_free_all(c);
        return fhe_fail(FHE_EDEVICE, "fhe_ctx_create: pointer-table ring allocation failed");
    }
    for (int i = 0; i < 8; ++i) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ctx_free_all(c);
            return fhe_fail(FHE_EDEVICE, "fhe_ctx_create: event creation failed");
        }
        c->tbl_pool.push_back(ev);
    }
    *out = c;
    return FHE_OK;
}

extern "C" void fhe_ctx_destroy(fhe_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    ctx_free_all(c);
}
extern "C" fhe_status fhe_ctx_set_tuning(fhe_ctx *c, const char *key, uint64_t value)
{
    if (!c || !key) return fhe_fail(FHE_EINVAL, "fhe_ctx_set_tuning: null argument");
    if (!std::strcmp(key, "chunk_items")) {
        c->tune_chunk = (uint32_t)std::min<uint64_t>(value, 1u << 30);
        return FHE_OK;
    }
    if (!std::strcmp(key, "ks_fuse_row_inner")) {
        c->tune_fuse_row_inner = value ? 1u : 0u;
        return FHE_OK;
    }
    if (!std::strcmp(key, "ks_nt")) {
        c->tune_ks_nt = value ? 1u : 0u;
        return FHE_OK;
    }
    if (!std::strcmp(key, "row_wg")) {
        if (value != 128 && value != 256) return fhe_fail(FHE_EINVAL, "fhe_ctx_set_tuning: row_wg must be 128 or 256");
        c->tune_row_wg = (uint32_t)value;
        return FHE_OK;
    }
    return fhe_fail(FHE_EINVAL, std::string("fhe_ctx_set_tuning: unknown key ") + key);
}
extern "C" fhe_status fhe_set_stream(fhe_ctx *c, void *s)
{
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if (c->capturing) return fhe_fail(FHE_EINVAL, "fhe_set_stream: context is capturing");
    c->stream = (hipStream_t)s;
    return FHE_OK;
}
extern "C" uint32_t fhe_ring_degree(const fhe_ctx *c) { return c ? c->N : 0; }
extern "C" uint64_t fhe_modulus(const fhe_ctx *c, uint32_t i) { return (c && i < c->L + c->K) ? c->mod[i] : 0; }
extern "C" size_t fhe_evk_bytes(const fhe_ctx *c)
{
    return c ? (size_t)c->dnum * 2 * (c->L + c->K) * c->N * sizeof(uint64_t) : 0;
}
extern "C" size_t fhe_ct_bytes(const fhe_ctx *c, uint32_t limbs, uint32_t polys)
{
    return c ? (size_t)polys * limbs * c->N * sizeof(uint64_t) : 0;
}
extern "C" uint64_t fhe_galois_elt(const fhe_ctx *c, int32_t step)
{
    if (!c) return 0;
    int64_t n = c->N / 2, r = ((int64_t)step % n + n) % n;
    uint64_t g = 1, m = 2ull * c->N, b = 5;
    for (; r; r >>= 1, b = b * b % m)
        if (r & 1) g = g * b % m;
    return g;
}
extern "C" uint64_t fhe_scratch_bytes(const fhe_ctx *c) { return c ? c->scratch_bytes : 0; }

// Device memory of the context's growable buffers: from the caller's allocator when
// one is set (fhe_ctx_set_allocator), else hipMalloc.
static fhe_status ctx_dev_alloc(fhe_ctx *c, size_t bytes, uint8_t **p)
{
    if (c->alloc_fn) {
        *p = (uint8_t *)c->alloc_fn(bytes, (void *)c->stream, c->alloc_user);
        if (!*p) return fhe_fail(FHE_ENOMEM, "the caller's allocator refused " + std::to_string(bytes) + " bytes");
        return FHE_OK;
    }
    HIPCHK(hipMalloc((void **)p, bytes));
    return FHE_OK;
}
static fhe_status ctx_dev_free(fhe_ctx *c, uint8_t *p)
{
    if (!p) return FHE_OK;
    if (c->alloc_fn) {
        c->free_fn(p, c->alloc_user);
        return FHE_OK;
    }
    HIPCHK(hipFree(p));
    return FHE_OK;
}
// Grow one of the buffers to `bytes` (its contents are not kept).
static fhe_status ctx_grow(fhe_ctx *c, uint8_t **buf, size_t *held, size_t bytes, const char *what)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes <= *held) return FHE_OK;
    if (c->no_alloc) return fhe_fail(FHE_ENOMEM, std::string(what) + " growth in a call that may not allocate");
    if (c->capturing) {
        c->cap_error = FHE_ENOMEM;
        return fhe_fail(FHE_ENOMEM, "graph capture: device memory must be sized by an eager run first");
    }
    if (c->used + (bytes - *held) > c->budget) return fhe_fail(FHE_ENOMEM, std::string(what) + " exceeds the HBM budget");
    HIPCHK(hipStreamSynchronize(c->stream));
    fhe_status s = ctx_dev_free(c, *buf);
    *buf = nullptr;
    c->used -= *held;
    *held = 0;
    if (s) return s;
    if ((s = ctx_dev_alloc(c, bytes, buf))) return s;
    *held = bytes;
    c->used += bytes;
    return FHE_OK;
}

fhe_status ctx_scratch(fhe_ctx *c, size_t bytes, uint8_t **out)
{
    fhe_status s = ctx_grow(c, &c->scratch, &c->scratch_bytes, bytes, "scratch");
    if (s) return s;
    *out = c->scratch;
    return FHE_OK;
}

// Same growth rule for the layer workspace (a separate buffer, so that a layer's
// intermediates survive the scratch use of the operations it calls).
fhe_status ctx_workspace(fhe_ctx *c, size_t bytes, uint8_t **out)
{
    fhe_status s = ctx_grow(c, &c->wksp, &c->wksp_bytes, bytes, "layer workspace");
    if (s) return s;
    *out = c->wksp;
    return FHE_OK;
}

extern "C" fhe_status fhe_ctx_set_allocator(fhe_ctx *c, fhe_alloc_fn alloc_fn, fhe_free_fn free_fn, void *user)
{
    if (!c || (!alloc_fn) != (!free_fn)) return fhe_fail(FHE_EINVAL, "fhe_ctx_set_allocator: need both functions or none");
    if (c->capturing) return fhe_fail(FHE_EINVAL, "fhe_ctx_set_allocator: context is capturing");
    // release what the previous allocator gave
    HIPCHK(hipStreamSynchronize(c->stream));
    fhe_status s = ctx_dev_free(c, c->scratch);
    if (!s) s = ctx_dev_free(c, c->wksp);
    c->used -= c->scratch_bytes + c->wksp_bytes;
    c->scratch = c->wksp = nullptr;
    c->scratch_bytes = c->wksp_bytes = 0;
    c->alloc_fn = alloc_fn;
    c->free_fn = free_fn;
    c->alloc_user = user;
    return s;
}
extern "C" uint64_t fhe_workspace_bytes(const fhe_ctx *c) { return c ? c->wksp_bytes : 0; }
extern "C" fhe_status fhe_ctx_release_buffers(fhe_ctx *c)
{
    if (!c) return fhe_fail(FHE_EINVAL, "null context");
    if (c->capturing) return fhe_fail(FHE_EINVAL, "fhe_ctx_release_buffers: context is capturing");
    HIPCHK(hipStreamSynchronize(c->stream));
    fhe_status s = ctx_dev_free(c, c->scratch);
    if (!s) s = ctx_dev_free(c, c->wksp);
    c->used -= c->scratch_bytes + c->wksp_bytes;
    c->scratch = c->wksp = nullptr;
    c->scratch_bytes = c->wksp_bytes = 0;
    return s;
}

// Upload a list of device pointers for the next launch(es) on the context's
// stream.  Tables live in a ring over a device arena (copied from its pinned
// twin on the stream); a table's region is reused only after the work enqueued
// before the following table request has completed, so the host runs up to a
// whole arena of tables ahead of the device.
fhe_status ctx_ptr_table(fhe_ctx *c, const std::vector<uint64_t *> &ptrs, uint64_t ***dev)
{
    const size_t n = ptrs.size() ? ptrs.size() : 1;
    if (c->capturing) {
        // the graph replays these launches later: keep the table in the capture arena
        const size_t off = (c->cap_used + 255) & ~(size_t)255, bytes = n * sizeof(uint64_t *);
        if (off + bytes > c->cap_bytes) {
            c->cap_error = FHE_ENOMEM;
            return fhe_fail(FHE_ENOMEM, "graph capture: pointer-table arena is full");
        }
        std::memcpy(c->cap_host + off, ptrs.data(), ptrs.size() * sizeof(uint64_t *));
        c->cap_used = off + bytes;
        *dev = (uint64_t **)(c->cap_dev + off);
        return FHE_OK;
    }
    const size_t bytes = (n * sizeof(uint64_t *) + 255) & ~(size_t)255;
    if (bytes > TBL_ARENA_BYTES) {
        if (c->no_alloc) return fhe_fail(FHE_ENOMEM, "pointer table larger than the context's table ring");
        HIPCHK(hipStreamSynchronize(c->stream));
        if (n > c->d_big_cap) {
            if (c->d_big) HIPCHK(hipFree(c->d_big));
            c->d_big = nullptr;
            HIPCHK(hipMalloc((void **)&c->d_big, n * sizeof(uint64_t *)));
            c->d_big_cap = n;
        }
        HIPCHK(hipMemcpy(c->d_big, ptrs.data(), ptrs.size() * sizeof(uint64_t *), hipMemcpyHostToDevice));
        *dev = c->d_big;
        return FHE_OK;
    }
    if (!c->tbl_dev) {
        if (c->no_alloc) return fhe_fail(FHE_ENOMEM, "pointer-table ring missing in a call that may not allocate");
        HIPCHK(hipMalloc((void **)&c->tbl_dev, TBL_ARENA_BYTES));
        HIPCHK(hipHostMalloc((void **)&c->tbl_host, TBL_ARENA_BYTES));
    }
    // every launch that reads the previous table has been enqueued: mark its release
    if (!c->tbl_live.empty() && !c->tbl_live.back().recorded) {
        HIPCHK(hipEventRecord(c->tbl_live.back().ev, c->stream));
        c->tbl_live.back().recorded = true;
    }
    size_t off = 0;
    for (;;) {
        if (c->tbl_live.empty()) {
            off = 0;
            break;
        }
        const size_t tail = c->tbl_live.front().off;
        const size_t head = c->tbl_live.back().off + c->tbl_live.back().len;
        const bool wrapped = c->tbl_live.back().off < tail;
        if (!wrapped && head + bytes <= TBL_ARENA_BYTES) {
            off = head;
            break;
        }
        if (!wrapped && bytes <= tail) {
            off = 0;
            break;
        }
        if (wrapped && head + bytes <= tail) {
            off = head;
            break;
        }
        // retire the oldest table (waits for the work enqueued up to its release point)
        fhe_ctx::TblAlloc a = c->tbl_live.front();
        HIPCHK(hipEventSynchronize(a.ev));
        c->tbl_pool.push_back(a.ev);
        c->tbl_live.pop_front();
    }
    hipEvent_t ev;
    if (!c->tbl_pool.empty()) {
        ev = c->tbl_pool.back();
        c->tbl_pool.pop_back();
    } else if (c->no_alloc && !c->tbl_live.empty()) {
        // no new event in a call that may not allocate: retire the oldest table
        // (its release point is the oldest in the stream) and take over its event
        fhe_ctx::TblAlloc a = c->tbl_live.front();
        HIPCHK(hipEventSynchronize(a.ev));
        c->tbl_live.pop_front();
        ev = a.ev;
    } else {
        if (c->no_alloc) return fhe_fail(FHE_ENOMEM, "pointer-table events exhausted in a call that may not allocate");
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    std::memcpy(c->tbl_host + off, ptrs.data(), ptrs.size() * sizeof(uint64_t *));
    HIPCHK(hipMemcpyAsync(c->tbl_dev + off, c->tbl_host + off, ptrs.size() * sizeof(uint64_t *),
                          hipMemcpyHostToDevice, c->stream));
    c->tbl_live.push_back(fhe_ctx::TblAlloc{off, bytes, ev, false});
    *dev = (uint64_t **)(c->tbl_dev + off);
    return FHE_OK;
}

LimbSet limbset_list(uint64_t *base, const uint32_t *mods, uint32_t period)
{
    LimbSet ls;
    std::memset((void *)&ls, 0, sizeof(ls));
    ls.base = base;
    ls.period = period;
    for (uint32_t i = 0; i < period && i < FHE_LIMBTAB; ++i) ls.mod[i] = (uint8_t)mods[i];
    return ls;
}
// count limbs with moduli first_mod .. first_mod+period_mods-1, repeating
LimbSet limbset_range(uint64_t *base, uint32_t first_mod, uint32_t count, uint32_t period_mods)
{
    (void)count;
    uint32_t m[FHE_LIMBTAB];
    for (uint32_t i = 0; i < period_mods; ++i) m[i] = first_mod + i;
    return limbset_list(base, m, period_mods);
}

static fhe_status check_modlist(fhe_ctx *c, uint32_t nlimbs, const uint32_t *modidx)
{
    if (!modidx) return fhe_fail(FHE_EINVAL, "null modulus list");
    if (nlimbs > FHE_LIMBTAB) return fhe_fail(FHE_EINVAL, "at most 128 limbs per call");
    for (uint32_t i = 0; i < nlimbs; ++i)
        if (modidx[i] >= c->L + c->K) return fhe_fail(FHE_EINVAL, "modulus index out of range");
    return FHE_OK;
}

extern "C" fhe_status fhe_ntt(fhe_ctx *c, uint64_t *d, uint32_t nlimbs, const uint32_t *modidx)
{
    if (!c || !d) return fhe_fail(FHE_EINVAL, "fhe_ntt: null argument");
    fhe_status s = check_modlist(c, nlimbs, modidx);
    if (s) return s;
    launch_ntt_fwd(c, limbset_list(d, modidx, nlimbs), nlimbs);
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
extern "C" fhe_status fhe_intt(fhe_ctx *c, uint64_t *d, uint32_t nlimbs, const uint32_t *modidx)
{
    if (!c || !d) return fhe_fail(FHE_EINVAL, "fhe_intt: null argument");
    fhe_status s = check_modlist(c, nlimbs, modidx);
    if (s) return s;
    launch_ntt_inv(c, limbset_list(d, modidx, nlimbs), nlimbs);
    HIPCHK(hipGetLastError());
    return FHE_OK;
}
extern "C" fhe_status fhe_export_limbs(fhe_ctx *c, const uint64_t *d, uint32_t nlimbs, const uint32_t *modidx,
                                       uint64_t *host_out)
{
    if (!c || !d || !host_out) return fhe_fail(FHE_EINVAL, "fhe_export_limbs: null argument");
    fhe_status s = check_modlist(c, nlimbs, modidx);
    if (s) return s;
    size_t bytes = (size_t)nlimbs * c->N * sizeof(uint64_t);
    uint8_t *tmp;
    if ((s = ctx_scratch(c, bytes, &tmp))) return s;
    HIPCHK(hipMemcpyAsync(tmp, d, bytes, hipMemcpyDeviceToDevice, c->stream));
    launch_ntt_inv(c, limbset_list((uint64_t *)tmp, modidx, nlimbs), nlimbs);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host_out, tmp, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return FHE_OK;
}
extern "C" fhe_status fhe_import_limbs(fhe_ctx *c, const uint64_t *host_in, uint32_t nlimbs, const uint32_t *modidx,
                                       uint64_t *d)
{
    if (!c || !d || !host_in) return fhe_fail(FHE_EINVAL, "fhe_import_limbs: null argument");
    fhe_status s = check_modlist(c, nlimbs, modidx);
    if (s) return s;
    for (uint32_t i = 0; i < nlimbs; ++i)
        for (uint32_t k = 0; k < c->N; ++k)
            if (host_in[(size_t)i * c->N + k] >= c->mod[modidx[i]])
                return fhe_fail(FHE_EINVAL, "import: residue not below its modulus");
    size_t bytes = (size_t)nlimbs * c->N * sizeof(uint64_t);
    HIPCHK(hipMemcpyAsync(d, host_in, bytes, hipMemcpyHostToDevice, c->stream));
    launch_ntt_fwd(c, limbset_list(d, modidx, nlimbs), nlimbs);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return FHE_OK;
}

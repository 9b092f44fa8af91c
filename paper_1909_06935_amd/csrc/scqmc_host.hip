// scqmc_host.hip -- host runtime behind the C ABI of include/scqmc.h.
//
// Owns device memory and the stream, validates every input on the host,
// runs the setup kernels (integral blocks, core folding, reference tables)
// and launches the walker kernels.  Finalisation of the sampled sums
// (energy, jackknife error, a0^2, Davidson correction, E^(2)) is host FP64
// on a handful of numbers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <chrono>
#include <mutex>

#include "../../include/scqmc.h"
#include "scqmc_setup.hip"
#include "scqmc_walk.hip"
#include "scqmc_refprops.hip"

namespace {

struct DBuf {
    void *p = nullptr;
    size_t n = 0;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    template <class T> T *as() const { return (T *)p; }
};

struct TableBufs {
    DBuf slots, ents;
    unsigned long long cap = 0, unique = 0;
    DevTable view() const {
        DevTable t;
        t.slots = slots.as<ulonglong2>();
        t.ents = ents.as<ListEnt>();
        t.mask = cap ? cap - 1 : 0;
        return t;
    }
};

struct Status {
    scqmc_status s;
};

}  // namespace

struct scqmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *scratch_ptr = nullptr;   // device address of this device's allocation-free scratch array
    std::string err;
    bool has_space = false, has_ints = false, has_ref = false, has_coef = false, has_dyall = false,
         has_walkers = false;
    int N = 0, C = 0, A = 0, V = 0, Np = 0, words = 0, na = 0, nb = 0, nea = 0, neb = 0;
    long long ncls = 0;
    scqmc_options opt{0.0, 0, 0, 0, 0};
    double e_core = 0.0, e0_ref = 0.0;
    double tau = 0.0;   // small-norm perturber screen of SC-NEVPT2(s): classes with N_l/N_0 < tau dropped
    DBuf heff, eri, ccls, eps, refcoef, refkey;
    DBuf wftab;   // [W][2][A][V] Fock tables of the walker kernel (scratch of each step)
    DBuf sftab;   // Fock tables of the snapshot kernel's wave slots
    DBuf heff32, eri32;                  // precision form: FP32 copies
    long long ints_version = 0, f32_version = -1;
    std::vector<double> refcoef_h;
    TableBufs ref, ytab, xtab;
    long long n_ref = 0;
    std::vector<double> ccls_h, eps_h;
    // walkers
    long long W = 0, step = 0;
    long long ncg = 0;   // walker groups with their own class sums (jackknife of E^(2))
    std::vector<double> am_m, am_v, am_vmax;   // AMSGrad moments (classes 1..n_classes-1)
    unsigned long long seed = 0;
    DBuf wkey, wvirt, wpsi, wsum, cacc, bad;
    DBuf worder;   // walker of each workgroup slot of a k_sample launch
    // snapshot scratch
    DBuf skey, svirt, svalid;
};

#define FAIL(ctx, code, msg)          \
    do {                              \
        (ctx)->err = (msg);           \
        return (code);                \
    } while (0)

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                \
            return e_ == hipErrorOutOfMemory ? SCQMC_E_OOM : SCQMC_E_DEVICE;               \
        }                                                                                  \
    } while (0)

static scqmc_status dalloc(scqmc_ctx *ctx, DBuf &b, size_t bytes) {
    b.release();
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        ctx->err = std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e);
        return SCQMC_E_OOM;
    }
    b.n = bytes;
    return SCQMC_OK;
}

#define TRY(x)                           \
    do {                                 \
        scqmc_status s_ = (x);           \
        if (s_ != SCQMC_OK) return s_;   \
    } while (0)

static inline unsigned grid1(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static DevProblem dev_problem(const scqmc_ctx *c) {
    DevProblem P;
    P.A = c->A;
    P.V = c->V;
    P.Np = c->Np;
    P.nea = c->nea;
    P.neb = c->neb;
    P.mode = c->opt.mode;
    P.active_only = 0;
    P.ncls = c->ncls;
    P.e_core = c->e_core;
    P.eps_screen = c->opt.eps_screen;
    P.heff = c->heff.as<double>();
    P.eri = c->eri.as<double>();
    P.heff32 = c->heff32.as<float>();
    P.eri32 = c->eri32.as<float>();
    P.ccls = c->ccls.as<double>();
    P.eps = c->eps.as<double>();
    P.ref = c->ref.view();
    P.ytab = c->ytab.view();
    P.xtab = c->xtab.view();
    P.seed = c->seed;
    return P;
}

static int lists_per_group(const scqmc_ctx *c) { return std::max(1, c->nea + c->neb); }

// bytes of one wave's Fock table, [2][A][V] doubles
static size_t ftab_bytes(const scqmc_ctx *c) { return sizeof(double) * 2 * (size_t)c->A * (size_t)c->V; }

// wave slots of a snapshot launch (grid-stride beyond that)
#define SCQ_EVAL_SLOTS 16384

// Class sums are kept per group of consecutive walkers (group of walker w:
// w * ncg / W), so that E^(2) gets a jackknife error like E_var.
static long long class_groups(long long W) { return std::min<long long>(W, 16); }
static size_t class_acc_bytes(const scqmc_ctx *c) { return (size_t)64 * c->ncg * c->ncls; }

// Host compaction of one full determinant: active key, packed virtual codes.
// Returns false (with a reason) if it is outside the allowed space.
static bool compact_host(const scqmc_ctx *c, const uint64_t *d, unsigned long long &key, unsigned &virt,
                         std::string &why) {
    key = 0;
    int vc[3], nv = 0;
    for (int s = 0; s < 2; s++) {
        int cnt = 0;
        for (int w = 0; w < c->words; w++) {
            uint64_t word = d[s * c->words + w];
            for (int b = 0; b < 64; b++) {
                if (!((word >> b) & 1ull)) continue;
                int p = 64 * w + b;
                if (p >= c->N) { why = "bit beyond n_orb set"; return false; }
                cnt++;
                if (p >= c->C && p < c->C + c->A) key |= 1ull << (32 * s + p - c->C);
                else if (p >= c->C + c->A) { if (nv < 3) vc[nv] = s * c->V + (p - c->C - c->A); nv++; }
            }
        }
        for (int p = 0; p < c->C; p++)
            if (!((d[s * c->words + (p >> 6)] >> (p & 63)) & 1ull)) { why = "core hole"; return false; }
        if (cnt != (s == 0 ? c->na : c->nb)) { why = "wrong electron count"; return false; }
    }
    if (nv > 2) { why = "more than two virtual electrons"; return false; }
    virt = (nv > 0 ? (unsigned)vc[0] : SCQ_NOVIRT) | ((nv > 1 ? (unsigned)vc[1] : SCQ_NOVIRT) << 16);
    return true;
}

static void expand_host(const scqmc_ctx *c, unsigned long long key, unsigned virt, uint64_t *d) {
    std::memset(d, 0, sizeof(uint64_t) * 2 * c->words);
    auto set = [&](int s, int p) { d[s * c->words + (p >> 6)] |= 1ull << (p & 63); };
    for (int s = 0; s < 2; s++) {
        for (int p = 0; p < c->C; p++) set(s, p);
        for (int t = 0; t < c->A; t++)
            if ((key >> (32 * s + t)) & 1ull) set(s, c->C + t);
    }
    for (int i = 0; i < 2; i++) {
        unsigned v = (virt >> (16 * i)) & 0xFFFFu;
        if (v == SCQ_NOVIRT) continue;
        int s = (int)v >= c->V;
        set(s, c->C + c->A + (int)v - s * c->V);
    }
}

static bool all_finite(const double *x, size_t n) {
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(x[i])) return false;
    return true;
}

extern "C" {

// ---------------------------------------------------------------------------
// Fixed device memory of the allocation-free snapshot entry point: the
// compacted copy of up to SCQMC_NOALLOC_MAX_DETS determinants (active key
// u64, virtual codes u32, valid flag i32 = 16 B each), then the per-wave Fock
// tables of the evaluation kernel (SCQMC_NOALLOC_FTAB_BYTES; the launch takes
// as many wave slots as tables fit).  Each GPU holds its own copy of the array
// for the life of the process.  Host code must never pass
// the array's name to a kernel (on the host it is only a stand-in symbol): its
// device address is taken once per device with hipGetSymbolAddress, at context
// creation with that device current, and kept in scratch_dev[].
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[(size_t)SCQMC_NOALLOC_MAX_DETS * 16 + SCQMC_NOALLOC_FTAB_BYTES];
#define SCQ_MAX_DEVICES 64
static std::mutex scratch_mu;
static void *scratch_dev[SCQ_MAX_DEVICES];

// device address of this device's scratch array (device must be current)
static hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= SCQ_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_dev[device] = p;
    }
    *out = scratch_dev[device];
    return hipSuccess;
}

scqmc_status scqmc_create(int device, void *hip_stream, scqmc_ctx **out) {
    if (!out) return SCQMC_E_INVALID_ARG;
    *out = nullptr;
    scqmc_ctx *c = new (std::nothrow) scqmc_ctx();
    if (!c) return SCQMC_E_OOM;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete c;
        return SCQMC_E_DEVICE;
    }
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return SCQMC_E_DEVICE; }
    if (scratch_address(device, &c->scratch_ptr) != hipSuccess) { delete c; return SCQMC_E_DEVICE; }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return SCQMC_E_DEVICE; }
        c->own_stream = true;
    }
    *out = c;
    return SCQMC_OK;
}

void scqmc_destroy(scqmc_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *scqmc_last_error(const scqmc_ctx *c) { return c ? c->err.c_str() : "null context"; }

scqmc_status scqmc_set_space(scqmc_ctx *c, const scqmc_space *s) {
    if (!c || !s) return SCQMC_E_INVALID_ARG;
    if (s->n_orb <= 0 || s->n_core < 0 || s->n_act <= 0 || s->n_core + s->n_act > s->n_orb)
        FAIL(c, SCQMC_E_INVALID_ARG, "bad orbital partition");
    if (s->n_orb > 128 || s->n_act > 32) FAIL(c, SCQMC_E_UNSUPPORTED, "n_orb > 128 or n_act > 32");
    int V = s->n_orb - s->n_core - s->n_act;
    if (2 * V > 65534) FAIL(c, SCQMC_E_UNSUPPORTED, "too many virtual orbitals");
    int nea = s->n_elec_a - s->n_core, neb = s->n_elec_b - s->n_core;
    if (nea < 0 || neb < 0 || nea > s->n_act || neb > s->n_act)
        FAIL(c, SCQMC_E_INVALID_ARG, "electron counts inconsistent with core / active sizes");
    if (nea + neb == 0) FAIL(c, SCQMC_E_INVALID_ARG, "no active electron");
    if (s->n_act == 32 && nea == 32 && neb == 32) FAIL(c, SCQMC_E_UNSUPPORTED, "active space completely filled");
    if (nea + neb > 23) FAIL(c, SCQMC_E_UNSUPPORTED, "more than 23 active electrons");
    c->N = s->n_orb; c->C = s->n_core; c->A = s->n_act; c->V = V; c->Np = s->n_act + V;
    c->words = (s->n_orb + 63) / 64;
    c->na = s->n_elec_a; c->nb = s->n_elec_b; c->nea = nea; c->neb = neb;
    long long V2 = 2LL * V;
    c->ncls = 1 + V2 + V2 * (V2 - 1) / 2;
    c->has_space = true;
    c->has_ints = c->has_ref = c->has_coef = c->has_dyall = c->has_walkers = false;
    c->err.clear();
    return SCQMC_OK;
}

static scqmc_status finish_integrals(scqmc_ctx *c, DBuf &full, DBuf &h1d, double e_const) {
    long long Np4 = (long long)c->Np * c->Np * c->Np * c->Np;
    TRY(dalloc(c, c->eri, sizeof(double) * Np4));
    TRY(dalloc(c, c->heff, sizeof(double) * c->Np * c->Np));
    DBuf ec;
    TRY(dalloc(c, ec, sizeof(double)));
    hipLaunchKernelGGL(k_noncore, dim3(grid1(std::max(Np4, (long long)c->Np * c->Np), 256)), dim3(256), 0, c->stream,
                       full.as<double>(), h1d.as<double>(), c->N, c->C, c->eri.as<double>(), c->heff.as<double>());
    hipLaunchKernelGGL(k_ecore, dim3(1), dim3(1), 0, c->stream, full.as<double>(), h1d.as<double>(), c->N, c->C,
                       e_const, ec.as<double>());
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&c->e_core, ec.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_ints = true;
    c->ints_version++;
    return SCQMC_OK;
}

// FP32 copies of the integrals for the precision form, made on demand and
// again whenever the integrals changed (set_integrals_*, semicanonicalize).
static scqmc_status ensure_f32(scqmc_ctx *c) {
    if (c->opt.precision != 1 || c->f32_version == c->ints_version) return SCQMC_OK;
    long long Np4 = (long long)c->Np * c->Np * c->Np * c->Np, Np2 = (long long)c->Np * c->Np;
    TRY(dalloc(c, c->eri32, sizeof(float) * Np4));
    TRY(dalloc(c, c->heff32, sizeof(float) * Np2));
    hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(256), 0, c->stream, c->eri.as<double>(), c->eri32.as<float>(), Np4);
    hipLaunchKernelGGL(k_to_f32, dim3(grid1(Np2, 256)), dim3(256), 0, c->stream, c->heff.as<double>(),
                       c->heff32.as<float>(), Np2);
    HIPCHK(c, hipGetLastError());
    c->f32_version = c->ints_version;
    return SCQMC_OK;
}

static bool symmetric_copy(const double *a, int n, std::vector<double> &out) {
    out.assign(a, a + (size_t)n * n);
    double mx = 0.0;
    for (int i = 0; i < n * n; i++) mx = std::max(mx, std::fabs(a[i]));
    for (int p = 0; p < n; p++)
        for (int q = p + 1; q < n; q++) {
            double x = a[p * n + q], y = a[q * n + p];
            if (std::fabs(x - y) > 1e-10 * (1.0 + mx)) return false;
            double m = 0.5 * (x + y);
            out[p * n + q] = out[q * n + p] = m;
        }
    return true;
}

scqmc_status scqmc_set_integrals_chol(scqmc_ctx *c, const double *h1, const double *chol, int32_t n_chol,
                                      double e_const) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_space) FAIL(c, SCQMC_E_STATE, "set_space first");
    if (!h1 || (!chol && n_chol > 0) || n_chol < 0) FAIL(c, SCQMC_E_INVALID_ARG, "null integral array");
    int N = c->N;
    long long N2 = (long long)N * N;
    if (!std::isfinite(e_const) || !all_finite(h1, N2) || !all_finite(chol, (size_t)N2 * n_chol))
        FAIL(c, SCQMC_E_NUMERIC, "non-finite integral");
    std::vector<double> hs, Bs((size_t)N2 * std::max(n_chol, 1)), tmp;
    if (!symmetric_copy(h1, N, hs)) FAIL(c, SCQMC_E_INVALID_ARG, "h1 not symmetric");
    for (int l = 0; l < n_chol; l++) {
        if (!symmetric_copy(chol + l * N2, N, tmp)) FAIL(c, SCQMC_E_INVALID_ARG, "Cholesky slice not symmetric");
        std::copy(tmp.begin(), tmp.end(), Bs.begin() + l * N2);
    }
    HIPCHK(c, hipSetDevice(c->device));
    DBuf Bd, h1d, full;
    TRY(dalloc(c, Bd, sizeof(double) * N2 * std::max(n_chol, 1)));
    TRY(dalloc(c, h1d, sizeof(double) * N2));
    TRY(dalloc(c, full, sizeof(double) * N2 * N2));
    HIPCHK(c, hipMemcpyAsync(Bd.p, Bs.data(), sizeof(double) * N2 * n_chol, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(h1d.p, hs.data(), sizeof(double) * N2, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_eri_chol, dim3(grid1(N2 * N2, 256)), dim3(256), 0, c->stream, Bd.as<double>(), n_chol, N2,
                       full.as<double>());
    HIPCHK(c, hipGetLastError());
    TRY(finish_integrals(c, full, h1d, e_const));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SCQMC_OK;
}

scqmc_status scqmc_set_integrals_dense(scqmc_ctx *c, const double *h1, const double *eri, double e_const) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_space) FAIL(c, SCQMC_E_STATE, "set_space first");
    if (!h1 || !eri) FAIL(c, SCQMC_E_INVALID_ARG, "null integral array");
    int N = c->N;
    long long N2 = (long long)N * N;
    if (!std::isfinite(e_const) || !all_finite(h1, N2) || !all_finite(eri, (size_t)N2 * N2))
        FAIL(c, SCQMC_E_NUMERIC, "non-finite integral");
    std::vector<double> hs;
    if (!symmetric_copy(h1, N, hs)) FAIL(c, SCQMC_E_INVALID_ARG, "h1 not symmetric");
    HIPCHK(c, hipSetDevice(c->device));
    DBuf h1d, full;
    TRY(dalloc(c, h1d, sizeof(double) * N2));
    TRY(dalloc(c, full, sizeof(double) * N2 * N2));
    HIPCHK(c, hipMemcpyAsync(h1d.p, hs.data(), sizeof(double) * N2, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(full.p, eri, sizeof(double) * N2 * N2, hipMemcpyHostToDevice, c->stream));
    TRY(finish_integrals(c, full, h1d, e_const));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SCQMC_OK;
}

// Multimap from 64-bit keys to lists of (signed coefficient, code), built on
// the device: expand the reference determinants into (key, payload) pairs,
// count distinct keys in a scratch table, insert into a table of at least 4x
// that many 16-byte slots (load <= 1/4), give every key a contiguous range,
// scatter the payloads, sort each list (deterministic content order).  Mode 0
// (the determinant table) keeps each key's coefficient in its slot and has no
// entry array.
static scqmc_status build_table(scqmc_ctx *c, int mode, const DBuf &rkeys, long long n, TableBufs &t) {
    int ne = c->nea + c->neb;
    long long per = mode == 0 ? 1 : mode == 1 ? ne : (long long)ne * (ne - 1) / 2;
    long long M = n * per;
    // list offsets, counts and entry indices are 32-bit on the device
    if (M >= (1LL << 32))
        FAIL(c, SCQMC_E_UNSUPPORTED, "reference expands to " + std::to_string(M) +
                                         " list entries; the tables hold fewer than 2^32");
    hipStream_t st = c->stream;
    DBuf ekeys, epay, cnt, off, cur, slot_of, tmp, total, scratch, uniq;
    TRY(dalloc(c, ekeys, sizeof(unsigned long long) * M));
    TRY(dalloc(c, epay, sizeof(unsigned long long) * M));
    TRY(dalloc(c, uniq, sizeof(unsigned)));
    unsigned long long cap1 = 64;
    while (cap1 < 2ull * (unsigned long long)std::max(M, 1LL)) cap1 <<= 1;
    TRY(dalloc(c, scratch, sizeof(unsigned long long) * cap1));
    if (M > 0)
        hipLaunchKernelGGL(k_expand, dim3(grid1(n, 128)), dim3(128), 0, st, rkeys.as<unsigned long long>(), n, mode,
                           (int)per, ekeys.as<unsigned long long>(), epay.as<unsigned long long>());
    hipLaunchKernelGGL(k_fill_u64, dim3(grid1(cap1, 256)), dim3(256), 0, st, scratch.as<unsigned long long>(),
                       (long long)cap1, SCQ_EMPTY_KEY);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(32), 0, st, uniq.as<unsigned>(), 1LL, 0u);
    if (M > 0)
        hipLaunchKernelGGL(k_insert, dim3(grid1(M, 256)), dim3(256), 0, st, ekeys.as<unsigned long long>(), M,
                           scratch.as<unsigned long long>(), 1, cap1 - 1, (unsigned *)nullptr, (unsigned *)nullptr,
                           uniq.as<unsigned>());
    unsigned U = 0;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&U, uniq.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    scratch.release();
    unsigned long long cap = 64;
    while (cap < 4ull * U) cap <<= 1;
    // device probes use 32-bit slot indices
    if (cap > (1ull << 32)) FAIL(c, SCQMC_E_UNSUPPORTED, "hash table of more than 2^32 slots");
    t.cap = cap;
    t.unique = U;
    TRY(dalloc(c, cnt, sizeof(unsigned) * cap));
    TRY(dalloc(c, off, sizeof(unsigned) * cap));
    TRY(dalloc(c, cur, sizeof(unsigned) * cap));
    TRY(dalloc(c, slot_of, sizeof(unsigned) * M));
    TRY(dalloc(c, tmp, sizeof(unsigned long long) * M));
    TRY(dalloc(c, total, sizeof(unsigned)));
    TRY(dalloc(c, t.slots, sizeof(ulonglong2) * cap));
    if (mode != 0) TRY(dalloc(c, t.ents, sizeof(ListEnt) * M));
    hipLaunchKernelGGL(k_fill_slots, dim3(grid1(cap, 256)), dim3(256), 0, st, t.slots.as<ulonglong2>(), (long long)cap);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid1(cap, 256)), dim3(256), 0, st, cnt.as<unsigned>(), (long long)cap, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid1(cap, 256)), dim3(256), 0, st, cur.as<unsigned>(), (long long)cap, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(32), 0, st, total.as<unsigned>(), 1LL, 0u);
    if (M > 0)
        hipLaunchKernelGGL(k_insert, dim3(grid1(M, 256)), dim3(256), 0, st, ekeys.as<unsigned long long>(), M,
                           (unsigned long long *)t.slots.p, 2, cap - 1, cnt.as<unsigned>(), slot_of.as<unsigned>(),
                           (unsigned *)nullptr);
    hipLaunchKernelGGL(k_assign, dim3(grid1(cap, 256)), dim3(256), 0, st, cnt.as<unsigned>(), (long long)cap,
                       off.as<unsigned>(), total.as<unsigned>());
    if (M > 0)
        hipLaunchKernelGGL(k_scatter, dim3(grid1(M, 256)), dim3(256), 0, st, slot_of.as<unsigned>(),
                           epay.as<unsigned long long>(), M, off.as<unsigned>(), cur.as<unsigned>(),
                           tmp.as<unsigned long long>());
    hipLaunchKernelGGL(k_finish, dim3(grid1(cap, 256)), dim3(256), 0, st, cnt.as<unsigned>(), off.as<unsigned>(),
                       (long long)cap, tmp.as<unsigned long long>(), c->refcoef.as<double>(), t.slots.as<ulonglong2>(),
                       mode != 0 ? t.ents.as<ListEnt>() : (ListEnt *)nullptr);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    return SCQMC_OK;
}

scqmc_status scqmc_set_reference(scqmc_ctx *c, int64_t n_det, const uint64_t *dets, const double *coeff) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_ints) FAIL(c, SCQMC_E_STATE, "set_integrals first");
    if (n_det <= 0 || !dets || !coeff) FAIL(c, SCQMC_E_INVALID_ARG, "empty reference");
    if (n_det > (1LL << 40)) FAIL(c, SCQMC_E_UNSUPPORTED, "reference too large");
    if (!all_finite(coeff, n_det)) FAIL(c, SCQMC_E_NUMERIC, "non-finite reference coefficient");
    std::vector<unsigned long long> keys(n_det);
    bool any = false;
    for (long long i = 0; i < n_det; i++) {
        unsigned virt;
        std::string why;
        if (!compact_host(c, dets + i * 2 * c->words, keys[i], virt, why))
            FAIL(c, SCQMC_E_INVALID_ARG, "reference determinant " + std::to_string(i) + ": " + why);
        if (virt != (SCQ_NOVIRT | (SCQ_NOVIRT << 16)))
            FAIL(c, SCQMC_E_INVALID_ARG, "reference determinant " + std::to_string(i) + " has a virtual electron");
        any |= coeff[i] != 0.0;
    }
    if (!any) FAIL(c, SCQMC_E_INVALID_ARG, "all reference coefficients are zero");
    std::vector<unsigned long long> sk(keys);
    std::sort(sk.begin(), sk.end());
    if (std::adjacent_find(sk.begin(), sk.end()) != sk.end()) FAIL(c, SCQMC_E_INVALID_ARG, "duplicate reference determinant");
    HIPCHK(c, hipSetDevice(c->device));
    DBuf &rk = c->refkey;
    TRY(dalloc(c, rk, sizeof(unsigned long long) * n_det));
    TRY(dalloc(c, c->refcoef, sizeof(double) * n_det));
    c->refcoef_h.assign(coeff, coeff + n_det);
    HIPCHK(c, hipMemcpyAsync(rk.p, keys.data(), sizeof(unsigned long long) * n_det, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->refcoef.p, c->refcoef_h.data(), sizeof(double) * n_det, hipMemcpyHostToDevice,
                             c->stream));
    TRY(build_table(c, 0, rk, n_det, c->ref));
    TRY(build_table(c, 1, rk, n_det, c->ytab));
    TRY(build_table(c, 2, rk, n_det, c->xtab));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->n_ref = n_det;
    c->has_ref = true;
    c->has_walkers = false;
    return SCQMC_OK;
}

scqmc_status scqmc_set_sc_coeffs(scqmc_ctx *c, double c0, const double *c_cls, int64_t n) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_ref) FAIL(c, SCQMC_E_STATE, "set_reference first");
    if (n != c->ncls - 1 || (n > 0 && !c_cls))
        FAIL(c, SCQMC_E_INVALID_ARG, "expected " + std::to_string(c->ncls - 1) + " class coefficients");
    if (!std::isfinite(c0) || !all_finite(c_cls, n)) FAIL(c, SCQMC_E_NUMERIC, "non-finite coefficient");
    c->ccls_h.assign(c->ncls, 0.0);
    c->ccls_h[0] = c0;
    for (long long i = 0; i < n; i++) c->ccls_h[i + 1] = c_cls[i];
    c->am_m.clear();
    c->am_v.clear();
    c->am_vmax.clear();
    HIPCHK(c, hipSetDevice(c->device));
    TRY(dalloc(c, c->ccls, sizeof(double) * c->ncls));
    HIPCHK(c, hipMemcpyAsync(c->ccls.p, c->ccls_h.data(), sizeof(double) * c->ncls, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_coef = true;
    c->has_walkers = false;
    return SCQMC_OK;
}

scqmc_status scqmc_set_dyall(scqmc_ctx *c, const double *eps_virt, double e0_ref) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_coef) FAIL(c, SCQMC_E_STATE, "set_sc_coeffs first");
    if (!eps_virt && c->V > 0) FAIL(c, SCQMC_E_INVALID_ARG, "null eps_virt");
    if (!std::isfinite(e0_ref) || !all_finite(eps_virt, c->V)) FAIL(c, SCQMC_E_NUMERIC, "non-finite Dyall input");
    c->eps_h.assign(eps_virt, eps_virt + c->V);
    HIPCHK(c, hipSetDevice(c->device));
    TRY(dalloc(c, c->eps, sizeof(double) * std::max(c->V, 1)));
    HIPCHK(c, hipMemcpyAsync(c->eps.p, c->eps_h.data(), sizeof(double) * c->V, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->e0_ref = e0_ref;
    c->has_dyall = true;
    return SCQMC_OK;
}

// ---------------------------------------------------------------------------
// reference properties and semicanonical virtual orbitals (Dyall setup)
// ---------------------------------------------------------------------------
static double fixed_to_double(unsigned long long lo, unsigned long long hi);
static size_t kernel_lds(const scqmc_ctx *c) { return WPB * wave_lds_bytes(lists_per_group(c)); }

static double ref_norm2(const scqmc_ctx *c) {
    double s = 0.0, comp = 0.0;   // Neumaier
    for (double x : c->refcoef_h) {
        double v = x * x, t = s + v;
        comp += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    return s + comp;
}

static scqmc_status ref_rdm1(scqmc_ctx *c, std::vector<double> &gamma) {
    int A = c->A;
    DBuf acc;
    TRY(dalloc(c, acc, sizeof(unsigned long long) * 2 * A * A));
    HIPCHK(c, hipMemsetAsync(acc.p, 0, sizeof(unsigned long long) * 2 * A * A, c->stream));
    DevProblem P = dev_problem(c);
    hipLaunchKernelGGL(k_ref_rdm1, dim3(grid1(c->n_ref, 64)), dim3(64), 0, c->stream, P,
                       c->refkey.as<unsigned long long>(), c->refcoef.as<double>(), (long long)c->n_ref,
                       acc.as<unsigned long long>());
    HIPCHK(c, hipGetLastError());
    std::vector<unsigned long long> h(2 * A * A);
    HIPCHK(c, hipMemcpyAsync(h.data(), acc.p, sizeof(unsigned long long) * 2 * A * A, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double n = ref_norm2(c);
    gamma.resize(A * A);
    for (int k = 0; k < A * A; k++) gamma[k] = fixed_to_double(h[2 * k], h[2 * k + 1]) / n;
    return SCQMC_OK;
}

static scqmc_status ref_energy(scqmc_ctx *c, double &e0) {
    long long n = c->n_ref;
    DBuf virt, valid, eloc, one;
    TRY(dalloc(c, virt, sizeof(unsigned) * n));
    TRY(dalloc(c, valid, sizeof(int) * n));
    TRY(dalloc(c, eloc, sizeof(double) * n));
    TRY(dalloc(c, one, sizeof(double)));
    std::vector<unsigned> hv(n, SCQ_NOVIRT | (SCQ_NOVIRT << 16));
    std::vector<int> hval(n);
    for (long long i = 0; i < n; i++) hval[i] = c->refcoef_h[i] != 0.0;
    const double h1 = 1.0;
    HIPCHK(c, hipMemcpyAsync(virt.p, hv.data(), sizeof(unsigned) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(valid.p, hval.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(one.p, &h1, sizeof(double), hipMemcpyHostToDevice, c->stream));
    // (H phi0)(d) / phi0(d) from the walker kernel over active-space neighbours
    // only, with the active-space coefficient c0 = 1
    DevProblem P = dev_problem(c);
    P.ccls = one.as<double>();
    P.mode = 0;
    P.eps_screen = 0.0;
    P.active_only = 1;
    int NL = lists_per_group(c);
    hipLaunchKernelGGL(k_eval<double>, dim3(grid1(n, WPB)), dim3(64 * WPB), kernel_lds(c), c->stream, P,
                       c->refkey.as<unsigned long long>(), virt.as<unsigned>(), valid.as<int>(), n, NL,
                       eloc.as<double>(), (double *)nullptr, (double *)nullptr, (double *)nullptr, (int *)nullptr,
                       (double *)nullptr);
    HIPCHK(c, hipGetLastError());
    std::vector<double> el(n);
    HIPCHK(c, hipMemcpyAsync(el.data(), eloc.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double s = 0.0, comp = 0.0;
    for (long long i = 0; i < n; i++) {
        double x = c->refcoef_h[i];
        if (x == 0.0) continue;
        if (!std::isfinite(el[i])) FAIL(c, SCQMC_E_NUMERIC, "non-finite local energy of a reference determinant");
        double v = x * x * el[i], t = s + v;
        comp += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    e0 = (s + comp) / ref_norm2(c);
    return SCQMC_OK;
}

// Eigen-decomposition of a symmetric matrix by cyclic Jacobi rotations;
// eigenvalues ascending, each eigenvector's largest-|component| positive.
static void jacobi_eigh(int n, std::vector<double> a, std::vector<double> &w, std::vector<double> &v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-34 * tot || off == 0.0) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; k++) {   // A <- A J (columns p, q)
                    double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = cs * akp - sn * akq;
                    a[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; k++) {   // A <- J^T A (rows p, q)
                    double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = cs * apk - sn * aqk;
                    a[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; k++) {   // V <- V J
                    double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    v[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; i++) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a[(size_t)x * n + x] < a[(size_t)y * n + y]; });
    std::vector<double> vs((size_t)n * n);
    w.resize(n);
    for (int k = 0; k < n; k++) {
        int j = ord[k];
        w[k] = a[(size_t)j * n + j];
        int imax = 0;
        for (int i = 1; i < n; i++)
            if (std::fabs(v[(size_t)i * n + j]) > std::fabs(v[(size_t)imax * n + j])) imax = i;
        double sg = v[(size_t)imax * n + j] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; i++) vs[(size_t)i * n + k] = sg * v[(size_t)i * n + j];
    }
    v.swap(vs);
}

scqmc_status scqmc_reference_energy(scqmc_ctx *c, double *e0) {
    if (!c || !e0) return SCQMC_E_INVALID_ARG;
    if (!c->has_ref) FAIL(c, SCQMC_E_STATE, "set_reference first");
    HIPCHK(c, hipSetDevice(c->device));
    return ref_energy(c, *e0);
}

scqmc_status scqmc_reference_rdm1(scqmc_ctx *c, double *gamma) {
    if (!c || !gamma) return SCQMC_E_INVALID_ARG;
    if (!c->has_ref) FAIL(c, SCQMC_E_STATE, "set_reference first");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<double> g;
    TRY(ref_rdm1(c, g));
    std::memcpy(gamma, g.data(), sizeof(double) * g.size());
    return SCQMC_OK;
}

scqmc_status scqmc_semicanonicalize(scqmc_ctx *c, double *eps_virt, double *u_out) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_ref) FAIL(c, SCQMC_E_STATE, "set_reference first");
    HIPCHK(c, hipSetDevice(c->device));
    int A = c->A, V = c->V, Np = c->Np;
    std::vector<double> gamma;
    TRY(ref_rdm1(c, gamma));
    std::vector<double> F((size_t)V * V), w, U;
    if (V > 0) {
        DBuf dg, dF;
        TRY(dalloc(c, dg, sizeof(double) * A * A));
        TRY(dalloc(c, dF, sizeof(double) * V * V));
        HIPCHK(c, hipMemcpyAsync(dg.p, gamma.data(), sizeof(double) * A * A, hipMemcpyHostToDevice, c->stream));
        DevProblem P = dev_problem(c);
        hipLaunchKernelGGL(k_virtual_fock, dim3(grid1((long long)V * V, 256)), dim3(256), 0, c->stream, P,
                           dg.as<double>(), dF.as<double>());
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(F.data(), dF.p, sizeof(double) * V * V, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int a = 0; a < V; a++)   // exact symmetry before the eigen-decomposition
            for (int b = a + 1; b < V; b++) {
                double m = 0.5 * (F[(size_t)a * V + b] + F[(size_t)b * V + a]);
                F[(size_t)a * V + b] = F[(size_t)b * V + a] = m;
            }
        if (!all_finite(F.data(), (long long)V * V)) FAIL(c, SCQMC_E_NUMERIC, "non-finite virtual Fock matrix");
        jacobi_eigh(V, F, w, U);
        // one-body operator: h' = T^T h T with T = diag(1_A, U)
        std::vector<double> h((size_t)Np * Np), h2((size_t)Np * Np);
        HIPCHK(c, hipMemcpyAsync(h.data(), c->heff.p, sizeof(double) * Np * Np, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        auto T = [&](int k, int j) -> double {   // T[k][j]
            if (k < A || j < A) return k == j ? 1.0 : 0.0;
            return U[(size_t)(k - A) * V + (j - A)];
        };
        for (int i = 0; i < Np; i++)
            for (int j = 0; j < Np; j++) {
                double s = 0.0;
                for (int k = 0; k < Np; k++) {
                    double tk = T(k, j);
                    if (tk != 0.0) s += h[(size_t)i * Np + k] * tk;
                }
                h2[(size_t)i * Np + j] = s;
            }
        for (int i = 0; i < Np; i++)
            for (int j = 0; j < Np; j++) {
                double s = 0.0;
                for (int k = 0; k < Np; k++) {
                    double tk = T(k, i);
                    if (tk != 0.0) s += tk * h2[(size_t)k * Np + j];
                }
                h[(size_t)i * Np + j] = s;
            }
        for (int i = 0; i < Np; i++)
            for (int j = i + 1; j < Np; j++) {
                double m = 0.5 * (h[(size_t)i * Np + j] + h[(size_t)j * Np + i]);
                h[(size_t)i * Np + j] = h[(size_t)j * Np + i] = m;
            }
        HIPCHK(c, hipMemcpyAsync(c->heff.p, h.data(), sizeof(double) * Np * Np, hipMemcpyHostToDevice, c->stream));
        // two-electron block: one index at a time
        DBuf dU, tmp;
        TRY(dalloc(c, dU, sizeof(double) * V * V));
        TRY(dalloc(c, tmp, c->eri.n));
        HIPCHK(c, hipMemcpyAsync(dU.p, U.data(), sizeof(double) * V * V, hipMemcpyHostToDevice, c->stream));
        for (int pos = 0; pos < 4; pos++) {
            const double *in = (pos & 1) ? tmp.as<double>() : c->eri.as<double>();
            double *out = (pos & 1) ? c->eri.as<double>() : tmp.as<double>();
            hipLaunchKernelGGL(k_rotate_eri, dim3(4096), dim3(256), 0, c->stream, in, out, Np, A,
                               dU.as<double>(), pos);
            HIPCHK(c, hipGetLastError());
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->ints_version++;
    }
    double e0;
    TRY(ref_energy(c, e0));
    c->eps_h.assign(w.begin(), w.end());
    TRY(dalloc(c, c->eps, sizeof(double) * std::max(V, 1)));
    if (V > 0)
        HIPCHK(c, hipMemcpyAsync(c->eps.p, c->eps_h.data(), sizeof(double) * V, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->e0_ref = e0;
    c->has_dyall = true;
    c->has_walkers = false;
    if (eps_virt && V > 0) std::memcpy(eps_virt, w.data(), sizeof(double) * V);
    if (u_out && V > 0) std::memcpy(u_out, U.data(), sizeof(double) * V * V);
    return SCQMC_OK;
}

scqmc_status scqmc_set_options(scqmc_ctx *c, const scqmc_options *o) {
    if (!c || !o) return SCQMC_E_INVALID_ARG;
    if (!c->has_space) FAIL(c, SCQMC_E_STATE, "set_space first");
    if (!std::isfinite(o->eps_screen) || o->eps_screen < 0) FAIL(c, SCQMC_E_INVALID_ARG, "eps_screen must be >= 0");
    if (o->mode != 0 && o->mode != 1) FAIL(c, SCQMC_E_INVALID_ARG, "mode must be 0 or 1");
    if (o->precision != 0 && o->precision != 1) FAIL(c, SCQMC_E_INVALID_ARG, "precision must be 0 (FP64) or 1 (FP32 form)");
    if (o->burn_in < 0 || o->block_len < 0) FAIL(c, SCQMC_E_INVALID_ARG, "negative burn_in / block_len");
    // walkers carry psi(n) of the form they were placed with
    if (o->precision != c->opt.precision) c->has_walkers = false;
    c->opt = *o;
    return SCQMC_OK;
}


static scqmc_status ready_for_walkers(scqmc_ctx *c) {
    if (!c->has_coef) FAIL(c, SCQMC_E_STATE, "set_space / integrals / reference / sc_coeffs first");
    if (c->opt.mode == 1 && !c->has_dyall) FAIL(c, SCQMC_E_STATE, "mode 1 needs set_dyall");
    return SCQMC_OK;
}

scqmc_status scqmc_init_walkers(scqmc_ctx *c, int64_t W, const uint64_t *dets, uint64_t seed) {
    if (!c) return SCQMC_E_INVALID_ARG;
    TRY(ready_for_walkers(c));
    if (W <= 0 || W >= (1LL << 31) || !dets) FAIL(c, SCQMC_E_INVALID_ARG, "n_walkers must be in [1, 2^31)");
    std::vector<unsigned long long> keys(W);
    std::vector<unsigned> virts(W);
    for (long long i = 0; i < W; i++) {
        std::string why;
        if (!compact_host(c, dets + i * 2 * c->words, keys[i], virts[i], why))
            FAIL(c, SCQMC_E_INVALID_ARG, "walker " + std::to_string(i) + ": " + why);
    }
    HIPCHK(c, hipSetDevice(c->device));
    TRY(dalloc(c, c->wkey, sizeof(unsigned long long) * W));
    TRY(dalloc(c, c->wvirt, sizeof(unsigned) * W));
    TRY(dalloc(c, c->worder, sizeof(int) * W));
    TRY(dalloc(c, c->wpsi, sizeof(double) * W));
    TRY(dalloc(c, c->wsum, sizeof(double) * 3 * W));
    c->ncg = class_groups(W);
    TRY(dalloc(c, c->cacc, class_acc_bytes(c)));
    TRY(dalloc(c, c->bad, sizeof(unsigned long long)));
    TRY(dalloc(c, c->wftab, ftab_bytes(c) * W));
    HIPCHK(c, hipMemcpyAsync(c->wkey.p, keys.data(), sizeof(unsigned long long) * W, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->wvirt.p, virts.data(), sizeof(unsigned) * W, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->wsum.p, 0, sizeof(double) * 3 * W, c->stream));
    HIPCHK(c, hipMemsetAsync(c->cacc.p, 0, class_acc_bytes(c), c->stream));
    HIPCHK(c, hipMemsetAsync(c->bad.p, 0, sizeof(unsigned long long), c->stream));
    c->seed = seed;
    TRY(ensure_f32(c));
    DevProblem P = dev_problem(c);
    if (c->opt.precision == 1)
        hipLaunchKernelGGL(k_psi<float>, dim3(grid1(W, 64)), dim3(64), 0, c->stream, P,
                           c->wkey.as<unsigned long long>(), c->wvirt.as<unsigned>(), (long long)W, c->wpsi.as<double>());
    else
        hipLaunchKernelGGL(k_psi<double>, dim3(grid1(W, 64)), dim3(64), 0, c->stream, P,
                           c->wkey.as<unsigned long long>(), c->wvirt.as<unsigned>(), (long long)W, c->wpsi.as<double>());
    HIPCHK(c, hipGetLastError());
    std::vector<double> psi(W);
    HIPCHK(c, hipMemcpyAsync(psi.data(), c->wpsi.p, sizeof(double) * W, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (long long i = 0; i < W; i++) {
        if (!std::isfinite(psi[i])) FAIL(c, SCQMC_E_NUMERIC, "walker " + std::to_string(i) + ": non-finite psi");
        if (psi[i] == 0.0) FAIL(c, SCQMC_E_INVALID_ARG, "walker " + std::to_string(i) + " has psi = 0");
    }
    c->W = W;
    c->step = 0;
    c->has_walkers = true;
    return SCQMC_OK;
}

// n_steps steps of every walker in launches of block_len steps, each launch
// preceded by the walker order of its dispatch (k_order)
static scqmc_status launch_sample(scqmc_ctx *c, long long n_steps, long long burn_in) {
    DevProblem P = dev_problem(c);
    WalkerArrays S;
    S.key = c->wkey.as<unsigned long long>();
    S.virt = c->wvirt.as<unsigned>();
    S.psi = c->wpsi.as<double>();
    S.wsum = c->wsum.as<double>();
    S.cacc = c->cacc.as<unsigned long long>();
    S.ncg = (int)c->ncg;
    S.bad = c->bad.as<unsigned long long>();
    S.ftab = c->wftab.as<double>();
    int NL = lists_per_group(c);
    size_t lds = kernel_lds(c);
    int *order = c->worder.as<int>();
    long long blk = c->opt.block_len > 0 ? c->opt.block_len : 1;
    for (long long done = 0; done < n_steps; done += blk) {
        int ns = (int)std::min(blk, n_steps - done);
        hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, c->stream, c->wvirt.as<const unsigned>(), c->W, (int)c->V,
                           order);
        if (c->opt.precision == 1)
            hipLaunchKernelGGL(k_sample<float>, dim3(grid1(c->W, WPB)), dim3(64 * WPB), lds, c->stream, P, S, order,
                               c->W, c->step + done, ns, burn_in, NL);
        else
            hipLaunchKernelGGL(k_sample<double>, dim3(grid1(c->W, WPB)), dim3(64 * WPB), lds, c->stream, P, S, order,
                               c->W, c->step + done, ns, burn_in, NL);
        HIPCHK(c, hipGetLastError());
    }
    c->step += n_steps;
    return SCQMC_OK;
}

scqmc_status scqmc_sample(scqmc_ctx *c, int64_t n_steps) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    if (c->opt.mode == 1 && !c->has_dyall) FAIL(c, SCQMC_E_STATE, "mode 1 needs set_dyall");
    if (n_steps < 0) FAIL(c, SCQMC_E_INVALID_ARG, "negative n_steps");
    if (c->step + n_steps >= (1LL << 31)) FAIL(c, SCQMC_E_UNSUPPORTED, "step counter limit (2^31) reached");
    HIPCHK(c, hipSetDevice(c->device));
    TRY(ensure_f32(c));
    return launch_sample(c, n_steps, (long long)c->opt.burn_in);
}

scqmc_status scqmc_synchronize(scqmc_ctx *c) {
    if (!c) return SCQMC_E_INVALID_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SCQMC_OK;
}

static double fixed_to_double(unsigned long long lo, unsigned long long hi) {
    return (double)(long long)hi + std::ldexp((double)lo, -64);
}

// ws: per-walker sums [3][W]; cs: class sums over all walkers [4][ncls] (exact
// 128-bit totals, then rounded); gs (optional): per walker group [ncg][4][ncls]
static scqmc_status download_sums(scqmc_ctx *c, std::vector<double> &ws, std::vector<double> &cs,
                                  std::vector<double> *gs = nullptr) {
    ws.resize(3 * c->W);
    long long n4 = 4 * c->ncls;
    std::vector<unsigned long long> acc(2 * n4 * c->ncg);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(ws.data(), c->wsum.p, sizeof(double) * 3 * c->W, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(acc.data(), c->cacc.p, class_acc_bytes(c), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    cs.resize(n4);
    if (gs) gs->resize(n4 * c->ncg);
    for (long long i = 0; i < n4; i++) {
        unsigned long long lo = 0, hi = 0;
        for (long long g = 0; g < c->ncg; g++) {
            unsigned long long l = acc[2 * (g * n4 + i)], h = acc[2 * (g * n4 + i) + 1];
            unsigned long long nl = lo + l;
            hi += h + (nl < lo ? 1ull : 0ull);
            lo = nl;
            if (gs) (*gs)[g * n4 + i] = fixed_to_double(l, h);
        }
        cs[i] = fixed_to_double(lo, hi);
    }
    return SCQMC_OK;
}

// E^(2) of eq:nevpt2e2 from class sums N_l = sum t/c_l^2, D_l = sum t E_D,L/c_l^2;
// perturbers whose relative norm N_l/N_0 is below tau are left out (the
// optional small-norm screen at the end of "SC-NEVPT2(s)")
static double e2_from_sums(const double *nl_, const double *dl_, long long n, double e0, double tau) {
    double n0 = nl_[0];
    if (!(n0 > 0)) return NAN;
    double e2 = 0;
    for (long long l = 1; l < n; l++) {
        double nl = nl_[l];
        if (nl <= 0 || nl / n0 < tau) continue;
        e2 += (nl / n0) / (e0 - dl_[l] / nl);
    }
    return e2;
}

// E_var, a0^2 and their delete-one jackknife errors over min(W, 256) groups
// of consecutive walkers, from the per-walker sums
static void energy_from_walker_sums(const scqmc_ctx *c, const std::vector<double> &ws, scqmc_estimates *out) {
    long long W = c->W;
    long long G = std::min<long long>(W, 256);
    std::vector<double> gt(G, 0.0), gte(G, 0.0), gt0(G, 0.0);
    for (long long w = 0; w < W; w++) {
        long long g = w * G / W;
        gt[g] += ws[w];
        gte[g] += ws[W + w];
        gt0[g] += ws[2 * W + w];
    }
    double St = 0, Ste = 0, St0 = 0;
    for (long long g = 0; g < G; g++) { St += gt[g]; Ste += gte[g]; St0 += gt0[g]; }
    std::memset(out, 0, sizeof(*out));
    out->n_walkers = W;
    out->n_steps_accumulated = std::max<long long>(0, c->step - c->opt.burn_in);
    if (St > 0) {
        out->e_var = Ste / St;
        out->a0_sq = St0 / St;
        double me = 0, ma = 0;
        std::vector<double> je(G), ja(G);
        for (long long g = 0; g < G; g++) {
            double d = St - gt[g];
            je[g] = d > 0 ? (Ste - gte[g]) / d : out->e_var;
            ja[g] = d > 0 ? (St0 - gt0[g]) / d : out->a0_sq;
            me += je[g];
            ma += ja[g];
        }
        me /= G;
        ma /= G;
        double ve = 0, va = 0;
        for (long long g = 0; g < G; g++) { ve += (je[g] - me) * (je[g] - me); va += (ja[g] - ma) * (ja[g] - ma); }
        out->e_var_err = G > 1 ? std::sqrt((G - 1.0) / G * ve) : NAN;
        out->a0_sq_err = G > 1 ? std::sqrt((G - 1.0) / G * va) : NAN;
    } else {
        out->e_var = out->e_var_err = out->a0_sq = out->a0_sq_err = NAN;
    }
}

scqmc_status scqmc_read_energy(scqmc_ctx *c, double *e_var, double *e_var_err, double *a0_sq) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<double> ws(3 * c->W);
    HIPCHK(c, hipMemcpyAsync(ws.data(), c->wsum.p, sizeof(double) * 3 * c->W, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    scqmc_estimates est;
    energy_from_walker_sums(c, ws, &est);
    if (e_var) *e_var = est.e_var;
    if (e_var_err) *e_var_err = est.e_var_err;
    if (a0_sq) *a0_sq = est.a0_sq;
    return SCQMC_OK;
}

scqmc_status scqmc_read_estimates(scqmc_ctx *c, scqmc_estimates *out) {
    if (!c || !out) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    std::vector<double> ws, cs, gsum;
    TRY(download_sums(c, ws, cs, &gsum));
    energy_from_walker_sums(c, ws, out);
    out->e_ref = c->has_dyall ? c->e0_ref : 0.0;
    out->davidson = c->has_dyall ? (1.0 - out->a0_sq) * (out->e_var - c->e0_ref) : NAN;
    out->e2 = NAN;
    out->e2_err = NAN;
    if (c->opt.mode == 1 && c->has_dyall) {
        long long n = c->ncls, K = c->ncg;
        out->e2 = e2_from_sums(&cs[2 * n], &cs[3 * n], n, c->e0_ref, c->tau);
        // delete-one jackknife over the walker groups of the class sums
        if (K > 1 && std::isfinite(out->e2)) {
            std::vector<double> nl(n), dl(n), je(K);
            double m = 0;
            bool ok = true;
            for (long long g = 0; g < K; g++) {
                const double *gp = &gsum[g * 4 * n];
                for (long long l = 0; l < n; l++) {
                    nl[l] = cs[2 * n + l] - gp[2 * n + l];
                    dl[l] = cs[3 * n + l] - gp[3 * n + l];
                }
                je[g] = e2_from_sums(nl.data(), dl.data(), n, c->e0_ref, c->tau);
                ok = ok && std::isfinite(je[g]);
                m += je[g];
            }
            if (ok) {
                m /= K;
                double v = 0;
                for (long long g = 0; g < K; g++) v += (je[g] - m) * (je[g] - m);
                out->e2_err = std::sqrt((K - 1.0) / K * v);
            }
        }
    }
    return SCQMC_OK;
}

scqmc_status scqmc_set_nevpt2_screen(scqmc_ctx *c, double tau) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!(tau >= 0.0) || !std::isfinite(tau)) FAIL(c, SCQMC_E_INVALID_ARG, "tau must be finite and >= 0");
    c->tau = tau;
    return SCQMC_OK;
}

// First-order wave function of SC-NEVPT2: psi1 = sum_l P_l H phi0 / (E_0 - E_l),
// i.e. coefficient 1/(E_0 - E_l) for the unnormalised perturber of class l,
// with E_l = D_l / N_l from the sampled class sums; delete-one jackknife over
// the walker groups for the error of each coefficient.
scqmc_status scqmc_read_first_order(scqmc_ctx *c, double *coef, double *coef_err, double *e_l, double *rel_norm,
                                    int64_t n) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    if (!(c->opt.mode == 1 && c->has_dyall)) FAIL(c, SCQMC_E_STATE, "needs mode 1 (set_dyall, set_options)");
    if (n != c->ncls - 1) FAIL(c, SCQMC_E_INVALID_ARG, "n must equal n_classes - 1");
    std::vector<double> ws, cs, gsum;
    TRY(download_sums(c, ws, cs, &gsum));
    long long nc = c->ncls, K = c->ncg;
    const double *N = &cs[2 * nc], *D = &cs[3 * nc];
    double n0 = N[0];
    auto coef_of = [&](double nl, double dl, double base) -> double {
        if (!(nl > 0) || !(base > 0)) return NAN;
        if (nl / base < c->tau) return 0.0;
        return 1.0 / (c->e0_ref - dl / nl);
    };
    for (long long l = 1; l < nc; l++) {
        double x = coef_of(N[l], D[l], n0);
        if (coef) coef[l - 1] = x;
        if (e_l) e_l[l - 1] = N[l] > 0 ? D[l] / N[l] : NAN;
        if (rel_norm) rel_norm[l - 1] = n0 > 0 ? N[l] / n0 : NAN;
        if (coef_err) {
            double err = NAN;
            if (K > 1 && std::isfinite(x)) {
                double m = 0, v = 0;
                std::vector<double> je(K);
                bool ok = true;
                for (long long g = 0; g < K; g++) {
                    const double *gp = &gsum[g * 4 * nc];
                    je[g] = coef_of(N[l] - gp[2 * nc + l], D[l] - gp[3 * nc + l], n0 - gp[2 * nc]);
                    ok = ok && std::isfinite(je[g]);
                    m += je[g];
                }
                if (ok) {
                    m /= K;
                    for (long long g = 0; g < K; g++) v += (je[g] - m) * (je[g] - m);
                    err = std::sqrt((K - 1.0) / K * v);
                }
            }
            coef_err[l - 1] = err;
        }
    }
    return SCQMC_OK;
}

scqmc_status scqmc_read_class_sums(scqmc_ctx *c, double *n_l, double *d_l, double *t_l, double *te_l, int64_t n) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    if (n != c->ncls) FAIL(c, SCQMC_E_INVALID_ARG, "n must equal n_classes");
    std::vector<double> ws, cs;
    TRY(download_sums(c, ws, cs));
    for (long long l = 0; l < n; l++) {
        if (t_l) t_l[l] = cs[l];
        if (te_l) te_l[l] = cs[n + l];
        if (n_l) n_l[l] = cs[2 * n + l];
        if (d_l) d_l[l] = cs[3 * n + l];
    }
    return SCQMC_OK;
}

scqmc_status scqmc_read_walker_sums(scqmc_ctx *c, double *sum_t, double *sum_te, double *sum_t0, int64_t n) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    if (n != c->W) FAIL(c, SCQMC_E_INVALID_ARG, "n must equal n_walkers");
    std::vector<double> ws, cs;
    TRY(download_sums(c, ws, cs));
    for (long long w = 0; w < n; w++) {
        if (sum_t) sum_t[w] = ws[w];
        if (sum_te) sum_te[w] = ws[n + w];
        if (sum_t0) sum_t0[w] = ws[2 * n + w];
    }
    return SCQMC_OK;
}

scqmc_status scqmc_read_walkers(scqmc_ctx *c, uint64_t *dets, double *psi, int64_t n) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    if (n != c->W) FAIL(c, SCQMC_E_INVALID_ARG, "n must equal n_walkers");
    std::vector<unsigned long long> keys(n);
    std::vector<unsigned> virts(n);
    std::vector<double> ps(n);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(keys.data(), c->wkey.p, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(virts.data(), c->wvirt.p, sizeof(unsigned) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ps.data(), c->wpsi.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (long long w = 0; w < n; w++) {
        if (dets) expand_host(c, keys[w], virts[w], dets + w * 2 * c->words);
        if (psi) psi[w] = ps[w];
    }
    return SCQMC_OK;
}

scqmc_status scqmc_read_counters(scqmc_ctx *c, int64_t *steps, int64_t *bad_steps) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    unsigned long long b = 0;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(&b, c->bad.p, sizeof(b), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (steps) *steps = c->step;
    if (bad_steps) *bad_steps = (int64_t)b;
    return SCQMC_OK;
}

scqmc_status scqmc_eval_snapshot(scqmc_ctx *c, int64_t n, const uint64_t *d_dets, double *d_eloc, double *d_psi,
                                 double *d_gamma, double *d_eloc_dyall, int32_t *d_class) {
    if (!c) return SCQMC_E_INVALID_ARG;
    TRY(ready_for_walkers(c));
    if (n < 0 || (n > 0 && !d_dets)) FAIL(c, SCQMC_E_INVALID_ARG, "bad snapshot arguments");
    if (n == 0) return SCQMC_OK;
    HIPCHK(c, hipSetDevice(c->device));
    if (c->skey.n < sizeof(unsigned long long) * n) {
        TRY(dalloc(c, c->skey, sizeof(unsigned long long) * n));
        TRY(dalloc(c, c->svirt, sizeof(unsigned) * n));
        TRY(dalloc(c, c->svalid, sizeof(int) * n));
    }
    hipLaunchKernelGGL(k_compact, dim3(grid1(n, 128)), dim3(128), 0, c->stream, (const unsigned long long *)d_dets,
                       (long long)n, c->words, c->N, c->C, c->A, c->na, c->nb, c->skey.as<unsigned long long>(),
                       c->svirt.as<unsigned>(), c->svalid.as<int>());
    TRY(ensure_f32(c));
    DevProblem P = dev_problem(c);
    int NL = lists_per_group(c);
    double *d_eld = (c->opt.mode == 1 && c->has_dyall) ? d_eloc_dyall : nullptr;
    long long slots = std::min<long long>(n, SCQ_EVAL_SLOTS);
    if (c->sftab.n < ftab_bytes(c) * slots) TRY(dalloc(c, c->sftab, ftab_bytes(c) * slots));
    unsigned grid = grid1(slots, WPB);
    if (c->opt.precision == 1)
        hipLaunchKernelGGL(k_eval<float>, dim3(grid), dim3(64 * WPB), kernel_lds(c), c->stream, P,
                           c->skey.as<unsigned long long>(), c->svirt.as<unsigned>(), c->svalid.as<int>(),
                           (long long)n, NL, d_eloc, d_psi, d_gamma, d_eld, (int *)d_class, c->sftab.as<double>());
    else
        hipLaunchKernelGGL(k_eval<double>, dim3(grid), dim3(64 * WPB), kernel_lds(c), c->stream, P,
                           c->skey.as<unsigned long long>(), c->svirt.as<unsigned>(), c->svalid.as<int>(),
                           (long long)n, NL, d_eloc, d_psi, d_gamma, d_eld, (int *)d_class, c->sftab.as<double>());
    HIPCHK(c, hipGetLastError());
    if (d_eloc_dyall && !(c->opt.mode == 1 && c->has_dyall)) {
        std::vector<double> nanv(n, NAN);
        HIPCHK(c, hipMemcpyAsync(d_eloc_dyall, nanv.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return SCQMC_OK;
}

scqmc_status scqmc_eval_snapshot_noalloc(scqmc_ctx *c, int64_t n, const uint64_t *d_dets, double *d_eloc,
                                         double *d_psi, double *d_gamma, double *d_eloc_dyall, int32_t *d_class) {
    if (!c) return SCQMC_E_INVALID_ARG;
    TRY(ready_for_walkers(c));
    if (n < 0 || (n > 0 && !d_dets)) FAIL(c, SCQMC_E_INVALID_ARG, "bad snapshot arguments");
    if (n > SCQMC_NOALLOC_MAX_DETS)
        FAIL(c, SCQMC_E_INVALID_ARG, "snapshot of " + std::to_string(n) + " determinants; the allocation-free entry "
                                     "point takes at most " + std::to_string(SCQMC_NOALLOC_MAX_DETS));
    if (c->opt.precision == 1 && c->f32_version != c->ints_version)
        FAIL(c, SCQMC_E_STATE, "precision form: the FP32 integral copies are not made yet (any sample or "
                               "eval_snapshot call makes them)");
    if (!c->scratch_ptr) FAIL(c, SCQMC_E_DEVICE, "no scratch address for this device");
    if (n == 0) return SCQMC_OK;
    HIPCHK(c, hipSetDevice(c->device));
    unsigned char *base = (unsigned char *)c->scratch_ptr;
    unsigned long long *skey = (unsigned long long *)base;
    unsigned *svirt = (unsigned *)(base + (size_t)SCQMC_NOALLOC_MAX_DETS * 8);
    int *svalid = (int *)(base + (size_t)SCQMC_NOALLOC_MAX_DETS * 12);
    // k_compact writes every entry i < n, so nothing has to be cleared
    hipLaunchKernelGGL(k_compact, dim3(grid1(n, 128)), dim3(128), 0, c->stream, (const unsigned long long *)d_dets,
                       (long long)n, c->words, c->N, c->C, c->A, c->na, c->nb, skey, svirt, svalid);
    DevProblem P = dev_problem(c);
    int NL = lists_per_group(c);
    bool dy = c->opt.mode == 1 && c->has_dyall;
    // wave slots: as many Fock tables as the fixed array holds (at least one:
    // a table is at most 2 * 32 * 96 doubles), grid-stride beyond
    double *ftab = (double *)(base + (size_t)SCQMC_NOALLOC_MAX_DETS * 16);
    long long slots = std::min<long long>({(long long)n, (long long)SCQ_EVAL_SLOTS,
                                           (long long)(SCQMC_NOALLOC_FTAB_BYTES / ftab_bytes(c))});
    unsigned grid = (unsigned)std::max<long long>(1, slots / WPB);
    if (c->opt.precision == 1)
        hipLaunchKernelGGL(k_eval<float>, dim3(grid), dim3(64 * WPB), kernel_lds(c), c->stream, P, skey, svirt,
                           svalid, (long long)n, NL, d_eloc, d_psi, d_gamma, dy ? d_eloc_dyall : nullptr,
                           (int *)d_class, ftab);
    else
        hipLaunchKernelGGL(k_eval<double>, dim3(grid), dim3(64 * WPB), kernel_lds(c), c->stream, P, skey, svirt,
                           svalid, (long long)n, NL, d_eloc, d_psi, d_gamma, dy ? d_eloc_dyall : nullptr,
                           (int *)d_class, ftab);
    if (d_eloc_dyall && !dy)   // no Dyall energies in mode 0: NaN, filled by a kernel (no copy, no wait)
        hipLaunchKernelGGL(k_fill_u64, dim3(grid1(n, 256)), dim3(256), 0, c->stream, (unsigned long long *)d_eloc_dyall,
                           (long long)n, 0x7FF8000000000000ull);
    HIPCHK(c, hipGetLastError());
    return SCQMC_OK;
}

scqmc_status scqmc_debug_neighbors(scqmc_ctx *c, const uint64_t *det, int64_t cap, uint64_t *out_dets,
                                   int8_t *out_phase, double *out_hnm, double *out_psi, int64_t *out_count) {
    if (!c) return SCQMC_E_INVALID_ARG;
    TRY(ready_for_walkers(c));
    if (!det || cap < 0 || !out_count) FAIL(c, SCQMC_E_INVALID_ARG, "bad arguments");
    unsigned long long key;
    unsigned virt;
    std::string why;
    if (!compact_host(c, det, key, virt, why)) FAIL(c, SCQMC_E_INVALID_ARG, "determinant: " + why);
    HIPCHK(c, hipSetDevice(c->device));
    long long m = std::max<long long>(cap, 1);
    DBuf k, v, ph, h, p, cnt;
    TRY(dalloc(c, k, sizeof(unsigned long long) * m));
    TRY(dalloc(c, v, sizeof(unsigned) * m));
    TRY(dalloc(c, ph, sizeof(signed char) * m));
    TRY(dalloc(c, h, sizeof(double) * m));
    TRY(dalloc(c, p, sizeof(double) * m));
    TRY(dalloc(c, cnt, sizeof(unsigned long long)));
    HIPCHK(c, hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), c->stream));
    DevProblem P = dev_problem(c);
    int NL = lists_per_group(c);
    hipLaunchKernelGGL(k_neighbors, dim3(1), dim3(64), wave_lds_bytes(NL), c->stream, P, key, virt, NL, (long long)cap,
                       k.as<unsigned long long>(), v.as<unsigned>(), ph.as<signed char>(), h.as<double>(),
                       p.as<double>(), cnt.as<unsigned long long>());
    HIPCHK(c, hipGetLastError());
    unsigned long long total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, cnt.p, sizeof(total), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    long long nw = std::min<long long>((long long)total, cap);
    std::vector<unsigned long long> kk(nw);
    std::vector<unsigned> vv(nw);
    if (nw > 0) {
        HIPCHK(c, hipMemcpy(kk.data(), k.p, sizeof(unsigned long long) * nw, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(vv.data(), v.p, sizeof(unsigned) * nw, hipMemcpyDeviceToHost));
        if (out_phase) HIPCHK(c, hipMemcpy(out_phase, ph.p, nw, hipMemcpyDeviceToHost));
        if (out_hnm) HIPCHK(c, hipMemcpy(out_hnm, h.p, sizeof(double) * nw, hipMemcpyDeviceToHost));
        if (out_psi) HIPCHK(c, hipMemcpy(out_psi, p.p, sizeof(double) * nw, hipMemcpyDeviceToHost));
        if (out_dets)
            for (long long i = 0; i < nw; i++) expand_host(c, kk[i], vv[i], out_dets + i * 2 * c->words);
    }
    *out_count = (int64_t)total;
    return SCQMC_OK;
}

// checkpoint layout: header of 12 int64, then key[W] u64, virt[W] u32 (padded to 8),
// psi[W], wsum[3W], class sums [ncg][4][ncls] x 2 u64 (ncg = min(W, 16)), bad u64
static const int64_t kMagic = 0x31435153514d4353LL;

static int64_t state_bytes(const scqmc_ctx *c) {
    int64_t W = c->W;
    return 12 * 8 + 8 * W + ((4 * W + 7) / 8) * 8 + 8 * W + 24 * W + 64 * class_groups(W) * c->ncls + 8;
}

scqmc_status scqmc_save_state(scqmc_ctx *c, void *buf, int64_t cap, int64_t *used) {
    if (!c || !used) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    int64_t need = state_bytes(c);
    *used = need;
    if (!buf || cap < need) FAIL(c, SCQMC_E_INVALID_ARG, "buffer too small");
    char *b = (char *)buf;
    std::memset(b, 0, need);
    int64_t hdr[12] = {kMagic, 2, c->W, c->ncls, c->N, c->C, c->A, c->na, c->nb, c->step, (int64_t)c->seed, c->n_ref};
    std::memcpy(b, hdr, sizeof(hdr));
    int64_t W = c->W, o = 96;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(b + o, c->wkey.p, 8 * W, hipMemcpyDeviceToHost)); o += 8 * W;
    HIPCHK(c, hipMemcpy(b + o, c->wvirt.p, 4 * W, hipMemcpyDeviceToHost)); o += ((4 * W + 7) / 8) * 8;
    HIPCHK(c, hipMemcpy(b + o, c->wpsi.p, 8 * W, hipMemcpyDeviceToHost)); o += 8 * W;
    HIPCHK(c, hipMemcpy(b + o, c->wsum.p, 24 * W, hipMemcpyDeviceToHost)); o += 24 * W;
    HIPCHK(c, hipMemcpy(b + o, c->cacc.p, class_acc_bytes(c), hipMemcpyDeviceToHost)); o += class_acc_bytes(c);
    HIPCHK(c, hipMemcpy(b + o, c->bad.p, 8, hipMemcpyDeviceToHost));
    return SCQMC_OK;
}

scqmc_status scqmc_load_state(scqmc_ctx *c, const void *buf, int64_t len) {
    if (!c || !buf) return SCQMC_E_INVALID_ARG;
    TRY(ready_for_walkers(c));
    if (len < 96) FAIL(c, SCQMC_E_INVALID_ARG, "state buffer too short");
    int64_t hdr[12];
    std::memcpy(hdr, buf, sizeof(hdr));
    if (hdr[0] != kMagic || hdr[1] != 2) FAIL(c, SCQMC_E_INVALID_ARG, "not a checkpoint of this format");
    if (hdr[3] != c->ncls || hdr[4] != c->N || hdr[5] != c->C || hdr[6] != c->A || hdr[7] != c->na ||
        hdr[8] != c->nb || hdr[11] != c->n_ref)
        FAIL(c, SCQMC_E_INVALID_ARG, "checkpoint from a different problem");
    int64_t W = hdr[2];
    if (W <= 0 || W >= (1LL << 31)) FAIL(c, SCQMC_E_INVALID_ARG, "bad walker count in checkpoint");
    c->W = W;
    c->ncg = class_groups(W);
    if (len < state_bytes(c)) FAIL(c, SCQMC_E_INVALID_ARG, "state buffer too short");
    const char *b = (const char *)buf;
    HIPCHK(c, hipSetDevice(c->device));
    TRY(dalloc(c, c->wkey, 8 * W));
    TRY(dalloc(c, c->wvirt, 4 * W));
    TRY(dalloc(c, c->worder, 4 * W));
    TRY(dalloc(c, c->wpsi, 8 * W));
    TRY(dalloc(c, c->wsum, 24 * W));
    TRY(dalloc(c, c->cacc, class_acc_bytes(c)));
    TRY(dalloc(c, c->bad, 8));
    TRY(dalloc(c, c->wftab, ftab_bytes(c) * W));
    int64_t o = 96;
    HIPCHK(c, hipMemcpy(c->wkey.p, b + o, 8 * W, hipMemcpyHostToDevice)); o += 8 * W;
    HIPCHK(c, hipMemcpy(c->wvirt.p, b + o, 4 * W, hipMemcpyHostToDevice)); o += ((4 * W + 7) / 8) * 8;
    HIPCHK(c, hipMemcpy(c->wpsi.p, b + o, 8 * W, hipMemcpyHostToDevice)); o += 8 * W;
    HIPCHK(c, hipMemcpy(c->wsum.p, b + o, 24 * W, hipMemcpyHostToDevice)); o += 24 * W;
    HIPCHK(c, hipMemcpy(c->cacc.p, b + o, class_acc_bytes(c), hipMemcpyHostToDevice)); o += class_acc_bytes(c);
    HIPCHK(c, hipMemcpy(c->bad.p, b + o, 8, hipMemcpyHostToDevice));
    c->step = hdr[9];
    c->seed = (unsigned long long)hdr[10];
    c->has_walkers = true;
    return SCQMC_OK;
}


// ---------------------------------------------------------------------------
// SC coefficient optimisation ("SC-MRCI(s)"): AMSGrad on the sampled gradient
// ---------------------------------------------------------------------------


static scqmc_status refresh_psi(scqmc_ctx *c) {
    DevProblem P = dev_problem(c);
    long long W = c->W;
    if (c->opt.precision == 1)
        hipLaunchKernelGGL(k_psi<float>, dim3(grid1(W, 64)), dim3(64), 0, c->stream, P,
                           c->wkey.as<unsigned long long>(), c->wvirt.as<unsigned>(), W, c->wpsi.as<double>());
    else
        hipLaunchKernelGGL(k_psi<double>, dim3(grid1(W, 64)), dim3(64), 0, c->stream, P,
                           c->wkey.as<unsigned long long>(), c->wvirt.as<unsigned>(), W, c->wpsi.as<double>());
    HIPCHK(c, hipGetLastError());
    std::vector<double> psi(W);
    HIPCHK(c, hipMemcpyAsync(psi.data(), c->wpsi.p, sizeof(double) * W, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (long long i = 0; i < W; i++)
        if (!(std::isfinite(psi[i]) && psi[i] != 0.0))
            FAIL(c, SCQMC_E_NUMERIC, "walker " + std::to_string(i) + " has psi = 0 or non-finite after an update");
    return SCQMC_OK;
}

scqmc_status scqmc_optimize(scqmc_ctx *c, const scqmc_amsgrad *o, int64_t n_iter, double *e_trace, double *g_trace) {
    if (!c || !o) return SCQMC_E_INVALID_ARG;
    if (!c->has_walkers) FAIL(c, SCQMC_E_STATE, "init_walkers first");
    if (c->opt.mode == 1 && !c->has_dyall) FAIL(c, SCQMC_E_STATE, "mode 1 needs set_dyall");
    if (n_iter < 0 || o->steps_per_iter <= 0 || o->equil_steps < 0 || !(o->lr > 0) || !(o->eps > 0) ||
        !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1))
        FAIL(c, SCQMC_E_INVALID_ARG, "bad AMSGrad parameters");
    long long need = (long long)n_iter * (o->steps_per_iter + o->equil_steps);
    if (c->step + need >= (1LL << 31)) FAIL(c, SCQMC_E_UNSUPPORTED, "step counter limit (2^31) reached");
    HIPCHK(c, hipSetDevice(c->device));
    TRY(ensure_f32(c));
    long long n = c->ncls;
    if ((long long)c->am_m.size() != n) {
        c->am_m.assign(n, 0.0);
        c->am_v.assign(n, 0.0);
        c->am_vmax.assign(n, 0.0);
    }
    const long long never = (1LL << 62);
    for (long long it = 0; it < n_iter; it++) {
        TRY(refresh_psi(c));
        if (o->equil_steps > 0) TRY(launch_sample(c, o->equil_steps, never));
        HIPCHK(c, hipMemsetAsync(c->wsum.p, 0, sizeof(double) * 3 * c->W, c->stream));
        HIPCHK(c, hipMemsetAsync(c->cacc.p, 0, class_acc_bytes(c), c->stream));
        TRY(launch_sample(c, o->steps_per_iter, 0));
        std::vector<double> ws, cs;
        TRY(download_sums(c, ws, cs));
        double St = 0, Ste = 0;
        for (long long l = 0; l < n; l++) { St += cs[l]; Ste += cs[n + l]; }
        if (!(St > 0)) FAIL(c, SCQMC_E_NUMERIC, "no residence time sampled");
        double E = Ste / St, g2 = 0;
        for (long long l = 1; l < n; l++) {
            double cl = c->ccls_h[l];
            if (cl == 0.0) continue;
            double g = (cs[n + l] - E * cs[l]) / (cl * St);
            g2 += g * g;
            double &m = c->am_m[l], &v = c->am_v[l], &vm = c->am_vmax[l];
            m = o->beta1 * m + (1 - o->beta1) * g;
            v = o->beta2 * v + (1 - o->beta2) * g * g;
            vm = std::max(vm, v);
            c->ccls_h[l] = cl - o->lr * m / (std::sqrt(vm) + o->eps);
            if (c->ccls_h[l] == 0.0) c->ccls_h[l] = cl;   // a class never gets switched off
        }
        if (!all_finite(c->ccls_h.data(), n)) FAIL(c, SCQMC_E_NUMERIC, "non-finite coefficient after an update");
        HIPCHK(c, hipMemcpyAsync(c->ccls.p, c->ccls_h.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        if (e_trace) e_trace[it] = E;
        if (g_trace) g_trace[it] = std::sqrt(g2);
    }
    TRY(refresh_psi(c));
    return SCQMC_OK;
}

scqmc_status scqmc_read_sc_coeffs(scqmc_ctx *c, double *c0, double *c_cls, int64_t n) {
    if (!c) return SCQMC_E_INVALID_ARG;
    if (!c->has_coef) FAIL(c, SCQMC_E_STATE, "set_sc_coeffs first");
    if (n != c->ncls - 1) FAIL(c, SCQMC_E_INVALID_ARG, "n must equal n_classes - 1");
    if (c0) *c0 = c->ccls_h[0];
    if (c_cls) for (long long i = 0; i < n; i++) c_cls[i] = c->ccls_h[i + 1];
    return SCQMC_OK;
}


// ---------------------------------------------------------------------------
// Batched form: several contexts (systems) walked by one launch
// ---------------------------------------------------------------------------
}  // extern "C"

struct scqmc_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<scqmc_ctx *> ctx;
    int precision = 0;
    int order = 0;          // 0: system by system, 1: walkers interleaved, 2: costliest systems first
    int spl = 1;            // steps per launch
    int bin = 0;            // 0: hardware dispatch of the slots; >= 1: persistent grid, work items of bin slots
    int ncu = 0;            // compute units of the device (persistent grid size)
    int wpg = 1;            // walkers (waves) per workgroup of the hardware-dispatched launch: 1, 2, 4
    int wps = 4;            // minimum waves per SIMD the kernel is compiled for: 3, 4, 5 (wpg 1 only)
    long long nslots = 0;
    std::vector<long long> Ws;
    int sched_order = -1;
    DBuf dsys, dslot_sys, dslot_w;
    DBuf dhead;             // work counter of the persistent form (zero between launches)
    size_t lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_spl = 0, graph_bin = -1, graph_wpg = 0, graph_wps = 0;
    long long graph_slots = -1;
};

namespace {
#define BFAIL(b, code, msg)        \
    do {                           \
        (b)->err = (msg);          \
        return (code);             \
    } while (0)
#define BHIP(b, call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (b)->err = std::string(#call) + ": " + hipGetErrorString(e_);              \
            return e_ == hipErrorOutOfMemory ? SCQMC_E_OOM : SCQMC_E_DEVICE;           \
        }                                                                              \
    } while (0)

// relative cost of one walker-step of a system: neighbours ~ (electrons x
// orbitals)^2 of the non-core space
double batch_cost(const scqmc_ctx *c) {
    double e = c->nea + c->neb, o = 2.0 * c->Np;
    return e * e * o * o;
}

void free_graph(scqmc_batch *b) {
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_spl = 0;
}

scqmc_status batch_schedule(scqmc_batch *b) {
    int n = (int)b->ctx.size();
    std::vector<long long> Ws(n);
    long long tot = 0;
    for (int i = 0; i < n; i++) { Ws[i] = b->ctx[i]->W; tot += Ws[i]; }
    if (Ws == b->Ws && b->sched_order == b->order) return SCQMC_OK;
    if (tot >= (1LL << 31)) BFAIL(b, SCQMC_E_UNSUPPORTED, "too many walkers in one batch");
    std::vector<int> ss, ww;
    ss.reserve(tot);
    ww.reserve(tot);
    std::vector<int> sys_order(n);
    for (int i = 0; i < n; i++) sys_order[i] = i;
    if (b->order == 2)
        std::stable_sort(sys_order.begin(), sys_order.end(),
                         [&](int x, int y) { return batch_cost(b->ctx[x]) > batch_cost(b->ctx[y]); });
    if (b->order == 1) {
        long long mx = *std::max_element(Ws.begin(), Ws.end());
        for (long long w = 0; w < mx; w++)
            for (int i = 0; i < n; i++)
                if (w < Ws[i]) { ss.push_back(i); ww.push_back((int)w); }
    } else {
        for (int i : sys_order)
            for (long long w = 0; w < Ws[i]; w++) { ss.push_back(i); ww.push_back((int)w); }
    }
    hipError_t e1 = hipSuccess;
    b->dslot_sys.release();
    b->dslot_w.release();
    e1 = hipMalloc(&b->dslot_sys.p, sizeof(int) * tot);
    if (e1 == hipSuccess) e1 = hipMalloc(&b->dslot_w.p, sizeof(int) * tot);
    if (e1 != hipSuccess) BFAIL(b, SCQMC_E_OOM, "schedule arrays");
    b->dslot_sys.n = b->dslot_w.n = sizeof(int) * tot;
    BHIP(b, hipMemcpy(b->dslot_sys.p, ss.data(), sizeof(int) * tot, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->dslot_w.p, ww.data(), sizeof(int) * tot, hipMemcpyHostToDevice));
    b->nslots = tot;
    b->Ws = Ws;
    b->sched_order = b->order;
    free_graph(b);
    return SCQMC_OK;
}

scqmc_status batch_upload(scqmc_batch *b) {
    int n = (int)b->ctx.size();
    std::vector<BatchSys> hs(n);
    int NLmax = 1;
    for (int i = 0; i < n; i++) {
        scqmc_ctx *c = b->ctx[i];
        if (!c->has_walkers) BFAIL(b, SCQMC_E_STATE, "context " + std::to_string(i) + " has no walkers");
        if (c->opt.precision != b->precision) BFAIL(b, SCQMC_E_INVALID_ARG, "contexts differ in precision");
        if (c->opt.mode == 1 && !c->has_dyall) BFAIL(b, SCQMC_E_STATE, "mode 1 needs set_dyall");
        scqmc_status st = ensure_f32(c);
        if (st != SCQMC_OK) BFAIL(b, st, c->err);
        BatchSys &B = hs[i];
        std::memset(&B, 0, sizeof(B));
        B.P = dev_problem(c);
        B.S.key = c->wkey.as<unsigned long long>();
        B.S.virt = c->wvirt.as<unsigned>();
        B.S.psi = c->wpsi.as<double>();
        B.S.wsum = c->wsum.as<double>();
        B.S.cacc = c->cacc.as<unsigned long long>();
        B.S.ncg = (int)c->ncg;
        B.S.bad = c->bad.as<unsigned long long>();
        B.S.ftab = c->wftab.as<double>();
        B.order = c->worder.as<int>();
        B.W = c->W;
        B.step0 = c->step;
        B.burn_in = c->opt.burn_in;
        B.NL = lists_per_group(c);
        NLmax = std::max(NLmax, B.NL);
        if (c->step >= (1LL << 31) - (1LL << 20)) BFAIL(b, SCQMC_E_UNSUPPORTED, "step counter limit");
    }
    for (int i = 0; i < n; i++) BHIP(b, hipStreamSynchronize(b->ctx[i]->stream));
    if (b->dsys.n < sizeof(BatchSys) * n) {
        b->dsys.release();
        if (hipMalloc(&b->dsys.p, sizeof(BatchSys) * n) != hipSuccess) BFAIL(b, SCQMC_E_OOM, "batch descriptors");
        b->dsys.n = sizeof(BatchSys) * n;
        free_graph(b);
    }
    BHIP(b, hipMemcpy(b->dsys.p, hs.data(), sizeof(BatchSys) * n, hipMemcpyHostToDevice));
    if (!b->dhead.p) {
        if (hipMalloc(&b->dhead.p, sizeof(unsigned)) != hipSuccess) BFAIL(b, SCQMC_E_OOM, "work counter");
        b->dhead.n = sizeof(unsigned);
        BHIP(b, hipMemset(b->dhead.p, 0, sizeof(unsigned)));
        BHIP(b, hipDeviceSynchronize());
    }
    b->lds = wave_lds_bytes(NLmax);   // per wave; a workgroup of wpg walkers takes wpg times this
    return SCQMC_OK;
}

// the hardware-dispatched batch kernel for (precision, walkers per workgroup,
// waves per SIMD); FP32 has the default variant only
using BatchKernel = void (*)(const BatchSys *, const int *, const int *, long long, int, unsigned);
static BatchKernel batch_kernel(int precision, int wpg, int wps) {
    if (precision == 1) return (wpg == 1 && wps == 4) ? k_sample_batch<float, 1, 4> : nullptr;
    if (wps == 4) {
        if (wpg == 1) return k_sample_batch<double, 1, 4>;
        if (wpg == 2) return k_sample_batch<double, 2, 4>;
        if (wpg == 4) return k_sample_batch<double, 4, 4>;
        return nullptr;
    }
    if (wpg != 1) return nullptr;
    if (wps == 3) return k_sample_batch<double, 1, 3>;
    if (wps == 5) return k_sample_batch<double, 1, 5>;
    return nullptr;
}

scqmc_status batch_launch(scqmc_batch *b, int nsteps) {
    int n = (int)b->ctx.size();
    if (b->bin > 0) {
        dim3 blk(64);
        // persistent grid: sixteen workgroups (four waves per SIMD) per compute unit
        long long items = (b->nslots + b->bin - 1) / b->bin;
        long long g = std::min<long long>(items, 16LL * std::max(1, b->ncu));
        hipLaunchKernelGGL(k_order_batch, dim3(n), dim3(1024), 0, b->stream, b->dsys.as<const BatchSys>());
        if (b->precision == 1)
            hipLaunchKernelGGL(k_sample_batch_queue<float>, dim3((unsigned)g), blk, b->lds, b->stream,
                               b->dsys.as<const BatchSys>(), b->dslot_sys.as<const int>(), b->dslot_w.as<const int>(),
                               b->nslots, nsteps, b->dhead.as<unsigned>(), b->bin);
        else
            hipLaunchKernelGGL(k_sample_batch_queue<double>, dim3((unsigned)g), blk, b->lds, b->stream,
                               b->dsys.as<const BatchSys>(), b->dslot_sys.as<const int>(), b->dslot_w.as<const int>(),
                               b->nslots, nsteps, b->dhead.as<unsigned>(), b->bin);
        hipLaunchKernelGGL(k_batch_advance, dim3(grid1(n, 64)), dim3(64), 0, b->stream, b->dsys.as<BatchSys>(), n,
                           nsteps, b->dhead.as<unsigned>());
        BHIP(b, hipGetLastError());
        return SCQMC_OK;
    }
    BatchKernel kern = batch_kernel(b->precision, b->wpg, b->wps);
    if (!kern) BFAIL(b, SCQMC_E_UNSUPPORTED, "no batch kernel for this precision / walkers per workgroup / waves");
    dim3 grid(grid1(b->nslots, b->wpg)), blk(64 * b->wpg);
    hipLaunchKernelGGL(k_order_batch, dim3(n), dim3(1024), 0, b->stream, b->dsys.as<const BatchSys>());
    hipLaunchKernelGGL(kern, grid, blk, b->lds * b->wpg, b->stream, b->dsys.as<const BatchSys>(),
                       b->dslot_sys.as<const int>(), b->dslot_w.as<const int>(), b->nslots, nsteps,
                       (unsigned)b->lds);
    hipLaunchKernelGGL(k_batch_advance, dim3(grid1(n, 64)), dim3(64), 0, b->stream, b->dsys.as<BatchSys>(), n, nsteps,
                       (unsigned *)nullptr);
    BHIP(b, hipGetLastError());
    return SCQMC_OK;
}

// one graph per (steps per launch, schedule): a batched launch and the step
// advance, replayed as many times as needed
scqmc_status batch_graph(scqmc_batch *b) {
    if (b->gexec && b->graph_spl == b->spl && b->graph_slots == b->nslots && b->graph_bin == b->bin &&
        b->graph_wpg == b->wpg && b->graph_wps == b->wps)
        return SCQMC_OK;
    free_graph(b);
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    scqmc_status st = batch_launch(b, b->spl);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != SCQMC_OK) { if (g) hipGraphDestroy(g); return st; }
    if (e != hipSuccess) BFAIL(b, SCQMC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    b->graph = g;
    BHIP(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    b->graph_spl = b->spl;
    b->graph_slots = b->nslots;
    b->graph_bin = b->bin;
    b->graph_wpg = b->wpg;
    b->graph_wps = b->wps;
    return SCQMC_OK;
}

scqmc_status batch_run(scqmc_batch *b, long long n_steps) {
    if (n_steps <= 0) return SCQMC_OK;
    scqmc_status st = batch_schedule(b);
    if (st != SCQMC_OK) return st;
    st = batch_upload(b);
    if (st != SCQMC_OK) return st;
    long long full = n_steps / b->spl, rest = n_steps % b->spl;
    if (full > 0) {
        st = batch_graph(b);
        if (st != SCQMC_OK) return st;
        for (long long i = 0; i < full; i++) BHIP(b, hipGraphLaunch(b->gexec, b->stream));
    }
    if (rest > 0) {
        st = batch_launch(b, (int)rest);
        if (st != SCQMC_OK) return st;
    }
    BHIP(b, hipStreamSynchronize(b->stream));
    for (scqmc_ctx *c : b->ctx) c->step += n_steps;
    return SCQMC_OK;
}
}  // namespace

extern "C" {

scqmc_status scqmc_batch_create(scqmc_ctx *const *ctxs, int32_t n, scqmc_batch **out) {
    if (!out || !ctxs || n <= 0) return SCQMC_E_INVALID_ARG;
    *out = nullptr;
    int dev = ctxs[0] ? ctxs[0]->device : 0;
    for (int i = 0; i < n; i++) {
        if (!ctxs[i]) return SCQMC_E_INVALID_ARG;
        if (ctxs[i]->device != dev) return SCQMC_E_INVALID_ARG;
        for (int j = 0; j < i; j++)
            if (ctxs[j] == ctxs[i]) return SCQMC_E_INVALID_ARG;
    }
    scqmc_batch *b = new (std::nothrow) scqmc_batch();
    if (!b) return SCQMC_E_OOM;
    b->device = dev;
    b->ctx.assign(ctxs, ctxs + n);
    b->precision = ctxs[0]->opt.precision;
    if (hipSetDevice(dev) != hipSuccess || hipStreamCreate(&b->stream) != hipSuccess ||
        hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        if (b->stream) hipStreamDestroy(b->stream);
        delete b;
        return SCQMC_E_DEVICE;
    }
    *out = b;
    return SCQMC_OK;
}

void scqmc_batch_destroy(scqmc_batch *b) {
    if (!b) return;
    hipSetDevice(b->device);
    if (b->stream) hipStreamSynchronize(b->stream);
    free_graph(b);
    b->dsys.release();
    b->dslot_sys.release();
    b->dslot_w.release();
    b->dhead.release();
    if (b->stream) hipStreamDestroy(b->stream);
    delete b;
}

const char *scqmc_batch_last_error(const scqmc_batch *b) { return b ? b->err.c_str() : "null batch"; }

scqmc_status scqmc_batch_sample(scqmc_batch *b, int64_t n_steps) {
    if (!b) return SCQMC_E_INVALID_ARG;
    if (n_steps < 0) BFAIL(b, SCQMC_E_INVALID_ARG, "negative n_steps");
    BHIP(b, hipSetDevice(b->device));
    b->precision = b->ctx[0]->opt.precision;
    return batch_run(b, n_steps);
}

scqmc_status scqmc_batch_tune(scqmc_batch *b, int64_t trial_steps, int32_t *order, int32_t *steps_per_launch,
                              int32_t *bin, double *ms_per_step) {
    if (!b) return SCQMC_E_INVALID_ARG;
    if (trial_steps <= 0) BFAIL(b, SCQMC_E_INVALID_ARG, "trial_steps must be positive");
    BHIP(b, hipSetDevice(b->device));
    b->precision = b->ctx[0]->opt.precision;
    const int orders[3] = {0, 1, 2}, spls[3] = {1, 2, 4}, bins[3] = {0, 1, 4};
    double best = 1e300;
    b->wpg = 1;
    b->wps = 4;
    int bo = 0, bs = 1, bb = 0;
    for (int o : orders)
        for (int sp : spls)
            for (int bn : bins) {
                b->order = o;
                b->spl = sp;
                b->bin = bn;
                long long nst = ((trial_steps + sp - 1) / sp) * sp;
                // untimed first call builds the schedule and the graph
                scqmc_status st = batch_run(b, sp);
                if (st != SCQMC_OK) return st;
                auto t0 = std::chrono::steady_clock::now();
                st = batch_run(b, nst);
                if (st != SCQMC_OK) return st;
                double ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / nst;
                if (ms < best) { best = ms; bo = o; bs = sp; bb = bn; }
            }
    b->order = bo;
    b->spl = bs;
    b->bin = bb;
    // second phase, hardware hand-out only: walkers per workgroup and the
    // waves-per-SIMD register budget of the kernel (FP64; the precision form
    // has the default variant only)
    int bw = 1, bv = 4;
    if (bb == 0 && b->precision == 0) {
        const int kv[4][2] = {{2, 4}, {4, 4}, {1, 3}, {1, 5}};
        for (const auto &k : kv) {
            b->wpg = k[0];
            b->wps = k[1];
            long long nst = ((trial_steps + bs - 1) / bs) * bs;
            scqmc_status st = batch_run(b, bs);
            if (st != SCQMC_OK) return st;
            auto t0 = std::chrono::steady_clock::now();
            st = batch_run(b, nst);
            if (st != SCQMC_OK) return st;
            double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / nst;
            if (ms < best) { best = ms; bw = k[0]; bv = k[1]; }
        }
    }
    b->wpg = bw;
    b->wps = bv;
    if (order) *order = bo;
    if (steps_per_launch) *steps_per_launch = bs;
    if (bin) *bin = bb;
    if (ms_per_step) *ms_per_step = best;
    return SCQMC_OK;
}

scqmc_status scqmc_batch_set_schedule(scqmc_batch *b, int32_t order, int32_t steps_per_launch) {
    if (!b) return SCQMC_E_INVALID_ARG;
    if (order < 0 || order > 2 || steps_per_launch < 1 || steps_per_launch > 1024)
        BFAIL(b, SCQMC_E_INVALID_ARG, "order must be 0..2, steps_per_launch 1..1024");
    b->order = order;
    b->spl = steps_per_launch;
    return SCQMC_OK;
}

scqmc_status scqmc_batch_set_kernel(scqmc_batch *b, int32_t walkers_per_group, int32_t waves_per_simd) {
    if (!b) return SCQMC_E_INVALID_ARG;
    if (!batch_kernel(0, walkers_per_group, waves_per_simd))
        BFAIL(b, SCQMC_E_INVALID_ARG, "supported: (1, 3), (1, 4), (1, 5), (2, 4), (4, 4)");
    b->wpg = walkers_per_group;
    b->wps = waves_per_simd;
    return SCQMC_OK;
}

scqmc_status scqmc_batch_get_kernel(const scqmc_batch *b, int32_t *walkers_per_group, int32_t *waves_per_simd) {
    if (!b) return SCQMC_E_INVALID_ARG;
    if (walkers_per_group) *walkers_per_group = b->wpg;
    if (waves_per_simd) *waves_per_simd = b->wps;
    return SCQMC_OK;
}

scqmc_status scqmc_batch_set_queue(scqmc_batch *b, int32_t bin) {
    if (!b) return SCQMC_E_INVALID_ARG;
    if (bin < 0 || bin > 4096) BFAIL(b, SCQMC_E_INVALID_ARG, "bin must be 0..4096");
    b->bin = bin;
    return SCQMC_OK;
}

}  // extern "C"

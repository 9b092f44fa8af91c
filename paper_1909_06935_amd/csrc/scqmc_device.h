// scqmc_device.h -- device-side data structures and helpers of the gfx950
// local-energy engine (stochastic SC-MRCI / SC-NEVPT2, arXiv:1909.06935).
//
// Internal representation
//   * non-core spin-orbital g = sigma * Np + idx, idx in [0, Np) with
//     Np = A + V (active orbitals first, then virtual); g order = the
//     determinant's creation-operator order restricted to non-core orbitals
//     (all alpha, then all beta).  Core orbitals are always doubly occupied
//     and contribute only through the folded one-body operator and E_core.
//   * active code c = sigma * 32 + t (t in [0, A)): bit c of a 64-bit key.
//   * virtual code s = sigma * V + a: class labels (the subspaces S_l^(k) of
//     the paper's Theory section).
//   * a walker is (active key, packed virtual codes): two 16-bit codes,
//     ascending, 0xFFFF when absent.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SCQ_EMPTY_KEY 0xFFFFFFFFFFFFFFFFull
#define SCQ_NOVIRT 0xFFFFu

// Hash table of the reference: open addressing, 16-byte slots.  In the
// determinant table (key = active occupation) slot.y holds the coefficient
// itself; in the one- / two-electron-removed tables slot.y = count << 32 |
// offset of the key's list in `ents`.  A list entry is one 16-byte record:
// the reference coefficient times the parity of removing the electron(s) from
// that reference determinant, and the code of the removed electron(s) (t, or
// t << 6 | u) -- one load per entry, and a short list in one cache line.
struct __attribute__((aligned(16))) ListEnt {
    double val;
    unsigned code, pad;
};

struct DevTable {
    const ulonglong2 *slots;         // [cap]: .x key (SCQ_EMPTY_KEY = free)
    const ListEnt *ents;             // list entries (removed-electron tables only)
    unsigned long long mask;         // cap - 1 (cap a power of two)
};

struct DevProblem {
    int A, V, Np;           // active, virtual, non-core orbital counts
    int nea, neb;           // active-space electrons per spin (n_elec - n_core)
    int mode;               // 0: E_L; 1: + Dyall local energy
    int active_only;        // 1: only active-space neighbours (reference properties)
    long long ncls;         // number of classes
    double e_core;          // e_const + core energy
    double eps_screen;      // doubles with |<rs||pq>| <= eps are left out (0: keep all)
    const double *heff;     // [Np*Np] core-folded one-body operator
    const double *eri;      // [Np^4] (pq|rs) over non-core orbitals
    const float *heff32;    // FP32 copies for the precision form (null in FP64 runs)
    const float *eri32;
    const double *ccls;     // [ncls] SC coefficients, c0 at index 0
    const double *eps;      // [V] Dyall virtual orbital energies (mode 1)
    DevTable ref, ytab, xtab;
    unsigned long long seed;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int popc32(uint32_t x) { return __popc(x); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// MurmurHash3 64-bit finaliser (Appleby), used as the table hash.
__device__ __forceinline__ unsigned long long scq_hash(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Open-addressing lookup (linear probing, one 16-byte load per probe).
// Returns the (offset, count) of the key's entry list, count 0 when absent.
__device__ __forceinline__ uint2 table_find(const DevTable &t, unsigned long long key) {
    unsigned m = (unsigned)t.mask;   // capacities stay below 2^32
    unsigned slot = (unsigned)scq_hash(key) & m;
    while (true) {
        ulonglong2 s = t.slots[slot];
        if (s.x == key) return make_uint2((unsigned)s.y, (unsigned)(s.y >> 32));
        if (s.x == SCQ_EMPTY_KEY) return make_uint2(0u, 0u);
        slot = (slot + 1u) & m;
    }
}

// coefficient phi0(key) from the determinant table (0 when absent)
__device__ __forceinline__ double ref_coef(const DevTable &t, unsigned long long key) {
    unsigned m = (unsigned)t.mask;
    unsigned slot = (unsigned)scq_hash(key) & m;
    while (true) {
        ulonglong2 s = t.slots[slot];
        if (s.x == key) return __longlong_as_double((long long)s.y);
        if (s.x == SCQ_EMPTY_KEY) return 0.0;
        slot = (slot + 1u) & m;
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
        c[0] = y0; c[1] = lo1; c[2] = y2; c[3] = lo0;
    }
}

// Exponential variate E = -log(U), U = (k+1) 2^-53, k = top 53 bits of the
// first two Philox words; counter (walker, step | level<<31, a, b).
__device__ __forceinline__ double exp_draw(unsigned long long seed, uint32_t walker, uint32_t step, uint32_t level,
                                           uint32_t a, uint32_t b) {
    uint32_t c[4] = {walker, (step & 0x7fffffffu) | (level << 31), a, b};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    unsigned long long k = ((((unsigned long long)c[0]) << 32) | (unsigned long long)c[1]) >> 11;
    double u = (double)(k + 1ull) * 0x1.0p-53;
    return -log(u);
}

__device__ __forceinline__ long long class_id1(int V, int s) { return 1 + s; }
__device__ __forceinline__ long long class_id2(int V, int s1, int s2) {
    long long V2 = 2LL * V;
    return 1 + V2 + (long long)s1 * V2 - (long long)s1 * (s1 + 1) / 2 + (s2 - s1 - 1);
}

// ---------------------------------------------------------------------------
// determinants over non-core spin-orbitals
// ---------------------------------------------------------------------------
#define SCQ_NOG 0x3fffffff   // absent virtual electron (compares above every spin-orbital)

struct NDet {           // occupation: active key + up to two virtual electrons (g codes, ascending)
    unsigned long long key;
    int nv;
    int vg[2];          // SCQ_NOG where absent; only constant indices are used (registers, no scratch)
};

__device__ __forceinline__ int g_of_active(const DevProblem &P, int c) { return (c >> 5) * P.Np + (c & 31); }
__device__ __forceinline__ int g_of_virtual(const DevProblem &P, int s) {
    int sg = s >= P.V;
    return sg * P.Np + P.A + (s - sg * P.V);
}
__device__ __forceinline__ int g_spin(const DevProblem &P, int g) { return g >= P.Np; }
__device__ __forceinline__ int g_idx(const DevProblem &P, int g) { return g >= P.Np ? g - P.Np : g; }

// number of occupied non-core spin-orbitals of d below g (creation order)
__device__ __forceinline__ int below(const DevProblem &P, const NDet &d, int g) {
    int sg = g >= P.Np;
    int idx = g - sg * P.Np;
    uint32_t act = (uint32_t)(d.key >> (32 * sg));
    int c = 0;
    if (sg) c += popc32((uint32_t)d.key) + (d.vg[0] < P.Np) + (d.vg[1] < P.Np);
    if (idx < P.A) {
        c += popc32(act & ((1u << idx) - 1u));
    } else {
        int lo = sg * P.Np;
        c += popc32(act) + (d.vg[0] >= lo && d.vg[0] < g) + (d.vg[1] >= lo && d.vg[1] < g);
    }
    return c;
}

// number of non-core occupied spin-orbitals of an active-space determinant
// (key) below active code c, in creation order (all alpha, then beta)
__device__ __forceinline__ int key_below(unsigned long long k, int c) {
    int sg = c >> 5, t = c & 31;
    unsigned mask = (1u << t) - 1u;
    return sg ? __popc((unsigned)k) + __popc((unsigned)(k >> 32) & mask) : __popc((unsigned)k & mask);
}

// sign of <m| a+_Q a_P |b>
__device__ __forceinline__ double phase_single(const DevProblem &P, const NDet &b, int gP, int gQ) {
    int e = below(P, b, gP) + below(P, b, gQ) - (gP < gQ ? 1 : 0);
    return (e & 1) ? -1.0 : 1.0;
}
// sign of <m| a+_Q1 a+_Q2 a_P2 a_P1 |b>, P1 < P2 removed from b, Q1 < Q2 added
__device__ __forceinline__ double phase_double(const DevProblem &P, const NDet &b, int P1, int P2, int Q1, int Q2) {
    int e = below(P, b, P1);
    e += below(P, b, P2) - (P1 < P2);
    e += below(P, b, Q2) - (P1 < Q2) - (P2 < Q2);
    e += below(P, b, Q1) - (P1 < Q1) - (P2 < Q1) + (Q2 < Q1);
    return (e & 1) ? -1.0 : 1.0;
}

// Integral storage of the two forms of the walk: FP64 (R = double) or the
// precision form, whose off-diagonal Slater-Condon terms are computed in
// FP32 (R = float) from FP32 copies and added to FP64 sums.
template <class R> struct Ints;
template <> struct Ints<double> {
    static __device__ __forceinline__ const double *eri(const DevProblem &P) { return P.eri; }
    static __device__ __forceinline__ const double *heff(const DevProblem &P) { return P.heff; }
};
template <> struct Ints<float> {
    static __device__ __forceinline__ const float *eri(const DevProblem &P) { return P.eri32; }
    static __device__ __forceinline__ const float *heff(const DevProblem &P) { return P.heff32; }
};

// (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq): the element is read at the
// permutation that puts the largest orbital index last.  Virtual orbitals
// carry the largest indices and are what varies from lane to lane (the rows
// of a group differ in their virtual electrons), so neighbouring lanes read
// neighbouring addresses and the block actually touched (e.g. (t a|u b) with
// t, u active) stays compact instead of one cache line per element.
// Integral indices are formed with 24-bit multiplies (full rate on the vector
// unit, where a 32-bit multiply takes four passes): with at most 128
// non-core orbitals (the space check of the set-up) every factor is below
// 2^24 and every index below 2^28.
template <class R = double>
__device__ __forceinline__ R eri4(const DevProblem &P, int p, int q, int r, int s) {
    unsigned Np = (unsigned)P.Np;
    int mpq = max(p, q), mrs = max(r, s);
    int a = p, b = q, c = r, d = s;
    if (mpq > mrs) { a = r; b = s; c = p; d = q; }
    int lo = min(c, d), hi = max(c, d);
    return Ints<R>::eri(P)[__umul24(__umul24(__umul24((unsigned)a, Np) + (unsigned)b, Np) + (unsigned)lo, Np) + (unsigned)hi];
}
// spin-orbital chemist integral (PQ|RS)
template <class R = double>
__device__ __forceinline__ R seri(const DevProblem &P, int gP, int gQ, int gR, int gS) {
    if (g_spin(P, gP) != g_spin(P, gQ) || g_spin(P, gR) != g_spin(P, gS)) return R(0);
    return eri4<R>(P, g_idx(P, gP), g_idx(P, gQ), g_idx(P, gR), g_idx(P, gS));
}
// <Q1 Q2 || P1 P2> piece of a double: (Q1 P1|Q2 P2) - (Q1 P2|Q2 P1)
template <class R = double>
__device__ __forceinline__ R double_elem(const DevProblem &P, int P1, int P2, int Q1, int Q2) {
    return seri<R>(P, Q1, P1, Q2, P2) - seri<R>(P, Q1, P2, Q2, P1);
}
// The same with a lane-varying added spin-orbital X (X = Q1 or Q2; the virtual
// that differs between the rows a wave evaluates side by side), Y the other
// added one: with PX / PY the removed partners of X / Y in the first term,
//   (Q1 P1|Q2 P2) = (Y PY|X PX) at [Y][PY][PX][X],
//   (Q1 P2|Q2 P1) = (Y PX|X PY) at [Y][PX][PY][X],
// so X is the last index of both reads and the lanes of a load share lines
// whatever the order of X and the other indices.
template <class R = double>
__device__ __forceinline__ R double_elem_x(const DevProblem &P, int P1, int P2, int Q1, int Q2, bool x_is_q2) {
    int X = x_is_q2 ? Q2 : Q1, Y = x_is_q2 ? Q1 : Q2;
    int PX = x_is_q2 ? P2 : P1, PY = x_is_q2 ? P1 : P2;
    int sx = g_spin(P, X), sy = g_spin(P, Y), spx = g_spin(P, PX), spy = g_spin(P, PY);
    unsigned Np = (unsigned)P.Np;
    unsigned x = (unsigned)g_idx(P, X), y = (unsigned)g_idx(P, Y), px = (unsigned)g_idx(P, PX),
             py = (unsigned)g_idx(P, PY);
    const R *E = Ints<R>::eri(P);
    R a = (sy == spy && sx == spx) ? E[__umul24(__umul24(__umul24(y, Np) + py, Np) + px, Np) + x] : R(0);
    R b = (sy == spx && sx == spy) ? E[__umul24(__umul24(__umul24(y, Np) + px, Np) + py, Np) + x] : R(0);
    return a - b;
}

// one-body part of a single P -> Q from determinant b:
// h_eff[Q][P] + sum_{J in b, J != P} [(QP|JJ) - (QJ|JP)]; with_virt = 0 drops
// the virtual electrons from the sum (Dyall's H_0 acts on the active space only)
template <class R = double>
__device__ __forceinline__ double single_elem(const DevProblem &P, const NDet &b, int gP, int gQ, bool with_virt) {
    int p = g_idx(P, gP), q = g_idx(P, gQ), sp = g_spin(P, gP);
    double v = (double)Ints<R>::heff(P)[q * P.Np + p];
    for (int s = 0; s < 2; s++) {
        uint32_t act = (uint32_t)(b.key >> (32 * s));
        while (act) {
            int t = __ffs(act) - 1;
            act &= act - 1u;
            int gJ = s * P.Np + t;
            if (gJ == gP) continue;
            // (qp|jj) = (jj|pq) and (qj|jp) = (pj|jq): the lane-varying index goes last
            R J = eri4<R>(P, t, t, p, q);
            R K = (s == sp) ? eri4<R>(P, p, t, t, q) : R(0);
            v += (double)(J - K);
        }
    }
    if (with_virt) {
#pragma unroll
        for (int i = 0; i < 2; i++) {
            if (i >= b.nv) break;
            int gJ = b.vg[i];
            if (gJ == gP) continue;
            int j = g_idx(P, gJ), s = g_spin(P, gJ);
            R J = eri4<R>(P, j, j, p, q);
            R K = (s == sp) ? eri4<R>(P, p, j, j, q) : R(0);
            v += (double)(J - K);
        }
    }
    return v;
}

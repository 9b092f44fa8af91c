// scqmc_walk.hip -- the hot path: one continuous-time step of every walker
// (local energy of eq:locE with the overlaps of eq:ovlp, the rates and move of
// the rejection-free walk of "SC-MRCI(s)", the Dyall local energy of eq:nevpt).
//
// Layout: one wave64 per walker.  The neighbours m of walker n are grouped by
// their active part x_m = x_n - Ra + Pa (Ra: up to two removed active
// spin-orbitals, Pa: up to two added).  Members of a group differ only in the
// virtual occupation l_m, i.e. the SC class.  Groups are swept in "blocks"
// fixed by the spin kinds of Ra and Pa (none, a, b, aa, ab, bb each): inside a
// block every group has the same R rows (virtual sets reachable by at most a
// double excitation), in the same order, and the same overlap type.
//   * 64 groups at a time, one per lane: decode (Ra, Pa), form x_m and do the
//     group's reference-table lookups once
//        l_m empty      : phi0(x_m)                       (reference table)
//        one virtual    : y-list of x_m, x-lists of x_m - r for each electron r
//        two virtuals   : x-list of x_m
//     (a y-list / x-list holds the reference determinants a determinant with
//     one / two active electrons removed came from, with their coefficients
//     pre-multiplied by the parity of that removal);
//   * every group is given a sub-wave of S = 2^k >= min(R, 64) lanes; a lane's
//     row index is the same for every group of the block, so its row decode
//     (virtual set, class, SC coefficient) is done once per block (per 64-row
//     tile when R > 64) and reused for every group;
//   * a row costs H_nm (Slater-Condon, phase from a per-walker LDS table) and
//     psi(m) = c_l <m|H|phi0> summed over the group's lists, i.e. over nonzero
//     reference terms only; per-group rate sums are sub-wave reductions in a
//     fixed order.
// The next state: first-reaction method at two levels (exponential clocks keyed
// by (walker, step, x_m), then by (walker, step, class)) -- independent of the
// visiting order.
#include "scqmc_device.h"

#define WAVE 64
// One walker (wave) per workgroup: walkers differ widely in cost (an
// active-space walker has several times the neighbours of a two-virtual one)
// and a workgroup holds its LDS and registers until its last wave ends, so
// single-wave workgroups return their slot as soon as their walker is done.
#define WPB 1

// wave-uniform values: keep them in scalar registers
__device__ __forceinline__ unsigned uni(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uni(unsigned long long v) {
    return ((unsigned long long)uni((unsigned)(v >> 32)) << 32) | (unsigned long long)uni((unsigned)v);
}
__device__ __forceinline__ double uni(double v) {
    return __longlong_as_double((long long)uni((unsigned long long)__double_as_longlong(v)));
}

struct GroupInfo {
    unsigned long long xkey;
    double phi;           // phi0(x_m) for groups without virtual electrons
    double gam;           // sum over rows of |psi(m)|
    short rg[2], pg[2];   // removed / added active spin-orbitals (g codes, -1 if absent)
    int nl;               // one virtual electron: nonempty x-lists stored after the y-list
    int live;             // some row of the group can have psi(m) != 0
};

// Read-only table and integral loads.  With a wave-uniform index (U) they go
// through the constant address space, so the compiler issues scalar loads;
// otherwise plain vector loads.  Nothing a launch reads this way is written
// during the launch.
template <bool U, class T>
__device__ __forceinline__ T tload(const T *p, unsigned i) {
    if (U) return ((const __attribute__((address_space(4))) T *)p)[i];
    return p[i];
}

// a list entry (16 bytes): scalar loads of its two fields when the index is
// wave-uniform, one 16-byte vector load otherwise
template <bool U>
__device__ __forceinline__ ListEnt ent_load(const ListEnt *p, unsigned i) {
    ListEnt e;
    if (U) {
        const __attribute__((address_space(4))) double *v = (const __attribute__((address_space(4))) double *)(p + i);
        const __attribute__((address_space(4))) unsigned *c =
            (const __attribute__((address_space(4))) unsigned *)(p + i);
        e.val = v[0];
        e.code = c[2];
        e.pad = 0u;
    } else {
        e = p[i];
    }
    return e;
}

// The entries of a wave-uniform group's list, one per lane (lane j holds
// entry j), loaded by one vector load with every lane active; the overlap
// loops then take them with readlane instead of a scalar load per entry.
// n = ~0: the list is short (fewer than four entries) or longer than 64, and
// its entries are read with scalar loads.
struct VecEnts {
    double val;
    unsigned code;
    unsigned n;   // entries in the lanes (~0: none loaded)
};
__device__ __forceinline__ VecEnts vec_ents_off() {
    VecEnts v;
    v.val = 0.0;
    v.code = 0u;
    v.n = ~0u;
    return v;
}
// call with every lane of the wave active (ox wave-uniform)
__device__ __forceinline__ VecEnts vec_ents_load(const ListEnt *ents, uint2 ox, int lane) {
    VecEnts v = vec_ents_off();
    if (ox.y < 4u) return v;   // short lists: scalar loads cost less than the broadcast
    v.n = ox.y;
    if ((unsigned)lane < ox.y && ox.y <= 64u) {
        v.val = ents[ox.x + lane].val;
        v.code = ents[ox.x + lane].code;
    }
    return v;
}
__device__ __forceinline__ double readlane_d(double x, unsigned l) {
    long long b = __double_as_longlong(x);
    int lo = __builtin_amdgcn_readlane((int)b, (int)l), hi = __builtin_amdgcn_readlane((int)(b >> 32), (int)l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

struct WaveLDS {
    GroupInfo *G;          // [65]; slot 64 holds the selected group
    uint2 *lst;            // [65 * NL]
    unsigned char *occ;    // [2][32] active occupied codes per spin
    unsigned char *hol;    // [2][32] active holes per spin
    short *wg;             // [72] g codes of the walker's occupied non-core spin-orbitals (active, then virtual)
    unsigned char *bw;     // [256] electrons of the walker below each non-core spin-orbital g (phases)
    unsigned char *perm;   // [64] live groups of the current 64, in order
    int NL;
};

__host__ __device__ inline size_t wave_lds_bytes(int NL) {
    size_t b = 65 * sizeof(GroupInfo) + 65 * (size_t)NL * sizeof(uint2) + 128 + 72 * sizeof(short) + 256 + 64;
    return (b + 15) & ~(size_t)15;
}

__device__ inline WaveLDS carve(unsigned char *base, int NL) {
    WaveLDS L;
    L.G = (GroupInfo *)base;
    L.lst = (uint2 *)(base + 65 * sizeof(GroupInfo));
    L.occ = (unsigned char *)(L.lst + 65 * NL);
    L.hol = L.occ + 64;
    L.wg = (short *)(L.hol + 64);
    L.bw = (unsigned char *)(L.wg + 72);
    L.perm = L.bw + 256;
    L.NL = NL;
    return L;
}

struct WalkerCtx {
    NDet n;
    int vcode[2];   // virtual codes, ascending (-1 absent)
    int vs[2];      // virtual electrons per spin
    int e[2], h[2]; // active electrons / holes per spin
    int ne, nocc;   // active electrons, all non-core electrons
    double *ftab;   // global [2][A][V]: the walker's Fock elements (null: summed per term)
};

struct Block {
    int rk, pk;          // spin kinds of Ra and Pa: 0 none, 1 a, 2 b, 3 aa, 4 ab, 5 bb
    int vp[2];           // virtual electrons per spin of the block's neighbours
    int nra, npa;
    unsigned fam_end[4]; // cumulative rows per kept subset of the walker's virtual electrons
    unsigned R;          // rows per group
    unsigned ng, npk;    // groups, choices of Pa
};

__device__ __forceinline__ unsigned binom012(int n, int k) {
    if (k == 0) return 1u;
    if (n < k) return 0u;
    if (k == 1) return (unsigned)n;
    return (unsigned)(n * (n - 1) / 2);
}

// pair index k -> (i < j), k = j(j-1)/2 + i  (float estimate, one correction)
__device__ __forceinline__ void pair_decode(unsigned k, int &i, int &j) {
    int jj = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)k)) * 0.5f);
    jj -= (jj * (jj - 1) / 2 > (int)k);
    jj += ((jj + 1) * jj / 2 <= (int)k);
    j = jj;
    i = (int)k - jj * (jj - 1) / 2;
}

__device__ __forceinline__ int kind_a(int k) { return (k == 1 || k == 4) ? 1 : (k == 3 ? 2 : 0); }
__device__ __forceinline__ int kind_b(int k) { return (k == 2 || k == 4) ? 1 : (k == 5 ? 2 : 0); }
__device__ __forceinline__ unsigned kind_count(int k, int a, int b) {
    switch (k) {
        case 0: return 1u;
        case 1: return (unsigned)a;
        case 2: return (unsigned)b;
        case 3: return (unsigned)(a * (a - 1) / 2);
        case 4: return (unsigned)(a * b);
        default: return (unsigned)(b * (b - 1) / 2);
    }
}
// index within a kind -> up to two active codes (ascending)
__device__ __forceinline__ int kind_decode(int k, unsigned idx, const unsigned char *la, const unsigned char *lb,
                                           int nb, int &o0, int &o1) {
    o0 = o1 = -1;
    int i, j;
    switch (k) {
        case 0: return 0;
        case 1: o0 = la[idx]; return 1;
        case 2: o0 = lb[idx]; return 1;
        case 3: pair_decode(idx, i, j); o0 = la[i]; o1 = la[j]; return 2;
        case 4: o0 = la[idx / nb]; o1 = lb[idx % nb]; return 2;
        default: pair_decode(idx, i, j); o0 = lb[i]; o1 = lb[j]; return 2;
    }
}

// k-th virtual orbital of spin sg not occupied by the walker -> virtual code
__device__ __forceinline__ int avail_virtual(const DevProblem &P, const WalkerCtx &W, int sg, int k) {
    int a = k, lo = sg * P.V;
    int c0 = W.vcode[0] - lo, c1 = W.vcode[1] - lo;   // ascending; absent (-1) never in range
    if (W.vcode[0] >= lo && c0 < P.V && c0 <= a) a++;
    if (W.vcode[1] >= lo && c1 < P.V && c1 <= a) a++;
    return lo + a;
}

__device__ __forceinline__ bool block_setup(const DevProblem &P, const WalkerCtx &W, int rk, int pk, Block &b) {
    int r0 = kind_a(rk), r1 = kind_b(rk), p0 = kind_a(pk), p1 = kind_b(pk);
    b.rk = rk;
    b.pk = pk;
    b.vp[0] = W.vs[0] + r0 - p0;
    b.vp[1] = W.vs[1] + r1 - p1;
    if (b.vp[0] < 0 || b.vp[1] < 0 || b.vp[0] + b.vp[1] > 2) return false;
    b.nra = r0 + r1;
    b.npa = p0 + p1;
    unsigned nrk = kind_count(rk, W.e[0], W.e[1]);
    b.npk = kind_count(pk, W.h[0], W.h[1]);
    b.ng = nrk * b.npk;
    if (b.ng == 0) return false;
    unsigned tot = 0;
#pragma unroll
    for (int km = 0; km < 4; km++) {
        unsigned rows = 0;
        if (km < (1 << W.n.nv)) {
            int k0 = 0, k1 = 0, nk = 0;
#pragma unroll
            for (int i = 0; i < 2; i++)
                if (i < W.n.nv && ((km >> i) & 1)) { nk++; if (W.vcode[i] >= P.V) k1++; else k0++; }
            int a0 = b.vp[0] - k0, a1 = b.vp[1] - k1;
            int rem = b.nra + (W.n.nv - nk), add = b.npa + a0 + a1;
            if (a0 >= 0 && a1 >= 0 && rem >= 1 && rem <= 2 && add == rem)
                rows = binom012(P.V - W.vs[0], a0) * binom012(P.V - W.vs[1], a1);
        }
        tot += rows;
        b.fam_end[km] = tot;
    }
    b.R = tot;
    return tot > 0;
}

// Hash lookups whose first probe was already loaded (s = slots[slot]): most
// keys are settled by that one load, so several lookups can have their first
// loads in flight together; after a collision probing goes on one by one.
__device__ __forceinline__ uint2 probe_from(const DevTable &t, unsigned long long key, ulonglong2 s,
                                            unsigned slot) {
    while (true) {
        if (s.x == key) return make_uint2((unsigned)s.y, (unsigned)(s.y >> 32));
        if (s.x == SCQ_EMPTY_KEY) return make_uint2(0u, 0u);
        slot = (slot + 1u) & (unsigned)t.mask;
        s = t.slots[slot];
    }
}

// group g of block b: decode (Ra, Pa), form x_m, do the lookups of its overlap type
__device__ __forceinline__ void group_setup(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, const Block &b, unsigned g,
                            GroupInfo &G, uint2 *lst) {
    unsigned ri = g / b.npk, pi = g - ri * b.npk;
    int ra0, ra1, pa0, pa1;
    kind_decode(b.rk, ri, L.occ, L.occ + 32, W.e[1], ra0, ra1);
    kind_decode(b.pk, pi, L.hol, L.hol + 32, W.h[1], pa0, pa1);
    unsigned long long x = W.n.key;
    if (ra0 >= 0) x &= ~(1ull << ra0);
    if (ra1 >= 0) x &= ~(1ull << ra1);
    if (pa0 >= 0) x |= 1ull << pa0;
    if (pa1 >= 0) x |= 1ull << pa1;
    G.xkey = x;
    G.rg[0] = (short)(ra0 >= 0 ? g_of_active(P, ra0) : -1);
    G.rg[1] = (short)(ra1 >= 0 ? g_of_active(P, ra1) : -1);
    G.pg[0] = (short)(pa0 >= 0 ? g_of_active(P, pa0) : -1);
    G.pg[1] = (short)(pa1 >= 0 ? g_of_active(P, pa1) : -1);
    G.gam = 0.0;
    G.phi = 0.0;
    G.nl = 0;
    int vp = b.vp[0] + b.vp[1];
    if (vp == 0) {
        G.phi = ref_coef(P.ref, x);
        G.live = G.phi != 0.0;
    } else if (vp == 2) {
        lst[0] = table_find(P.xtab, x);
        G.live = lst[0].y != 0;
    } else {
        // y-list, then the nonempty x-lists of x - r (ascending r; r in the top
        // byte of .y); first probes issued four at a time
        unsigned hy = (unsigned)scq_hash(x) & (unsigned)P.ytab.mask;
        ulonglong2 sy = P.ytab.slots[hy];
        int k = 1;
        unsigned long long y = x;
        while (y) {
            int r0 = __ffsll((long long)y) - 1;
            y &= y - 1ull;
            int r1 = y ? __ffsll((long long)y) - 1 : -1;
            y &= y - 1ull;
            int r2 = y ? __ffsll((long long)y) - 1 : -1;
            y &= y - 1ull;
            int r3 = y ? __ffsll((long long)y) - 1 : -1;
            y &= y - 1ull;
            unsigned long long k0 = x & ~(1ull << r0);
            unsigned long long k1 = r1 >= 0 ? x & ~(1ull << r1) : k0;
            unsigned long long k2 = r2 >= 0 ? x & ~(1ull << r2) : k0;
            unsigned long long k3 = r3 >= 0 ? x & ~(1ull << r3) : k0;
            unsigned xm = (unsigned)P.xtab.mask;
            unsigned h0 = (unsigned)scq_hash(k0) & xm, h1 = (unsigned)scq_hash(k1) & xm;
            unsigned h2 = (unsigned)scq_hash(k2) & xm, h3 = (unsigned)scq_hash(k3) & xm;
            ulonglong2 s0 = P.xtab.slots[h0], s1 = P.xtab.slots[h1], s2 = P.xtab.slots[h2], s3 = P.xtab.slots[h3];
            uint2 o = probe_from(P.xtab, k0, s0, h0);
            if (o.y) lst[k++] = make_uint2(o.x, o.y | ((unsigned)r0 << 24));
            if (r1 >= 0) {
                o = probe_from(P.xtab, k1, s1, h1);
                if (o.y) lst[k++] = make_uint2(o.x, o.y | ((unsigned)r1 << 24));
            }
            if (r2 >= 0) {
                o = probe_from(P.xtab, k2, s2, h2);
                if (o.y) lst[k++] = make_uint2(o.x, o.y | ((unsigned)r2 << 24));
            }
            if (r3 >= 0) {
                o = probe_from(P.xtab, k3, s3, h3);
                if (o.y) lst[k++] = make_uint2(o.x, o.y | ((unsigned)r3 << 24));
            }
        }
        lst[0] = probe_from(P.ytab, x, sy, hy);
        G.nl = k - 1;
        G.live = (lst[0].y != 0) || k > 1;
    }
}

// phases of excitations from the walker, from its below-table
__device__ __forceinline__ double wphase_single(const WaveLDS &L, int gP, int gQ) {
    int e = L.bw[gP] + L.bw[gQ] - (gP < gQ);
    return (e & 1) ? -1.0 : 1.0;
}
__device__ __forceinline__ double wphase_double(const WaveLDS &L, int P1, int P2, int Q1, int Q2) {
    int e = L.bw[P1] + L.bw[P2] - (P1 < P2) + L.bw[Q2] - (P1 < Q2) - (P2 < Q2) + L.bw[Q1] - (P1 < Q1) - (P2 < Q1) +
            (Q2 < Q1);
    return (e & 1) ? -1.0 : 1.0;
}

// single P -> Q from the walker: returns the element with every non-core
// electron in the sum; *act receives the sum over active electrons only
// (Dyall's H_0)
// Coulomb and exchange integrals of electron j with the pair (p, q), lo/hi
// = min/max(p, q), or hi = the lane-varying one:  (jj|pq) at
// j (Np^3 + Np^2) + lo Np + hi and (pj|jq) = (lo j|j hi) at
// lo Np^3 + hi + j (Np^2 + Np): two multiply-adds per electron, the varying
// (or else the largest) index last.
struct JKOff {
    unsigned offJ, offK, cJ, cK;
};
// v: the lane-varying orbital if it is p or q (it becomes `hi`, the last index)
__device__ __forceinline__ JKOff jk_offsets(const DevProblem &P, int p, int q, int v = -1) {
    unsigned Np = (unsigned)P.Np, N2 = Np * Np, N3 = N2 * Np;
    unsigned lo = (unsigned)min(p, q), hi = (unsigned)max(p, q);
    if (v >= 0 && (v == p || v == q)) { hi = (unsigned)v; lo = (unsigned)(p + q - v); }
    JKOff o;
    o.offJ = lo * Np + hi;
    o.offK = lo * N3 + hi;
    o.cJ = N3 + N2;
    o.cK = N2 + Np;
    return o;
}
template <class R>
__device__ __forceinline__ R jk_term(const DevProblem &P, const JKOff &o, int j, bool same_spin) {
    const R *E = Ints<R>::eri(P);
    R J = E[__umul24((unsigned)j, o.cJ) + o.offJ];
    R K = same_spin ? E[__umul24((unsigned)j, o.cK) + o.offK] : R(0);
    return J - K;
}

template <class R>
__device__ __forceinline__ double single_elem_w2(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int gP,
                                                 int gQ, int vq, double *act) {
    int p = g_idx(P, gP), q = g_idx(P, gQ), sp = g_spin(P, gP);
    JKOff o = jk_offsets(P, p, q, vq);
    double v = (double)Ints<R>::heff(P)[q * P.Np + p];
#pragma unroll 4
    for (int i = 0; i < W.ne; i++) {
        int gJ = L.wg[i];
        double t = (double)jk_term<R>(P, o, g_idx(P, gJ), g_spin(P, gJ) == sp);
        v += (gJ == gP) ? 0.0 : t;
    }
    *act = v;
#pragma unroll
    for (int i = 0; i < 2; i++) {
        if (i >= W.n.nv) break;
        int gJ = W.n.vg[i];
        if (gJ == gP) continue;
        v += (double)jk_term<R>(P, o, g_idx(P, gJ), g_spin(P, gJ) == sp);
    }
    return v;
}

// h_eff[s][t] + sum_{j in y} [(st|jj) - delta (sj|jt)] with y = x_n - Ra + Pa,
// iterated as the walker's active electrons minus Ra plus Pa
template <class R>
__device__ __forceinline__ double fock_y(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int r0,
                                         int r1, int p0, int p1, int gT, int gS) {
    int t = g_idx(P, gT), s = g_idx(P, gS), st = g_spin(P, gT);
    JKOff o = jk_offsets(P, t, s);
    if (W.ftab) {
        // the walker's element (fock_table) minus the removed, plus the added electrons
        double v = W.ftab[(st * P.A + t) * P.V + (s - P.A)];
        double x[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            int gJ = c == 0 ? r0 : c == 1 ? r1 : c == 2 ? p0 : p1;
            x[c] = gJ >= 0 ? (double)jk_term<R>(P, o, g_idx(P, gJ), g_spin(P, gJ) == st) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 4; c++) v += c < 2 ? -x[c] : x[c];
        return v;
    }
    double v = (double)Ints<R>::heff(P)[s * P.Np + t];
#pragma unroll 4
    for (int i = 0; i < W.ne; i++) {
        int gJ = L.wg[i];
        double x = (double)jk_term<R>(P, o, g_idx(P, gJ), g_spin(P, gJ) == st);
        v += (gJ == r0 || gJ == r1) ? 0.0 : x;
    }
#pragma unroll
    for (int i = 0; i < 2; i++) {
        int gJ = i ? p1 : p0;
        if (gJ < 0) continue;
        v += (double)jk_term<R>(P, o, g_idx(P, gJ), g_spin(P, gJ) == st);
    }
    return v;
}

// The walker's Fock elements, for every active t and virtual a of either spin:
//   F[sg][t][a] = h_eff[A+a][t] + sum_{j in x_n} [(A+a t|j j) - [spin j = sg] (A+a j|j t)],
// the one-body element of an excitation t -> a with the walker's active
// electrons as the spectators.  The single terms of an overlap (a y-list
// entry: y = x_n - Ra + Pa as spectators) then cost one read and at most
// four corrections instead of a sum over every electron.  Lanes run along
// a, the last index of both integrals.  The wave reads the table back right
// after writing it: the fence orders its stores before those loads.
__device__ __forceinline__ void fock_table(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int lane) {
    int A = P.A, V = P.V, AV = A * V, tot = 2 * AV;
    for (int idx = lane; idx < tot; idx += WAVE) {
        int sg = idx >= AV, rem = idx - sg * AV, t = rem / V, a = rem - t * V;
        int s = A + a;
        JKOff o = jk_offsets(P, t, s);
        double v = P.heff[s * P.Np + t];
#pragma unroll 4
        for (int i = 0; i < W.ne; i++) {
            int gJ = L.wg[i];
            v += (double)jk_term<double>(P, o, g_idx(P, gJ), g_spin(P, gJ) == sg);
        }
        W.ftab[idx] = v;
    }
    __threadfence_block();
}

// <m|H|phi0> for m = y + virtual s of spin sg (0 alpha, 1 beta).  Table
// coefficients carry the part of each Slater-Condon phase that depends on the
// reference determinant (the annihilation of its removed electrons); the rest
// depends on spins and on the electron r only.  `fock` gives the
// single-excitation element.
// lists(0) is the y-list of y; lists(1..nl) are x-lists of y - r with r in
// the top byte of .y (ascending r; empty ones may be left out).
template <bool U, class R, class ListFn, class FockFn>
__device__ __forceinline__ double phi1(const DevProblem &P, unsigned long long y, int s, int sg, int nl, ListFn lists,
                       FockFn fock) {
    int gs = g_of_virtual(P, s);
    int bs = sg ? P.nea + P.neb : P.nea;   // electrons below s in any active-space determinant
    double acc1 = 0.0;
    uint2 oc = lists(0);
    for (unsigned k = 0; k < oc.y; k++) {
        ListEnt e = ent_load<U>(P.ytab.ents, oc.x + k);
        acc1 += e.val * fock(g_of_active(P, (int)e.code), gs);
    }
    double acc = ((bs - 1) & 1) ? -acc1 : acc1;
    // Doubles {t,u} -> {s, r}.  With Q1 < Q2 the sorted pair, the element is
    // (Q1 P1|Q2 P2) - (Q1 P2|Q2 P1) = sgn [(s p1|r p2) - (s p2|r p1)] with
    // sgn = +1 when s precedes r, each term present only for matching spins;
    // read as (p2 r|p1 s) = J and (p1 r|p2 s) = K so that the virtual s, the
    // only index that differs between the rows of a group, is the last one.
    //
    // Everything but the integrals is fixed per list (per r).  The reference
    // determinant d = y - r + t + u has the same electrons per spin as m, so
    // the number of alpha electrons among t < u is [s alpha] + [r alpha]:
    //   s, r of one spin:  t, u of that spin, element K - J;
    //   s alpha, r beta:   t alpha, u beta, element J (s precedes r);
    //   s beta, r alpha:   t alpha, u beta, element K.
    // The sign is (-1)^e, e = b(Q1) + b(Q2) - sum_Q [(P1 < Q) + (P2 < Q)] with
    // b(Q) the electrons of d below Q: b(s) = bs; b(r) = (electrons of y
    // below r) + [t < r] + [u < r], whose last two terms cancel (P < r);
    // (P < s) is 1 for every active P when s is beta and [P alpha] when s is
    // alpha.  So e = bs + (electrons of y below r) + [s alpha, r beta] mod 2.
    // (The part of the phase that depends on d alone is folded into the
    // stored coefficient.)
    // A list is taken in masked batches (eight entries with a wave-uniform
    // group U, whose entries are scalars; four in the lane path, where each
    // lane has its own group): the loads of a batch's entries, and then of
    // their integrals, are in flight together.  Same order of additions as
    // one entry at a time.
    unsigned Np = (unsigned)P.Np, N2 = Np * Np, N3 = N2 * Np;
    unsigned sp = (unsigned)g_idx(P, gs);
    const R *E = Ints<R>::eri(P);
    constexpr int B = (U ? 8 : 4);
    for (int li = 1; li <= nl; li++) {
        uint2 ox = lists(li);
        unsigned cnt = ox.y & 0xFFFFFFu;
        if (!cnt) continue;
        int r = (int)(ox.y >> 24);
        int sr = r >> 5;                         // spin of r
        bool needJ = !(sg == 1 && sr == 0), needK = !(sg == 0 && sr == 1);
        R jsign = (sg == sr) ? R(-1) : R(1);
        bool neg = ((bs + key_below(y, r) + (sg == 0 && sr == 1)) & 1) != 0;
        const R *Er = E + (unsigned)(r & 31) * N2 + sp;
        for (unsigned k = 0; k < cnt; k += B) {
            ListEnt ev[B];
            R Jv[B], Kv[B];
#pragma unroll
            for (int j = 0; j < B; j++) {
                if (k + j < cnt) {
                    ev[j] = ent_load<U>(P.xtab.ents, ox.x + k + j);
                } else {
                    ev[j].val = 0.0;
                    ev[j].code = (unsigned)(r << 6 | r);   // past the end: skipped below
                }
            }
#pragma unroll
            for (int j = 0; j < B; j++) {
                int t = (int)(ev[j].code >> 6), u = (int)(ev[j].code & 63u);
                bool use = t != r && u != r;
                unsigned q1 = (unsigned)(t & 31), q2 = (unsigned)(u & 31);
                Jv[j] = (use && needJ) ? Er[__umul24(q2, N3) + __umul24(q1, Np)] : R(0);
                Kv[j] = (use && needK) ? Er[__umul24(q1, N3) + __umul24(q2, Np)] : R(0);
            }
#pragma unroll
            for (int j = 0; j < B; j++) {
                int t = (int)(ev[j].code >> 6), u = (int)(ev[j].code & 63u);
                if (t == r || u == r) continue;   // a single y -> y + u (summed with the y-list), or past the end
                double el = (double)(Kv[j] + jsign * Jv[j]);
                acc += neg ? -ev[j].val * el : ev[j].val * el;
            }
        }
    }
    return acc;
}

// <m|H|phi0> for m = x + virtuals s1 < s2, from the x-list of x (signed coefficients)
// (a1 t|a2 u) is read as (t a1|u a2) at [t][a1][u][a2] (lane offset
// a1*Np^2 + a2, entry offset t*Np^3 + u*Np), or, when a1 is the virtual
// orbital that changes from lane to lane (vq), as (u a2|t a1) at
// [u][a2][t][a1]: either way the lane-varying index is the last one.
template <bool U, class R>
__device__ __forceinline__ double phi2(const DevProblem &P, int s1, int s2, uint2 ox, int vq, const VecEnts &ve) {
    int sg1 = s1 >= P.V, sg2 = s2 >= P.V;
    unsigned Np = (unsigned)P.Np, N3 = Np * Np * Np;
    unsigned a1 = (unsigned)(P.A + s1 - sg1 * P.V), a2 = (unsigned)(P.A + s2 - sg2 * P.V);
    bool sw = vq == (int)a1;
    const R *E = Ints<R>::eri(P) + (sw ? (a2 * Np) * Np + a1 : (a1 * Np) * Np + a2);
    unsigned Ct = sw ? Np : N3, Cu = sw ? N3 : Np;   // entry offset t*Ct + u*Cu of (t a1|u a2)
    double acc = 0.0;
    // masked batches of four entries whose loads, then their integrals'
    // loads, are in flight together; same order of additions as one entry at
    // a time
    constexpr int B = 4;
    bool ab = sg1 != sg2;   // alpha-beta pair: only (s1 t|s2 u) survives
    // a block fixes the spins of m's virtual electrons, so with a
    // wave-uniform group (every row of the wave in one block) this is uniform
    if (U) ab = uni((int)ab) != 0;
    unsigned vn = uni(ve.n);
    if (U && vn <= 64u) {
        constexpr int BV = 8;
        // entries already in the lanes: broadcast a batch, then its integrals' loads in flight together
        for (unsigned k = 0; k < vn; k += BV) {
            unsigned cd[BV];
            double wv[BV];
            R e1[BV], e2[BV];
#pragma unroll
            for (int j = 0; j < BV; j++) {
                unsigned src = min(k + j, 63u);
                cd[j] = (unsigned)__builtin_amdgcn_readlane((int)ve.code, (int)src);
                wv[j] = k + j < vn ? readlane_d(ve.val, src) : 0.0;   // past the end: weight 0
            }
#pragma unroll
            for (int j = 0; j < BV; j++) {
                unsigned t = (cd[j] >> 6) & 31u, u = cd[j] & 31u;
                bool in = k + j < vn;
                e1[j] = in ? E[__umul24(t, Ct) + __umul24(u, Cu)] : R(0);
                e2[j] = (in && !ab) ? E[__umul24(u, Ct) + __umul24(t, Cu)] : R(0);
            }
#pragma unroll
            for (int j = 0; j < BV; j++) acc += wv[j] * (double)(e1[j] - e2[j]);
        }
        return (ab && ((P.neb + 1) & 1)) ? -acc : acc;
    }
    for (unsigned k = 0; k < ox.y; k += B) {
        ListEnt ev[B];
        R e1[B], e2[B];
#pragma unroll
        for (int j = 0; j < B; j++) {
            if (k + j < ox.y) {
                ev[j] = ent_load<U>(P.xtab.ents, ox.x + k + j);
            } else {
                ev[j].val = 0.0;
                ev[j].code = 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < B; j++) {
            unsigned t = (ev[j].code >> 6) & 31u, u = ev[j].code & 31u;
            bool in = k + j < ox.y;
            e1[j] = in ? E[__umul24(t, Ct) + __umul24(u, Cu)] : R(0);
            e2[j] = (in && !ab) ? E[__umul24(u, Ct) + __umul24(t, Cu)] : R(0);
        }
#pragma unroll
        for (int j = 0; j < B; j++)
            if (k + j < ox.y) acc += ev[j].val * (double)(e1[j] - e2[j]);
    }
    // alpha-beta: spin part of the phase (-1)^(n_beta + 1)
    return (ab && ((P.neb + 1) & 1)) ? -acc : acc;
}

// psi of one determinant with its own lookups (one lane; initialisation / snapshots)
template <class R>
__device__ __forceinline__ double psi_direct(const DevProblem &P, unsigned long long key, unsigned virt) {
    int vcode[2] = {(int)(virt & 0xFFFFu), (int)(virt >> 16)};
    int nv = (vcode[0] != (int)SCQ_NOVIRT) + (vcode[1] != (int)SCQ_NOVIRT);
    if (nv == 0) return P.ccls[0] * ref_coef(P.ref, key);
    if (nv == 1) {
        double phi = phi1<false, R>(
            P, key, vcode[0], (int)(vcode[0] >= P.V), popc64(key),
            [&](int k) -> uint2 {
                if (k == 0) return table_find(P.ytab, key);
                unsigned long long y = key;
                for (int i = 1; i < k; i++) y &= y - 1ull;
                int r = __ffsll((long long)y) - 1;
                uint2 ox = table_find(P.xtab, key & ~(1ull << r));
                return make_uint2(ox.x, ox.y | ((unsigned)r << 24));
            },
            [&](int gT, int gS) -> double {
                NDet d;
                d.nv = 0;
                d.vg[0] = d.vg[1] = SCQ_NOG;
                d.key = key | (1ull << ((gT >= P.Np ? 32 : 0) + g_idx(P, gT)));
                return single_elem<R>(P, d, gT, gS, false);
            });
        return P.ccls[class_id1(P.V, vcode[0])] * phi;
    }
    return P.ccls[class_id2(P.V, vcode[0], vcode[1])] *
           phi2<false, R>(P, vcode[0], vcode[1], table_find(P.xtab, key), -1, vec_ents_off());
}

// Row r of a block, independent of the group: the virtual set of m, its
// class and SC coefficient, and the virtual parts of the excitation n -> m.
struct RowDec {
    int Lp0, Lp1;        // virtual codes of m (ascending, -1 absent)
    int rv0, rv1;        // removed virtual electrons (g codes, -1 absent)
    int ad0, ad1;        // added virtual electrons (g codes, -1 absent)
    double c;            // SC coefficient of m's class
    int cls;
    int vq;              // orbital index (0..Np-1) of the added virtual electron that changes fastest
                         // from row to row (consecutive lanes), -1 if none is added
    bool same;           // m keeps the walker's virtual set
};

__device__ __forceinline__ void row_decode(const DevProblem &P, const WalkerCtx &W, const Block &b, unsigned r,
                                           RowDec &d) {
    int km = 0;
    unsigned start = 0;
    if (r >= b.fam_end[0]) { km = 1; start = b.fam_end[0]; }
    if (r >= b.fam_end[1]) { km = 2; start = b.fam_end[1]; }
    if (r >= b.fam_end[2]) { km = 3; start = b.fam_end[2]; }
    r -= start;
    int kc0 = -1, kc1 = -1, nk = 0, k0 = 0, k1 = 0;
    d.rv0 = d.rv1 = -1;
#pragma unroll
    for (int i = 0; i < 2; i++) {
        if (i >= W.n.nv) break;
        int c = W.vcode[i];
        if ((km >> i) & 1) {
            if (nk == 0) kc0 = c; else kc1 = c;
            nk++;
            if (c >= P.V) k1++; else k0++;
        } else {
            int g = W.n.vg[i];
            if (d.rv0 < 0) d.rv0 = g; else d.rv1 = g;
        }
    }
    int a0 = b.vp[0] - k0, a1 = b.vp[1] - k1;
    int x0 = -1, x1 = -1, nad = 0;   // added virtual codes
    if (a0 + a1 > 0) {
        unsigned c1 = binom012(P.V - W.vs[1], a1);
        unsigned i0 = (unsigned)((float)r / (float)c1);
        i0 -= (i0 * c1 > r);
        i0 += ((i0 + 1) * c1 <= r);
        unsigned i1 = r - i0 * c1;
        if (a0 == 1) { x0 = avail_virtual(P, W, 0, (int)i0); nad = 1; }
        else if (a0 == 2) { int i, j; pair_decode(i0, i, j); x0 = avail_virtual(P, W, 0, i); x1 = avail_virtual(P, W, 0, j); nad = 2; }
        if (a1 == 1) { int v = avail_virtual(P, W, 1, (int)i1); if (nad == 0) x0 = v; else x1 = v; nad++; }
        else if (a1 == 2) { int i, j; pair_decode(i1, i, j); x0 = avail_virtual(P, W, 1, i); x1 = avail_virtual(P, W, 1, j); nad = 2; }
    }
    d.ad0 = x0 >= 0 ? g_of_virtual(P, x0) : -1;
    d.ad1 = x1 >= 0 ? g_of_virtual(P, x1) : -1;
    // r = i0 * c1 + i1: the beta part (i1) changes fastest; inside a pair the
    // smaller index i does; so it is x0 except for an alpha-beta pair (x1)
    int xf = (a0 == 1 && a1 == 1) ? x1 : x0;
    d.vq = xf >= 0 ? g_idx(P, g_of_virtual(P, xf)) : -1;
    int vp = b.vp[0] + b.vp[1];
    if (vp == 0) {
        d.Lp0 = d.Lp1 = -1;
        d.cls = 0;
    } else if (vp == 1) {
        d.Lp0 = nk ? kc0 : x0;
        d.Lp1 = -1;
        d.cls = 1 + d.Lp0;
    } else {
        int y0 = nk > 0 ? kc0 : x0;
        int y1 = nk > 1 ? kc1 : (nk == 1 ? x0 : x1);
        d.Lp0 = y0 < y1 ? y0 : y1;
        d.Lp1 = y0 < y1 ? y1 : y0;
        int V2 = 2 * P.V;
        d.cls = 1 + V2 + d.Lp0 * V2 - d.Lp0 * (d.Lp0 + 1) / 2 + (d.Lp1 - d.Lp0 - 1);
    }
    d.c = P.ccls[d.cls];
    d.same = (nad == 0 && nk == W.n.nv);
}

struct RowRes {
    double hnm, psi, hd, phase;
    bool ok;
};

// A group as one lane sees it.  U: the same group for the whole wave, its
// fields held in scalar registers and its lists read with scalar loads.
struct GroupView {
    unsigned long long xkey;
    double phi;
    int rg0, rg1, pg0, pg1, nl;
    const uint2 *lst;
};

template <bool U>
__device__ __forceinline__ GroupView group_view(const WaveLDS &L, unsigned gi) {
    const GroupInfo &G = L.G[gi];
    GroupView v;
    v.xkey = G.xkey;
    v.phi = G.phi;
    v.rg0 = G.rg[0];
    v.rg1 = G.rg[1];
    v.pg0 = G.pg[0];
    v.pg1 = G.pg[1];
    v.nl = G.nl;
    if (U) {
        v.xkey = uni(v.xkey);
        v.phi = uni(v.phi);
        v.rg0 = uni(v.rg0);
        v.rg1 = uni(v.rg1);
        v.pg0 = uni(v.pg0);
        v.pg1 = uni(v.pg1);
        v.nl = uni(v.nl);
    }
    v.lst = L.lst + gi * L.NL;
    return v;
}

template <bool U>
__device__ __forceinline__ uint2 view_list(const GroupView &v, int k) {
    uint2 o = v.lst[k];
    if (U) {
        o.x = uni(o.x);
        o.y = uni(o.y);
    }
    return o;
}

// row d of group G: <m|H|n>, psi(m), the Dyall element if m keeps n's virtual set.
// R is the precision of the two-electron terms of psi(m) (the doubles of the
// reference expansion); <m|H|n> and the one-body (Fock) elements inside psi(m)
// are FP64 in both forms: they are few per row and the largest terms, so
// they would carry most of the FP32 rounding of a local energy.
template <int VP, bool U, class R>
__device__ __forceinline__ void row_eval(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L,
                                         const RowDec &d, const GroupView &G, const VecEnts &ve, RowRes &o) {
    // outer excitation n -> m: removed P*, added Q* (ascending spin-orbital order)
    int Pr0 = G.rg0, Pr1 = G.rg1, Qa0 = G.pg0, Qa1 = G.pg1;
    if (Pr0 < 0) { Pr0 = d.rv0; Pr1 = d.rv1; } else if (Pr1 < 0) Pr1 = d.rv0;
    if (Qa0 < 0) { Qa0 = d.ad0; Qa1 = d.ad1; } else if (Qa1 < 0) Qa1 = d.ad0;
    if (Pr1 >= 0 && Pr0 > Pr1) { int t = Pr0; Pr0 = Pr1; Pr1 = t; }
    if (Qa1 >= 0 && Qa0 > Qa1) { int t = Qa0; Qa0 = Qa1; Qa1 = t; }
    o.ok = true;
    o.hd = 0.0;
    if (Pr1 < 0) {
        double ph = wphase_single(L, Pr0, Qa0);
        double act;
        o.phase = ph;
        o.hnm = ph * single_elem_w2<double>(P, W, L, Pr0, Qa0, d.vq, &act);
        o.hd = ph * act;
    } else {
        double ph = wphase_double(L, Pr0, Pr1, Qa0, Qa1);
        o.phase = ph;
        // the lane-varying virtual, when the row adds one, is read as the last index
        double e = (d.vq >= 0) ? double_elem_x<double>(P, Pr0, Pr1, Qa0, Qa1, g_idx(P, Qa1) == d.vq)
                               : double_elem<double>(P, Pr0, Pr1, Qa0, Qa1);
        o.hnm = ph * e;
        o.hd = o.hnm;
        if (P.eps_screen > 0.0 && !(fabs(o.hnm) > P.eps_screen)) { o.ok = false; o.psi = 0.0; return; }
    }
    double phi;
    if (VP == 0) {
        phi = G.phi;
    } else if (VP == 1) {
        // the block fixes the spin of the one virtual electron, so it is the
        // same for every row of the wave: a scalar
        phi = phi1<U, R>(P, G.xkey, d.Lp0, uni((int)(d.Lp0 >= P.V)), G.nl,
                         [&](int k) -> uint2 { return view_list<U>(G, k); },
                         [&](int gT, int gS) -> double {
                             return fock_y<double>(P, W, L, G.rg0, G.rg1, G.pg0, G.pg1, gT, gS);
                         });
    } else {
        phi = phi2<U, R>(P, d.Lp0, d.Lp1, view_list<U>(G, 0), d.vq, ve);
    }
    o.psi = d.c * phi;
}

template <bool U, class R>
__device__ __forceinline__ void row_eval_any(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int vp,
                                             const RowDec &d, const GroupView &G, const VecEnts &ve, RowRes &o) {
    if (vp == 0) row_eval<0, U, R>(P, W, L, d, G, ve, o);
    else if (vp == 1) row_eval<1, U, R>(P, W, L, d, G, ve, o);
    else row_eval<2, U, R>(P, W, L, d, G, ve, o);
}

// Sum over the 64 lanes of a wave with DPP moves (no LDS round trips):
// prefix sums inside each row of 16 lanes (row_shr 1, 2, 4, 8), then row
// totals carried across rows (row_bcast 15 into rows 1 and 3, row_bcast 31
// into rows 2 and 3).  Lane 63 ends with the total, which is returned
// wave-uniform.  Fixed order of additions, so the result is deterministic.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
    long long b = __double_as_longlong(v);
    int lo = (int)b, hi = (int)(b >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0x111, 0xf>(v);   // row_shr:1
    v += dpp_d<0x112, 0xf>(v);   // row_shr:2
    v += dpp_d<0x114, 0xf>(v);   // row_shr:4
    v += dpp_d<0x118, 0xf>(v);   // row_shr:8
    v += dpp_d<0x142, 0xa>(v);   // row_bcast:15 -> rows 1, 3
    v += dpp_d<0x143, 0xc>(v);   // row_bcast:31 -> rows 2, 3
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ void walker_setup(const DevProblem &P, const WaveLDS &L, int lane, unsigned long long key,
                                    unsigned virt, WalkerCtx &W) {
    key = uni(key);
    virt = uni(virt);
    W.n.key = key;
    unsigned v0 = virt & 0xFFFFu, v1 = virt >> 16;   // ascending; v1 present only if v0 is
    bool h0 = v0 != SCQ_NOVIRT, h1 = v1 != SCQ_NOVIRT;
    W.n.nv = (int)h0 + (int)h1;
    W.vcode[0] = h0 ? (int)v0 : -1;
    W.vcode[1] = h1 ? (int)v1 : -1;
    W.n.vg[0] = h0 ? g_of_virtual(P, (int)v0) : SCQ_NOG;
    W.n.vg[1] = h1 ? g_of_virtual(P, (int)v1) : SCQ_NOG;
    W.vs[0] = (h0 && v0 < (unsigned)P.V) + (h1 && v1 < (unsigned)P.V);
    W.vs[1] = W.n.nv - W.vs[0];
    uint32_t am = (P.A >= 32) ? 0xFFFFFFFFu : ((1u << P.A) - 1u);
    for (int s = 0; s < 2; s++) {
        uint32_t occ = (uint32_t)(key >> (32 * s)) & am;
        uint32_t hol = ~(uint32_t)(key >> (32 * s)) & am;
        W.e[s] = popc32(occ);
        W.h[s] = popc32(hol);
        if (lane < 32) {
            uint32_t below = lane ? ((1u << lane) - 1u) : 0u;
            if ((occ >> lane) & 1u) L.occ[32 * s + popc32(occ & below)] = (unsigned char)(32 * s + lane);
            if ((hol >> lane) & 1u) L.hol[32 * s + popc32(hol & below)] = (unsigned char)(32 * s + lane);
        }
    }
    W.ne = W.e[0] + W.e[1];
    W.nocc = W.ne + W.n.nv;
    W.ftab = nullptr;
    __syncwarp();
    if (lane < W.e[0]) L.wg[lane] = (short)g_of_active(P, L.occ[lane]);
    else if (lane < W.ne) L.wg[lane] = (short)g_of_active(P, L.occ[32 + lane - W.e[0]]);
    else if (lane == W.ne && W.n.nv > 0) L.wg[lane] = (short)W.n.vg[0];
    else if (lane == W.ne + 1 && W.n.nv > 1) L.wg[lane] = (short)W.n.vg[1];
    for (int g = lane; g < 2 * P.Np; g += WAVE) L.bw[g] = (unsigned char)below(P, W.n, g);
    __syncwarp();
}

// <n|H|n> (with_virt) or <n|H_0|n> (active part only), summed over lanes in a fixed tree
__device__ __forceinline__ double wave_diag(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int lane, bool with_virt) {
    int n = with_virt ? W.nocc : W.ne;
    double v = 0.0;
    if (lane < n) {
        int gi = L.wg[lane];
        int ii = g_idx(P, gi), si = g_spin(P, gi);
        double two = 0.0;
        for (int j = 0; j < n; j++) {
            int gj = L.wg[j];
            int jj = g_idx(P, gj);
            double J = eri4(P, ii, ii, jj, jj);
            double K = (g_spin(P, gj) == si) ? eri4(P, ii, jj, jj, ii) : 0.0;
            two += J - K;
        }
        v = P.heff[ii * P.Np + ii] + 0.5 * two;
    }
    return P.e_core + wave_sum(v);
}

struct EvalOut {
    double eloc, elocd, gamma, psi_new;
    unsigned long long key_new;
    unsigned virt_new;
    bool moved;
};

struct Acc {
    double E, D, G;                   // sum H psi, sum H_D psi, sum |psi|
    double best;                      // first-reaction clock of the best group so far
    unsigned long long bestkey;
    int bestblk;                      // rk * 6 + pk
    int bestg;
};

// sub-wave sum over S consecutive lanes (S a power of two), fixed tree
__device__ __forceinline__ double subwave_sum(double v, unsigned S) {
    for (unsigned d = 1; d < S; d <<= 1) v += __shfl_xor(v, (int)d);
    return v;
}

// rows r0 + t*S + (lane mod S), t < ntile, of the live groups (S lanes per
// group, 64/S groups per pass): group data differs between sub-waves
template <class R>
__device__ __forceinline__ void subwave_rows(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int lane,
                                             const Block &b, int vp, bool dy, unsigned S, unsigned r0, unsigned ntile,
                                             unsigned nlive, RowDec &d, bool decoded, Acc &a) {
    int sh = __ffs(S) - 1;
    unsigned gpi = WAVE >> sh;
    unsigned sub = (unsigned)lane & (S - 1), grp = (unsigned)lane >> sh;
    for (unsigned t = 0; t < ntile; t++) {
        unsigned r = r0 + t * S + sub;
        bool rv = r < b.R;
        if (!decoded && rv) row_decode(P, W, b, r, d);
        for (unsigned gp = 0; gp < nlive; gp += gpi) {
            unsigned gc = gp + grp;
            unsigned gi = gc < nlive ? L.perm[gc] : 0u;
            double v = 0.0;
            if (rv && gc < nlive) {
                RowRes o;
                GroupView gv = group_view<false>(L, gi);
                row_eval_any<false, R>(P, W, L, vp, d, gv, vec_ents_off(), o);
                if (o.ok) {
                    a.E += o.hnm * o.psi;
                    v = fabs(o.psi);
                    a.G += v;
                    if (dy && d.same) a.D += o.hd * o.psi;
                }
            }
            v = subwave_sum(v, S);
            if (sub == 0 && gc < nlive) L.G[gi].gam += v;
            __syncwarp();
        }
    }
}

// sweep one block: 64 groups set up at a time, each group owns a sub-wave of
// S lanes, lane row index r = tile*S + (lane mod S) fixed across groups.
// Groups of more than 32 rows own the whole wave (wave-uniform group data,
// 64-row tiles); a last tile of at most 32 rows is not given a whole wave
// per group but goes, for several groups at once, to sub-waves of 16 or 32
// lanes (the blocks with one virtual electron added have 75 or 76 rows:
// 64 + 11 or 12).
template <bool MOVE, class R>
__device__ __forceinline__ void sweep_block(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int lane, const Block &b,
                            uint32_t wid, uint32_t step, bool dy, Acc &a) {
    GroupInfo &mg = L.G[lane];
    uint2 *mlst = L.lst + lane * L.NL;
    unsigned S = 1;
    while (S < b.R && S < WAVE) S <<= 1;
    int sh = __ffs(S) - 1;
    unsigned ntile = (b.R + S - 1) >> sh;      // > 1 only when R > 64
    unsigned sub = (unsigned)lane & (S - 1);
    int vp = b.vp[0] + b.vp[1];
    // wave-uniform tiles and the short last tile (S == WAVE only)
    unsigned tail = b.R - WAVE * (ntile - 1);
    unsigned ntu = (S == WAVE && ntile > 1 && tail <= 32) ? ntile - 1 : ntile;
    unsigned St = tail <= 16 ? 16u : 32u;
    RowDec d;
    if (ntile == 1 && sub < b.R) row_decode(P, W, b, sub, d);
    for (unsigned gb = 0; gb < b.ng; gb += WAVE) {
        unsigned g = gb + (unsigned)lane;
        bool live = false;
        if (g < b.ng) {
            group_setup(P, W, L, b, g, mg, mlst);
            live = mg.live;
        }
        // rows of a group whose lookups all came back empty have psi(m) = 0:
        // they add nothing to E_L, E_D,L or the rates, so only live groups are swept
        unsigned long long lm = __ballot(live);
        unsigned nlive = (unsigned)__popcll(lm);
        if (live) L.perm[__popcll(lm & ((1ull << lane) - 1ull))] = (unsigned char)lane;
        __syncwarp();
        if (S == WAVE) {
            // one group per pass: its data is wave-uniform
            for (unsigned t = 0; t < ntu; t++) {
                unsigned r = t * WAVE + sub;
                bool rv = r < b.R;
                if (ntile > 1 && rv) row_decode(P, W, b, r, d);
                for (unsigned gc = 0; gc < nlive; gc++) {
                    unsigned gi = uni((unsigned)L.perm[gc]);
                    GroupView gv = group_view<true>(L, gi);
                    // the group's list entries into the lanes (every lane active here)
                    VecEnts ve = vp == 2 ? vec_ents_load(P.xtab.ents, view_list<true>(gv, 0), lane) : vec_ents_off();
                    double v = 0.0;
                    if (rv) {
                        RowRes o;
                        row_eval_any<true, R>(P, W, L, vp, d, gv, ve, o);
                        if (o.ok) {
                            a.E += o.hnm * o.psi;
                            v = fabs(o.psi);
                            a.G += v;
                            if (dy && d.same) a.D += o.hd * o.psi;
                        }
                    }
                    v = wave_sum(v);
                    if (lane == 0) L.G[gi].gam += v;
                    __syncwarp();
                }
            }
        }
        // sub-wave groups: all rows of small blocks, or the short last tile
        unsigned nts = S == WAVE ? ntile - ntu : ntile;
        if (nts)
            subwave_rows<R>(P, W, L, lane, b, vp, dy, S == WAVE ? St : S, S == WAVE ? WAVE * ntu : 0u, nts, nlive,
                            d, S != WAVE && ntile == 1, a);
        if (MOVE && g < b.ng && mg.gam > 0.0) {
            double tau = exp_draw(P.seed, wid, step, 0u, (uint32_t)mg.xkey, (uint32_t)(mg.xkey >> 32)) / mg.gam;
            if (tau < a.best || (tau == a.best && mg.xkey < a.bestkey)) {
                a.best = tau;
                a.bestkey = mg.xkey;
                a.bestblk = b.rk * 6 + b.pk;
                a.bestg = (int)g;
            }
        }
        __syncwarp();
    }
}

template <bool MOVE, class R>
__device__ __forceinline__ void walker_eval(const DevProblem &P, const WaveLDS &L, int lane, unsigned long long key, unsigned virt,
                            double psin, uint32_t wid, uint32_t step, double *ftab, EvalOut &out) {
    WalkerCtx W;
    walker_setup(P, L, lane, key, virt, W);
    // the Fock table pays where single terms are many: walkers with at most one
    // virtual electron (two-virtual walkers reach few one-virtual overlaps)
    W.ftab = W.n.nv < 2 ? ftab : nullptr;
    if (W.ftab) fock_table(P, W, L, lane);
    double hnn = wave_diag(P, W, L, lane, true);
    bool dy = (P.mode == 1 && W.n.nv > 0);
    double hdnn = 0.0;
    if (dy) {
        hdnn = wave_diag(P, W, L, lane, false);
#pragma unroll
        for (int i = 0; i < 2; i++) {
            if (i >= W.n.nv) break;
            int s = W.vcode[i];
            hdnn += P.eps[s >= P.V ? s - P.V : s];
        }
    }
    Acc a;
    a.E = a.D = a.G = 0.0;
    a.best = INFINITY;
    a.bestkey = ~0ull;
    a.bestblk = -1;
    a.bestg = -1;
    for (int rk = 0; rk < 6; rk++)
        for (int pk = 0; pk < 6; pk++) {
            Block b;
            if (!block_setup(P, W, rk, pk, b)) continue;
            if (P.active_only && b.vp[0] + b.vp[1] > 0) continue;
            sweep_block<MOVE, R>(P, W, L, lane, b, wid, step, dy, a);
        }
    double E = wave_sum(a.E), G = wave_sum(a.G);
    double D = dy ? wave_sum(a.D) : 0.0;
    out.eloc = hnn + E / psin;
    out.elocd = dy ? hdnn + D / psin : NAN;
    out.gamma = G / fabs(psin);
    out.moved = false;
    if (!MOVE) return;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        double ob = __shfl_xor(a.best, d);
        unsigned long long okk = __shfl_xor(a.bestkey, d);
        int obk = __shfl_xor(a.bestblk, d);
        int og = __shfl_xor(a.bestg, d);
        if (ob < a.best || (ob == a.best && okk < a.bestkey)) { a.best = ob; a.bestkey = okk; a.bestblk = obk; a.bestg = og; }
    }
    if (a.bestblk < 0) return;
    Block b;
    block_setup(P, W, a.bestblk / 6, a.bestblk % 6, b);
    GroupInfo &sg = L.G[WAVE];
    uint2 *slst = L.lst + WAVE * L.NL;
    if (lane == 0) group_setup(P, W, L, b, (unsigned)a.bestg, sg, slst);
    __syncwarp();
    GroupView sgv = group_view<true>(L, WAVE);
    int vp = b.vp[0] + b.vp[1];
    double b2 = INFINITY;
    int bcls = 0x7fffffff;
    double bpsi = 0.0;
    unsigned bvirt = 0;
    VecEnts sve = vp == 2 ? vec_ents_load(P.xtab.ents, view_list<true>(sgv, 0), lane) : vec_ents_off();
    for (unsigned r = lane; r < b.R; r += WAVE) {
        RowDec d;
        row_decode(P, W, b, r, d);
        RowRes o;
        row_eval_any<true, R>(P, W, L, vp, d, sgv, sve, o);
        if (!o.ok || o.psi == 0.0) continue;
        double tau = exp_draw(P.seed, wid, step, 1u, (uint32_t)d.cls, 0u) / fabs(o.psi);
        if (tau < b2 || (tau == b2 && d.cls < bcls)) {
            b2 = tau;
            bcls = d.cls;
            bpsi = o.psi;
            bvirt = (d.Lp0 >= 0 ? (unsigned)d.Lp0 : SCQ_NOVIRT) | ((d.Lp1 >= 0 ? (unsigned)d.Lp1 : SCQ_NOVIRT) << 16);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        double ob = __shfl_xor(b2, d);
        int oc = __shfl_xor(bcls, d);
        double op = __shfl_xor(bpsi, d);
        unsigned ov = __shfl_xor(bvirt, d);
        if (ob < b2 || (ob == b2 && oc < bcls)) { b2 = ob; bcls = oc; bpsi = op; bvirt = ov; }
    }
    __syncwarp();
    if (b2 == INFINITY) return;
    out.moved = true;
    out.psi_new = bpsi;
    out.key_new = sg.xkey;
    out.virt_new = bvirt;
}

// ---------------------------------------------------------------------------
// fixed-point (2^-64 resolution, 128-bit two's complement) accumulation:
// integer atomics make the per-class sums independent of arrival order
// ---------------------------------------------------------------------------
__device__ inline void to_fixed(double x, unsigned long long &lo, unsigned long long &hi) {
    lo = 0; hi = 0;
    if (x == 0.0 || !isfinite(x)) return;
    int e;
    double m = frexp(fabs(x), &e);
    unsigned long long M = (unsigned long long)ldexp(m, 53);
    int sh = e - 53 + 64;
    unsigned long long l, h;
    if (sh >= 64 + 10) { l = ~0ull; h = 0x7fffffffffffffffull; }
    else if (sh >= 64) { l = 0; h = M << (sh - 64); }
    else if (sh > 0) { l = M << sh; h = M >> (64 - sh); }
    else if (sh == 0) { l = M; h = 0; }
    else {
        int r = -sh;
        h = 0;
        l = r >= 64 ? 0ull : ((M + (1ull << (r - 1))) >> r);
    }
    if (x < 0) { l = ~l + 1ull; h = ~h + (l == 0 ? 1ull : 0ull); }
    lo = l; hi = h;
}
__device__ inline void fx_add(unsigned long long *slot, double x) {
    unsigned long long lo, hi;
    to_fixed(x, lo, hi);
    if (!lo && !hi) return;
    unsigned long long old = atomicAdd(slot, lo);
    unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
    atomicAdd(slot + 1, hi + carry);
}

struct WalkerArrays {
    double *ftab;                 // [W][2][A][V] per-walker Fock elements (scratch of the step)
    unsigned long long *key;
    unsigned *virt;
    double *psi;
    double *wsum;                 // [3][W]
    unsigned long long *cacc;     // [ncg][4][ncls][2]
    unsigned long long *bad;      // [1]
    int ncg;                      // walker groups of the class sums
};

__device__ __forceinline__ long long class_of_virt(const DevProblem &P, unsigned virt) {
    unsigned v0 = virt & 0xFFFFu, v1 = virt >> 16;
    if (v0 == SCQ_NOVIRT) return 0;
    if (v1 == SCQ_NOVIRT) return class_id1(P.V, (int)v0);
    return class_id2(P.V, (int)v0, (int)v1);
}

// One walker's nsteps continuous-time steps: evaluate, accumulate after
// burn-in, move.  Shared by the single-system and the batched launch.
template <class R>
__device__ __forceinline__ void sample_walker(const DevProblem &P, const WalkerArrays &S, long long W, long long w,
                                              long long step0, int nsteps, long long burn_in, const WaveLDS &L,
                                              int lane) {
    unsigned long long key = S.key[w];
    unsigned virt = S.virt[w];
    double psi = S.psi[w];
    double st = S.wsum[w], ste = S.wsum[W + w], st0 = S.wsum[2 * W + w];
    long long nbad = 0;
    double *ftab = S.ftab ? S.ftab + w * (2LL * P.A * P.V) : nullptr;
    for (int k = 0; k < nsteps; k++) {
        long long step = step0 + k;
        EvalOut o;
        key = uni(key);
        virt = uni(virt);
        if constexpr (sizeof(R) < sizeof(double)) {
            // precision form: the walker's own overlap, which divides every
            // term of E_L, is recomputed in FP64 (one lane, once per step)
            double pd = 0.0;
            if (lane == 0) pd = psi_direct<double>(P, key, virt);
            psi = __shfl(pd, 0);
        }
        psi = uni(psi);
        walker_eval<true, R>(P, L, lane, key, virt, psi, (uint32_t)w, (uint32_t)step, ftab, o);
        bool good = o.moved && isfinite(o.eloc) && o.gamma > 0.0 && isfinite(o.gamma);
        if (!good) { nbad++; continue; }
        if (step >= burn_in) {
            double t = 1.0 / o.gamma;
            long long cls = class_of_virt(P, virt);
            st += t;
            ste += t * o.eloc;
            if (cls == 0) st0 += t;
            if (lane < 4) {
                double c = P.ccls[cls];
                double q = lane == 0 ? t : lane == 1 ? t * o.eloc : lane == 2 ? t / (c * c)
                                                                  : ((P.mode == 1 && cls != 0) ? t * o.elocd / (c * c) : 0.0);
                long long grp = w * S.ncg / W;
                fx_add(S.cacc + ((grp * 4 + lane) * P.ncls + cls) * 2, q);
            }
        }
        key = o.key_new;
        virt = o.virt_new;
        psi = o.psi_new;
    }
    if (lane == 0) {
        S.key[w] = key;
        S.virt[w] = virt;
        S.psi[w] = psi;
        S.wsum[w] = st;
        S.wsum[W + w] = ste;
        S.wsum[2 * W + w] = st0;
        if (nbad) atomicAdd(S.bad, (unsigned long long)nbad);
    }
}

// Launch order of the walkers: a walker's cost grows with its neighbour count,
// which is largest with no virtual electron and smallest with two, so walkers
// are dispatched by ascending virtual-electron count.  The costly walks then
// start first and the launch does not end waiting on a few late ones.  Only
// the schedule changes: a walker's chain depends on its own id.  One
// workgroup of 1024 threads, counting sort over the three counts: thread t
// takes walkers t, t + 1024, t + 2048, ... (coalesced, OB loads in flight), a
// scan of the per-thread counts gives each thread its output positions, so
// the order inside a count is fixed (by thread, then by walker).
__device__ __forceinline__ int virt_count(unsigned v) {
    return ((v & 0xFFFFu) != SCQ_NOVIRT) + ((v >> 16) != SCQ_NOVIRT);
}
#define OB 16
__device__ void order_walkers(const unsigned *virt, long long W, int *order) {
    __shared__ int sc[3][1024];
    int t = threadIdx.x;
    int c[3] = {0, 0, 0};
    for (long long i0 = t; i0 < W; i0 += 1024LL * OB) {
        unsigned v[OB];
#pragma unroll
        for (int k = 0; k < OB; k++) {
            long long i = i0 + 1024LL * k;
            v[k] = i < W ? virt[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < OB; k++)
            if (i0 + 1024LL * k < W) c[virt_count(v[k])]++;
    }
#pragma unroll
    for (int k = 0; k < 3; k++) sc[k][t] = c[k];
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int v[3];
#pragma unroll
        for (int k = 0; k < 3; k++) v[k] = t >= d ? sc[k][t - d] : 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 3; k++) sc[k][t] += v[k];
        __syncthreads();
    }
    int n0 = sc[0][1023], n1 = sc[1][1023];
    int base[3] = {sc[0][t] - c[0], n0 + sc[1][t] - c[1], n0 + n1 + sc[2][t] - c[2]};
    for (long long i0 = t; i0 < W; i0 += 1024LL * OB) {
        unsigned v[OB];
#pragma unroll
        for (int k = 0; k < OB; k++) {
            long long i = i0 + 1024LL * k;
            v[k] = i < W ? virt[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < OB; k++) {
            long long i = i0 + 1024LL * k;
            if (i < W) order[base[virt_count(v[k])]++] = (int)i;
        }
    }
}

// The single-system form also keeps L2 locality.  Workgroups are handed to
// the eight XCDs round-robin (slot s runs on XCD s mod 8) and each XCD has its
// own L2.  Inside each virtual-electron count the walkers are bucketed by
// their virtual spin-orbitals (the one, or the pair), and every XCD gets a
// contiguous run of that bucket order (its share of the count's slots, in
// order): the walkers an XCD holds at one time then share virtual orbitals,
// and with them most of the integrals they read.  The cost order is kept:
// counts still run in ascending order on every XCD.  Order inside a bucket
// follows LDS atomics, so it can differ between runs; results cannot.
#define NXCD 8
#define OB1 1024   // buckets of one-virtual walkers
#define OB2 8192   // buckets of two-virtual walkers
#define OBN 10240  // 1 + OB1 + OB2, rounded up to 10 per thread
__device__ __forceinline__ int order_key(unsigned v, int V2, int sh1, int sh2) {
    int c = virt_count(v);
    unsigned v0 = v & 0xFFFFu, v1 = v >> 16;
    if (c == 0) return 0;
    if (c == 1) return 1 + (int)(v0 >> sh1);
    return 1 + OB1 + (int)((v0 * (unsigned)V2 + v1) >> sh2);
}
__global__ __launch_bounds__(1024) void k_order(const unsigned *virt, long long W, int V, int *order) {
    __shared__ int hist[OBN];
    __shared__ int cur[OBN];
    __shared__ int tot[1024];
    int t = threadIdx.x;
    int V2 = 2 * V, sh1 = 0, sh2 = 0;
    while (((V2 - 1) >> sh1) >= OB1) sh1++;
    while ((((unsigned)V2 * (unsigned)V2 - 1u) >> sh2) >= (unsigned)OB2) sh2++;
    for (int k = t; k < OBN; k += 1024) hist[k] = 0;
    __syncthreads();
    for (long long i0 = t; i0 < W; i0 += 1024LL * OB) {
        unsigned v[OB];
#pragma unroll
        for (int k = 0; k < OB; k++) {
            long long i = i0 + 1024LL * k;
            v[k] = i < W ? virt[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < OB; k++)
            if (i0 + 1024LL * k < W) atomicAdd(&hist[order_key(v[k], V2, sh1, sh2)], 1);
    }
    __syncthreads();
    // exclusive scan of the bucket counts, ten per thread
    constexpr int PT = OBN / 1024;
    int a[PT], sum = 0;
#pragma unroll
    for (int k = 0; k < PT; k++) { a[k] = hist[PT * t + k]; sum += a[k]; }
    tot[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int x = t >= d ? tot[t - d] : 0;
        __syncthreads();
        tot[t] += x;
        __syncthreads();
    }
    int ex = tot[t] - sum;
#pragma unroll
    for (int k = 0; k < PT; k++) { cur[PT * t + k] = ex; ex += a[k]; }
    __syncthreads();
    // counts: 0 -> key 0, 1 -> keys [1, 1 + OB1), 2 -> [1 + OB1, OBN)
    int S[3] = {0, cur[1], cur[1 + OB1]};
    int n[3] = {cur[1], cur[1 + OB1] - cur[1], (int)W - cur[1 + OB1]};
    __syncthreads();
    for (long long i0 = t; i0 < W; i0 += 1024LL * OB) {
        unsigned v[OB];
#pragma unroll
        for (int k = 0; k < OB; k++) {
            long long i = i0 + 1024LL * k;
            v[k] = i < W ? virt[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < OB; k++) {
            long long i = i0 + 1024LL * k;
            if (i >= W) continue;
            int key = order_key(v[k], V2, sh1, sh2), c = virt_count(v[k]);
            int tc = atomicAdd(&cur[key], 1) - S[c];   // rank inside the count
            // XCD j owns the slots S_c + s' (0 <= s' < n_c) with (S_c + s') mod 8 = j:
            // s' = r_j + 8 q, r_j = (j - S_c) mod 8, q < m_j; ranks are dealt to
            // XCD 0, 1, ... in runs of m_j
            int start = 0, slot = -1;
#pragma unroll
            for (int j = 0; j < NXCD; j++) {
                int r = (j - S[c]) & (NXCD - 1);
                int m = n[c] > r ? (n[c] - r + NXCD - 1) / NXCD : 0;
                if (slot < 0 && tc < start + m) slot = S[c] + r + NXCD * (tc - start);
                start += m;
            }
            order[slot] = (int)i;
        }
    }
}

// order: walker of each workgroup slot (a permutation of 0..W-1)
template <class R>
__global__ __launch_bounds__(64 * WPB, 4) void k_sample(DevProblem P, WalkerArrays S, const int *order, long long W,
                                                   long long step0, int nsteps, long long burn_in, int NL) {
    extern __shared__ unsigned char smem[];
    int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    long long slot = (long long)blockIdx.x * WPB + wave;
    if (slot >= W) return;
    long long w = (long long)uni(order[slot]);
    WaveLDS L = carve(smem + wave * wave_lds_bytes(NL), NL);
    sample_walker<R>(P, S, W, w, step0, nsteps, burn_in, L, lane);
}

// ---------------------------------------------------------------------------
// Batched form: many independent systems (their own integrals, references,
// class tables and walkers) in one launch.  A schedule maps each workgroup
// slot to (system, walker); a walker's chain depends only on its own id and
// the system's step counter, so any schedule gives the same results as the
// systems walked one by one.
// ---------------------------------------------------------------------------
struct BatchSys {
    DevProblem P;
    WalkerArrays S;
    int *order;          // walker of each rank (k_order_batch)
    long long W;         // walkers of the system
    long long step0;     // global step index of its next step
    long long burn_in;
    int NL;              // list headers per group (LDS layout)
    int pad;
};

// every system's walker order (one workgroup per system)
__global__ __launch_bounds__(1024) void k_order_batch(const BatchSys *sys) {
    const BatchSys &B = sys[blockIdx.x];
    order_walkers(B.S.virt, B.W, B.order);
}

// slot -> (system, rank): the rank's walker comes from the system's order.
// NW walkers (waves) per workgroup and at least MINW waves per SIMD (the
// register budget the compiler works to) are the two kernel parameters the
// batched form's autotuner chooses among.
// The waves of a workgroup may walk walkers of different systems, whose LDS
// layouts differ in size: each wave's region starts at wave * wstride, wstride
// = the LDS of the largest layout of the batch.
template <class R, int NW, int MINW>
__global__ __launch_bounds__(64 * NW, MINW) void k_sample_batch(const BatchSys *sys, const int *slot_sys,
                                                              const int *slot_w, long long nslots, int nsteps,
                                                              unsigned wstride) {
    extern __shared__ unsigned char smem[];
    int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    long long slot = (long long)blockIdx.x * NW + wave;
    if (slot >= nslots) return;
    int s = uni(slot_sys[slot]);
    const BatchSys &B = sys[s];
    long long w = (long long)uni(B.order[slot_w[slot]]);
    DevProblem P = B.P;
    WalkerArrays S = B.S;
    int NL = uni(B.NL);
    WaveLDS L = carve(smem + wave * wstride, NL);
    long long Wn = (long long)uni((unsigned long long)B.W), st0 = (long long)uni((unsigned long long)B.step0);
    long long bi = (long long)uni((unsigned long long)B.burn_in);
    sample_walker<R>(P, S, Wn, w, st0, nsteps, bi, L, lane);
}

// Persistent form of the batched launch: a grid of about as many workgroups
// as the GPU holds at once, whose waves take work items -- bins of `bin`
// consecutive schedule slots -- from a device counter until the schedule is
// exhausted (every wave leaves at the first item past the end).  The slots
// are the same as in k_sample_batch; only the hand-out is dynamic.
template <class R>
__global__ __launch_bounds__(64 * WPB, 4) void k_sample_batch_queue(const BatchSys *sys, const int *slot_sys,
                                                               const int *slot_w, long long nslots, int nsteps,
                                                               unsigned *head, int bin) {
    extern __shared__ unsigned char smem[];
    int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    while (true) {
        unsigned it = 0;
        if (lane == 0) it = atomicAdd(head, 1u);
        it = uni((unsigned)__shfl((int)it, 0));
        long long s0 = (long long)it * bin;
        if (s0 >= nslots) break;
        long long s1 = min(nslots, s0 + (long long)bin);
        for (long long slot = s0; slot < s1; slot++) {
            int s = uni(slot_sys[slot]);
            const BatchSys &B = sys[s];
            long long w = (long long)uni(B.order[slot_w[slot]]);
            DevProblem P = B.P;
            WalkerArrays S = B.S;
            int NL = uni(B.NL);
            WaveLDS L = carve(smem + wave * wave_lds_bytes(NL), NL);
            long long Wn = (long long)uni((unsigned long long)B.W), st0 = (long long)uni((unsigned long long)B.step0);
            long long bi = (long long)uni((unsigned long long)B.burn_in);
            sample_walker<R>(P, S, Wn, w, st0, nsteps, bi, L, lane);
            __syncwarp();
        }
    }
}

// step counters of every system advance after a batched launch (kept on the
// device so that a captured graph of launches can be replayed as is); the
// work counter of the persistent form is cleared for the next launch
__global__ void k_batch_advance(BatchSys *sys, int nsys, int nsteps, unsigned *head) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsys) sys[s].step0 += nsteps;
    if (s == 0 && head) *head = 0u;
}

// local energies without moving (parity / snapshots).  Grid-stride over the
// determinants: wave slot q takes q, q + slots, ...; its Fock table (ftab,
// null: none) is slot q's, so a launch needs tables for its slots only and
// the results do not depend on the grid.
template <class R>
__global__ __launch_bounds__(64 * WPB, 4) void k_eval(DevProblem P, const unsigned long long *keys, const unsigned *virts,
                                                 const int *valid, long long n, int NL, double *eloc, double *psi_out,
                                                 double *gamma, double *elocd, int *cls_out, double *ftab) {
    extern __shared__ unsigned char smem[];
    int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    long long q = (long long)blockIdx.x * WPB + wave, nslot = (long long)gridDim.x * WPB;
    WaveLDS L = carve(smem + wave * wave_lds_bytes(NL), NL);
    double *ft = ftab ? ftab + q * (2LL * P.A * P.V) : nullptr;
    for (long long i = q; i < n; i += nslot) {
        unsigned long long key = keys[i];
        unsigned virt = virts[i];
        int nv = ((virt & 0xFFFFu) != SCQ_NOVIRT) + ((virt >> 16) != SCQ_NOVIRT);
        double ps = 0.0;
        // psi(n) itself in FP64 in both forms: it divides every term of E_L
        if (lane == 0 && valid[i]) ps = psi_direct<double>(P, key, virt);
        ps = __shfl(ps, 0);
        EvalOut o;
        if (ps != 0.0) {
            walker_eval<false, R>(P, L, lane, key, virt, ps, (uint32_t)i, 0u, ft, o);
        } else {
            o.eloc = o.elocd = o.gamma = NAN;
        }
        if (lane == 0) {
            if (eloc) eloc[i] = o.eloc;
            if (psi_out) psi_out[i] = ps;
            if (gamma) gamma[i] = o.gamma;
            if (elocd) elocd[i] = (P.mode == 1 && nv > 0) ? o.elocd : NAN;
            if (cls_out) cls_out[i] = valid[i] ? (int)class_of_virt(P, virt) : -1;
        }
        __syncwarp();
    }
}

// psi of walkers (initialisation)
template <class R>
__global__ void k_psi(DevProblem P, const unsigned long long *keys, const unsigned *virts, long long n, double *psi) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    psi[i] = psi_direct<double>(P, keys[i], virts[i]);
}

// neighbour list of one walker (debug): one wave, groups and rows one lane at a time
__global__ __launch_bounds__(64) void k_neighbors(DevProblem P, unsigned long long key, unsigned virt, int NL,
                                                  long long cap, unsigned long long *okey, unsigned *ovirt,
                                                  signed char *ophase, double *ohnm, double *opsi,
                                                  unsigned long long *count) {
    extern __shared__ unsigned char smem[];
    int lane = threadIdx.x & 63;
    WaveLDS L = carve(smem, NL);
    WalkerCtx W;
    walker_setup(P, L, lane, key, virt, W);
    for (int rk = 0; rk < 6; rk++)
        for (int pk = 0; pk < 6; pk++) {
            Block b;
            if (!block_setup(P, W, rk, pk, b)) continue;
            int vp = b.vp[0] + b.vp[1];
            GroupInfo &mg = L.G[lane];
            uint2 *mlst = L.lst + lane * L.NL;
            for (unsigned gb = 0; gb < b.ng; gb += WAVE) {
                unsigned g = gb + (unsigned)lane;
                if (g < b.ng) {
                    group_setup(P, W, L, b, g, mg, mlst);
                    for (unsigned r = 0; r < b.R; r++) {
                        RowDec d;
                        row_decode(P, W, b, r, d);
                        RowRes o;
                        GroupView gv = group_view<false>(L, lane);
                        row_eval_any<false, double>(P, W, L, vp, d, gv, vec_ents_off(), o);
                        if (!o.ok) continue;
                        unsigned long long pos = atomicAdd(count, 1ull);
                        if ((long long)pos < cap) {
                            okey[pos] = mg.xkey;
                            ovirt[pos] = (d.Lp0 >= 0 ? (unsigned)d.Lp0 : SCQ_NOVIRT) |
                                         ((d.Lp1 >= 0 ? (unsigned)d.Lp1 : SCQ_NOVIRT) << 16);
                            ophase[pos] = (signed char)(o.phase > 0 ? 1 : -1);
                            ohnm[pos] = o.hnm;
                            opsi[pos] = o.psi;
                        }
                    }
                }
                __syncwarp();
            }
        }
}

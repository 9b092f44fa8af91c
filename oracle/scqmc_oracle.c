/*
 * scqmc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the local
 * energy and continuous-time walk of stochastic strongly contracted MRCI /
 * NEVPT2 (Mahajan, Blunt, Sabzevari, Sharma, "Multireference configuration
 * interaction and perturbation theory without reduced density matrices",
 * arXiv:1909.06935).  It exists to check the HIP path and nothing else: only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code with the GPU library.
 *
 * What it follows (section / equation of the paper):
 *  - the walker overlap with the SC wave function, Theory "SC-MRCI(s)",
 *    eq:ovlp and the overlap equation after it: psi(n) = c0 phi0(n) in the
 *    active space, c_{l_n} <n|H|phi0> outside it;
 *  - the local energy eq:locE (read with the sum over m, including m = n);
 *  - section "Implementation": neighbours m are generated from n and only
 *    those with at most two virtual electrons are kept; for m outside the
 *    active space the excitations of m that land back in the active space
 *    are generated and looked up in the reference; the reference lookup is a
 *    binary search over a sorted array (the paper uses a hash table; a
 *    different algorithm is used here on purpose);
 *  - the rejection-free continuous-time walk (BKL / Gillespie, cited in
 *    "SC-MRCI(s)"): rates |psi(m)/psi(n)|, residence weight 1/sum of rates,
 *    next state by the first-reaction method, two levels: first among the
 *    groups of neighbours sharing an active-space part, then within the
 *    winning group;
 *  - Dyall's Hamiltonian of section "SC-NEVPT2(s)" for the NEVPT2 local
 *    energy used by eq:nevpt.
 *
 * Every Hamiltonian matrix element goes through one generic Slater-Condon
 * routine over ALL occupied spin-orbitals, core included (no core folding).
 * Sums of many terms use Neumaier's compensated summation.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written from its published definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXW 4          /* words per spin string: N <= 256 */
#define MAXE 128        /* non-core spin-orbitals listed per determinant */

typedef struct {
    int N, C, A, V, na, nb, W;
    double e_const;
    double *h1;          /* [N*N] */
    double *eri;         /* [N^4] chemist (pq|rs) */
    int64_t n_ref;
    uint64_t *ref;       /* [n_ref][2W] sorted lexicographically (see cmp_det) */
    double *ref_c;
    double c0;
    double *c_cls;       /* [n_cls-1] */
    int64_t n_cls;
    double *eps_v;       /* [V] or NULL */
    double e0;
    double eps_screen;
    int mode;            /* 0 = MRCI local energy, 1 = also Dyall local energy */
} orc_t;

/* ------------------------------------------------------------------ */
/* Neumaier compensated sum                                            */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                        */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Exponential variate for the first-reaction method.  Counter
 * (walker, step | level<<31, a, b), key = seed.  The 53-bit integer k is
 * taken from the first two output words, U = (k+1) 2^-53 in (0,1],
 * E = -log(U). */
double orc_exp_draw(uint64_t seed, uint32_t walker, uint32_t step, uint32_t level, uint32_t a, uint32_t b) {
    uint32_t ctr[4] = {walker, (step & 0x7fffffffu) | (level << 31), a, b};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    uint64_t k = ((((uint64_t)o[0]) << 32) | (uint64_t)o[1]) >> 11;
    double u = (double)(k + 1) * 0x1.0p-53;
    return -log(u);
}

/* ------------------------------------------------------------------ */
/* determinants                                                        */
/* ------------------------------------------------------------------ */
/* spin-orbital g = p + sigma*N; global order: all alpha then all beta */
static inline int bit(const orc_t *o, const uint64_t *d, int g) {
    int s = g / o->N, p = g % o->N;
    return (int)((d[s * o->W + (p >> 6)] >> (p & 63)) & 1ull);
}
static inline void flip(const orc_t *o, uint64_t *d, int g) {
    int s = g / o->N, p = g % o->N;
    d[s * o->W + (p >> 6)] ^= 1ull << (p & 63);
}
/* number of occupied spin-orbitals with global index below g */
static int below(const orc_t *o, const uint64_t *d, int g) {
    int s = g / o->N, p = g % o->N, c = 0;
    if (s == 1)
        for (int w = 0; w < o->W; w++) c += __builtin_popcountll(d[w]);      /* every alpha electron */
    for (int w = 0; w < (p >> 6); w++) c += __builtin_popcountll(d[s * o->W + w]);
    if (p & 63) c += __builtin_popcountll(d[s * o->W + (p >> 6)] & ((1ull << (p & 63)) - 1ull));
    return c;
}
static int cmp_det(const orc_t *o, const uint64_t *a, const uint64_t *b) {
    /* lexicographic with the last word most significant */
    for (int w = 2 * o->W - 1; w >= 0; w--) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}
/* reference coefficient phi0(d) by binary search; 0 when absent */
static double ref_lookup(const orc_t *o, const uint64_t *d) {
    int64_t lo = 0, hi = o->n_ref - 1;
    int W2 = 2 * o->W;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = cmp_det(o, o->ref + mid * W2, d);
        if (c == 0) return o->ref_c[mid];
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}
static inline int spin(const orc_t *o, int g) { return g / o->N; }
static inline int orb(const orc_t *o, int g) { return g % o->N; }
static inline int is_core(const orc_t *o, int g) { return orb(o, g) < o->C; }
static inline int is_act(const orc_t *o, int g) { int p = orb(o, g); return p >= o->C && p < o->C + o->A; }
static inline int is_virt(const orc_t *o, int g) { return orb(o, g) >= o->C + o->A; }

static inline double eri(const orc_t *o, int p, int q, int r, int s) {
    size_t N = (size_t)o->N;
    return o->eri[((p * N + q) * N + r) * N + s];
}
/* spin-orbital chemist integral (PQ|RS) */
static inline double seri(const orc_t *o, int P, int Q, int R, int S) {
    if (spin(o, P) != spin(o, Q) || spin(o, R) != spin(o, S)) return 0.0;
    return eri(o, orb(o, P), orb(o, Q), orb(o, R), orb(o, S));
}

static int n_virt_el(const orc_t *o, const uint64_t *d) {
    int c = 0;
    for (int s = 0; s < 2; s++)
        for (int p = o->C + o->A; p < o->N; p++) c += bit(o, d, p + s * o->N);
    return c;
}
static int core_full(const orc_t *o, const uint64_t *d) {
    for (int s = 0; s < 2; s++)
        for (int p = 0; p < o->C; p++) if (!bit(o, d, p + s * o->N)) return 0;
    return 1;
}
/* class id of the strongly contracted subspace holding d */
static int64_t class_of(const orc_t *o, const uint64_t *d) {
    int s[2], k = 0, V = o->V;
    for (int sg = 0; sg < 2; sg++)
        for (int a = 0; a < V; a++)
            if (bit(o, d, o->C + o->A + a + sg * o->N)) { if (k < 2) s[k] = a + sg * V; k++; }
    if (k == 0) return 0;
    if (k == 1) return 1 + s[0];
    if (k > 2) return -1;
    int64_t V2 = 2 * V, s1 = s[0], s2 = s[1];
    return 1 + V2 + s1 * V2 - s1 * (s1 + 1) / 2 + (s2 - s1 - 1);
}
static double class_coeff(const orc_t *o, int64_t cls) {
    if (cls == 0) return o->c0;
    return o->c_cls[cls - 1];
}
/* key of the active part: active alpha bits | active beta bits << 32 */
static uint64_t active_key(const orc_t *o, const uint64_t *d) {
    uint64_t k = 0;
    for (int s = 0; s < 2; s++)
        for (int t = 0; t < o->A; t++)
            if (bit(o, d, o->C + t + s * o->N)) k |= 1ull << (t + 32 * s);
    return k;
}

/* ------------------------------------------------------------------ */
/* Slater-Condon: <a|H|b> over all occupied spin-orbitals               */
/* ------------------------------------------------------------------ */
/* Returns the matrix element.  *phase receives the sign of the operator
 * string (single: <a|a+_Q a_P|b>; double with P1<P2 removed from b and
 * Q1<Q2 added: <a|a+_Q1 a+_Q2 a_P2 a_P1|b>; diagonal: +1); *nexc receives
 * the excitation level (0, 1, 2, or 3 meaning "more than two"). */
double orc_hmat(const orc_t *o, const uint64_t *a, const uint64_t *b, int *phase, int *nexc) {
    int N2 = 2 * o->N;
    int rem[3], add[3], nr = 0, na = 0;
    for (int s = 0; s < 2; s++)
        for (int w = 0; w < o->W; w++) {
            uint64_t x = a[s * o->W + w] ^ b[s * o->W + w];
            while (x) {
                int i = __builtin_ctzll(x);
                x &= x - 1;
                int g = 64 * w + i + s * o->N;
                if (bit(o, b, g)) { if (nr < 3) rem[nr] = g; nr++; }
                else { if (na < 3) add[na] = g; na++; }
            }
        }
    if (phase) *phase = 1;
    if (nr != na || nr > 2) { if (nexc) *nexc = 3; return 0.0; }
    if (nexc) *nexc = nr;
    if (nr == 0) {
        nsum acc = {o->e_const, 0.0};
        for (int i = 0; i < N2; i++) {
            if (!bit(o, b, i)) continue;
            nadd(&acc, o->h1[orb(o, i) * o->N + orb(o, i)]);
            for (int j = 0; j < N2; j++) {
                if (!bit(o, b, j)) continue;
                nadd(&acc, 0.5 * (seri(o, i, i, j, j) - seri(o, i, j, j, i)));
            }
        }
        return nval(&acc);
    }
    uint64_t t[2 * MAXW];
    memcpy(t, b, sizeof(uint64_t) * 2 * o->W);
    if (nr == 1) {
        int P = rem[0], Q = add[0];
        if (spin(o, P) != spin(o, Q)) return 0.0;
        int sg = below(o, t, P);
        flip(o, t, P);
        sg += below(o, t, Q);
        int ph = (sg & 1) ? -1 : 1;
        if (phase) *phase = ph;
        nsum acc = {o->h1[orb(o, Q) * o->N + orb(o, P)], 0.0};
        for (int J = 0; J < N2; J++) {
            if (!bit(o, b, J) || J == P) continue;
            nadd(&acc, seri(o, Q, P, J, J) - seri(o, Q, J, J, P));
        }
        return ph * nval(&acc);
    }
    /* double: remove P1 < P2 from b, add Q1 < Q2 */
    int P1 = rem[0], P2 = rem[1], Q1 = add[0], Q2 = add[1];
    int sg = 0;
    sg += below(o, t, P1); flip(o, t, P1);
    sg += below(o, t, P2); flip(o, t, P2);
    sg += below(o, t, Q2); flip(o, t, Q2);
    sg += below(o, t, Q1); flip(o, t, Q1);
    int ph = (sg & 1) ? -1 : 1;
    if (phase) *phase = ph;
    return ph * (seri(o, Q1, P1, Q2, P2) - seri(o, Q1, P2, Q2, P1));
}

/* strip the virtual electrons of d (the determinant seen by Dyall's H_0) */
static void strip_virtual(const orc_t *o, const uint64_t *d, uint64_t *out) {
    memcpy(out, d, sizeof(uint64_t) * 2 * o->W);
    for (int s = 0; s < 2; s++)
        for (int p = o->C + o->A; p < o->N; p++)
            if (bit(o, out, p + s * o->N)) flip(o, out, p + s * o->N);
}

/* ------------------------------------------------------------------ */
/* overlap with the SC wave function (eq:ovlp)                          */
/* ------------------------------------------------------------------ */
/* psi(m); *absum receives the sum of the magnitudes of the terms summed
 * (|psi(m)| itself in the active space), which bounds its rounding error. */
static double psi_abs(const orc_t *o, const uint64_t *m, double *absum) {
    *absum = 0.0;
    if (!core_full(o, m)) return 0.0;
    int nv = n_virt_el(o, m);
    if (nv > 2) return 0.0;
    int64_t cls = class_of(o, m);
    if (nv == 0) { double v = o->c0 * ref_lookup(o, m); *absum = fabs(v); return v; }
    /* <m|H|phi0> = sum over active-space determinants d reached from m by
     * moving every virtual electron of m into an active hole */
    int N2 = 2 * o->N;
    int vir[2], nvir = 0, occa[MAXE], nocca = 0, hol[MAXE], nhol = 0;
    for (int g = 0; g < N2; g++) {
        if (is_virt(o, g) && bit(o, m, g)) vir[nvir++] = g;
        if (is_act(o, g)) { if (bit(o, m, g)) occa[nocca++] = g; else hol[nhol++] = g; }
    }
    nsum acc = {0.0, 0.0}, ab = {0.0, 0.0};
    uint64_t d[2 * MAXW];
    if (nv == 1) {
        int X = vir[0];
        /* singles X -> T */
        for (int i = 0; i < nhol; i++) {
            int T = hol[i];
            if (spin(o, T) != spin(o, X)) continue;
            memcpy(d, m, sizeof(uint64_t) * 2 * o->W);
            flip(o, d, X); flip(o, d, T);
            double c = ref_lookup(o, d);
            if (c != 0.0) { double t = orc_hmat(o, m, d, NULL, NULL) * c; nadd(&acc, t); nadd(&ab, fabs(t)); }
        }
        /* doubles (X, R) -> {T, S}, R occupied active, T != S active holes */
        for (int r = 0; r < nocca; r++) {
            int R = occa[r];
            for (int i = 0; i < nhol; i++)
                for (int j = i + 1; j < nhol; j++) {
                    int T = hol[i], S = hol[j];
                    int s1 = spin(o, T) + spin(o, S), s0 = spin(o, X) + spin(o, R);
                    if (s1 != s0) continue;
                    memcpy(d, m, sizeof(uint64_t) * 2 * o->W);
                    flip(o, d, X); flip(o, d, R); flip(o, d, T); flip(o, d, S);
                    double c = ref_lookup(o, d);
                    if (c != 0.0) { double t = orc_hmat(o, m, d, NULL, NULL) * c; nadd(&acc, t); nadd(&ab, fabs(t)); }
                }
        }
    } else {
        int X = vir[0], Y = vir[1];
        for (int i = 0; i < nhol; i++)
            for (int j = i + 1; j < nhol; j++) {
                int T = hol[i], S = hol[j];
                if (spin(o, T) + spin(o, S) != spin(o, X) + spin(o, Y)) continue;
                memcpy(d, m, sizeof(uint64_t) * 2 * o->W);
                flip(o, d, X); flip(o, d, Y); flip(o, d, T); flip(o, d, S);
                double c = ref_lookup(o, d);
                if (c != 0.0) { double t = orc_hmat(o, m, d, NULL, NULL) * c; nadd(&acc, t); nadd(&ab, fabs(t)); }
            }
    }
    double c = class_coeff(o, cls);
    *absum = fabs(c) * nval(&ab);
    return c * nval(&acc);
}

double orc_psi(const orc_t *o, const uint64_t *m) {
    double a;
    return psi_abs(o, m, &a);
}

/* ------------------------------------------------------------------ */
/* neighbour enumeration: every single and double over non-core        */
/* spin-orbitals whose result has at most two virtual electrons        */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t det[2 * MAXW];
    double h;       /* <n|H|m> ... stored as <m|H|n> (real symmetric) */
    int phase;
    double psi;
    double absum;   /* sum of |terms| of psi(m) */
    double hd;      /* <n|H_D|m> if m has the same virtual occupation, else 0 */
    int same_cls;
    uint64_t key;   /* active key of m */
    int64_t cls;
} nbr_t;

typedef struct { nbr_t *v; int64_t n, cap; } nbr_list;
static void nbr_push(nbr_list *L, const nbr_t *x) {
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->v = (nbr_t *)realloc(L->v, sizeof(nbr_t) * L->cap);
    }
    L->v[L->n++] = *x;
}

static void consider(const orc_t *o, const uint64_t *n, uint64_t *m, int is_double, int64_t ncls, nbr_list *L) {
    if (n_virt_el(o, m) > 2) return;
    nbr_t x;
    memcpy(x.det, m, sizeof(uint64_t) * 2 * o->W);
    int ph, ne;
    x.h = orc_hmat(o, m, n, &ph, &ne);
    x.phase = ph;
    if (is_double && o->eps_screen > 0.0 && !(fabs(x.h) > o->eps_screen)) return;
    x.psi = psi_abs(o, m, &x.absum);
    x.cls = class_of(o, m);
    x.key = active_key(o, m);
    x.same_cls = (x.cls == ncls);
    x.hd = 0.0;
    if (x.same_cls && ncls != 0) {
        uint64_t sa[2 * MAXW], sb[2 * MAXW];
        strip_virtual(o, m, sa);
        strip_virtual(o, n, sb);
        x.hd = orc_hmat(o, sa, sb, NULL, NULL);
    }
    nbr_push(L, &x);
}

static void enumerate(const orc_t *o, const uint64_t *n, nbr_list *L) {
    int N2 = 2 * o->N;
    int occ[MAXE], no = 0, emp[2 * 256], ne = 0;
    for (int g = 0; g < N2; g++) {
        if (is_core(o, g)) continue;
        if (bit(o, n, g)) occ[no++] = g; else emp[ne++] = g;
    }
    int64_t ncls = class_of(o, n);
    uint64_t m[2 * MAXW];
    for (int i = 0; i < no; i++)
        for (int a = 0; a < ne; a++) {
            if (spin(o, occ[i]) != spin(o, emp[a])) continue;
            memcpy(m, n, sizeof(uint64_t) * 2 * o->W);
            flip(o, m, occ[i]); flip(o, m, emp[a]);
            consider(o, n, m, 0, ncls, L);
        }
    for (int i = 0; i < no; i++)
        for (int j = i + 1; j < no; j++)
            for (int a = 0; a < ne; a++)
                for (int b = a + 1; b < ne; b++) {
                    if (spin(o, occ[i]) + spin(o, occ[j]) != spin(o, emp[a]) + spin(o, emp[b])) continue;
                    memcpy(m, n, sizeof(uint64_t) * 2 * o->W);
                    flip(o, m, occ[i]); flip(o, m, occ[j]); flip(o, m, emp[a]); flip(o, m, emp[b]);
                    consider(o, n, m, 1, ncls, L);
                }
}

/* ------------------------------------------------------------------ */
/* one walker: local energies and rates                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    double eloc, eloc_d, psi, gamma, sabs, kappa;
    int64_t cls;
    int ok;
} eval_t;

static void eval_walker(const orc_t *o, const uint64_t *n, nbr_list *L, eval_t *e) {
    L->n = 0;
    double an;
    e->psi = psi_abs(o, n, &an);
    e->kappa = e->psi != 0.0 ? an / fabs(e->psi) : NAN;
    e->cls = class_of(o, n);
    e->ok = (e->psi != 0.0);
    enumerate(o, n, L);
    double hnn = orc_hmat(o, n, n, NULL, NULL);
    nsum s = {0, 0}, g = {0, 0}, sa = {0, 0}, sd = {0, 0};
    for (int64_t k = 0; k < L->n; k++) {
        nbr_t *x = &L->v[k];
        nadd(&s, x->h * x->psi);
        nadd(&sa, fabs(x->h) * x->absum);
        if (x->same_cls && e->cls != 0) nadd(&sd, x->hd * x->psi);
    }
    e->eloc = e->ok ? hnn + nval(&s) / e->psi : NAN;
    e->sabs = e->ok ? fabs(hnn) + nval(&sa) / fabs(e->psi) : NAN;
    /* rates */
    for (int64_t k = 0; k < L->n; k++) nadd(&g, fabs(L->v[k].psi));
    e->gamma = e->ok ? nval(&g) / fabs(e->psi) : NAN;
    e->eloc_d = NAN;
    if (o->mode == 1 && e->cls != 0 && e->ok && o->eps_v) {
        uint64_t sn[2 * MAXW];
        strip_virtual(o, n, sn);
        double hd = orc_hmat(o, sn, sn, NULL, NULL);
        for (int a = 0; a < o->V; a++)
            for (int sg = 0; sg < 2; sg++)
                if (bit(o, n, o->C + o->A + a + sg * o->N)) hd += o->eps_v[a];
        e->eloc_d = hd + nval(&sd) / e->psi;
    }
}

static int cmp_key_cls(const void *pa, const void *pb) {
    const nbr_t *a = (const nbr_t *)pa, *b = (const nbr_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->cls != b->cls) return a->cls < b->cls ? -1 : 1;
    return 0;
}

/* Next state by the two-level first-reaction method.  Returns the index of
 * the chosen neighbour in L (after L has been sorted by (key, class)), or -1
 * when every rate is zero. */
static int64_t select_next(const orc_t *o, nbr_list *L, double psin, uint64_t seed, uint32_t wid, uint32_t step) {
    qsort(L->v, (size_t)L->n, sizeof(nbr_t), cmp_key_cls);
    double best = INFINITY;
    int64_t bstart = -1, bend = -1;
    int64_t i = 0;
    while (i < L->n) {
        int64_t j = i;
        nsum g = {0, 0};
        while (j < L->n && L->v[j].key == L->v[i].key) { nadd(&g, fabs(L->v[j].psi / psin)); j++; }
        double G = nval(&g);
        if (G > 0.0) {
            uint64_t key = L->v[i].key;
            double tau = orc_exp_draw(seed, wid, step, 0, (uint32_t)key, (uint32_t)(key >> 32)) / G;
            if (tau < best) { best = tau; bstart = i; bend = j; }   /* ties: smaller key (first) wins */
        }
        i = j;
    }
    if (bstart < 0) return -1;
    double bt = INFINITY;
    int64_t pick = -1;
    for (int64_t k = bstart; k < bend; k++) {
        double r = fabs(L->v[k].psi / psin);
        if (!(r > 0.0)) continue;
        double tau = orc_exp_draw(seed, wid, step, 1, (uint32_t)L->v[k].cls, 0) / r;
        if (tau < bt) { bt = tau; pick = k; }
    }
    return pick;
}

/* ------------------------------------------------------------------ */
/* public API                                                          */
/* ------------------------------------------------------------------ */
orc_t *orc_create(int n_orb, int n_core, int n_act, int n_a, int n_b) {
    if (n_orb <= 0 || n_orb > 64 * MAXW || n_core < 0 || n_act <= 0 || n_act > 32) return NULL;
    if (n_core + n_act > n_orb) return NULL;
    if (2 * (n_orb - n_core) > 2 * 256 || n_a - n_core + n_b - n_core > MAXE) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->N = n_orb; o->C = n_core; o->A = n_act; o->V = n_orb - n_core - n_act;
    o->na = n_a; o->nb = n_b; o->W = (n_orb + 63) / 64;
    o->n_cls = 1 + 2 * (int64_t)o->V + (2 * (int64_t)o->V) * (2 * (int64_t)o->V - 1) / 2;
    o->c0 = 1.0;
    return o;
}

void orc_destroy(orc_t *o) {
    if (!o) return;
    free(o->h1); free(o->eri); free(o->ref); free(o->ref_c); free(o->c_cls); free(o->eps_v);
    free(o);
}

int64_t orc_n_classes(const orc_t *o) { return o->n_cls; }

int orc_set_integrals(orc_t *o, const double *h1, const double *eri4, double e_const) {
    size_t N = (size_t)o->N;
    free(o->h1); free(o->eri);
    o->h1 = (double *)malloc(sizeof(double) * N * N);
    o->eri = (double *)malloc(sizeof(double) * N * N * N * N);
    if (!o->h1 || !o->eri) return -4;
    memcpy(o->h1, h1, sizeof(double) * N * N);
    memcpy(o->eri, eri4, sizeof(double) * N * N * N * N);
    o->e_const = e_const;
    return 0;
}

/* (pq|rs) = sum_L B_pq B_rs computed here, for problems given in Cholesky form */
int orc_set_integrals_chol(orc_t *o, const double *h1, const double *B, int n_chol, double e_const) {
    size_t N = (size_t)o->N, N2 = N * N;
    free(o->h1); free(o->eri);
    o->h1 = (double *)malloc(sizeof(double) * N2);
    o->eri = (double *)malloc(sizeof(double) * N2 * N2);
    if (!o->h1 || !o->eri) return -4;
    memcpy(o->h1, h1, sizeof(double) * N2);
    #pragma omp parallel for schedule(static)
    for (int64_t pq = 0; pq < (int64_t)N2; pq++)
        for (size_t rs = 0; rs < N2; rs++) {
            double s = 0.0;
            for (int L = 0; L < n_chol; L++) s += B[L * N2 + pq] * B[L * N2 + rs];
            o->eri[pq * N2 + rs] = s;
        }
    o->e_const = e_const;
    return 0;
}

int orc_set_reference(orc_t *o, int64_t n, const uint64_t *dets, const double *coeff) {
    int W2 = 2 * o->W;
    free(o->ref); free(o->ref_c);
    o->ref = (uint64_t *)malloc(sizeof(uint64_t) * W2 * (n > 0 ? n : 1));
    o->ref_c = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    memcpy(o->ref, dets, sizeof(uint64_t) * W2 * n);
    memcpy(o->ref_c, coeff, sizeof(double) * n);
    o->n_ref = n;
    for (int64_t i = 1; i < n; i++)   /* must be sorted and unique */
        if (cmp_det(o, o->ref + (i - 1) * W2, o->ref + i * W2) >= 0) return -1;
    return 0;
}

int orc_set_coeffs(orc_t *o, double c0, const double *c_cls, int64_t n) {
    if (n != o->n_cls - 1) return -1;
    free(o->c_cls);
    o->c_cls = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    memcpy(o->c_cls, c_cls, sizeof(double) * n);
    o->c0 = c0;
    return 0;
}

int orc_set_dyall(orc_t *o, const double *eps_v, double e0) {
    free(o->eps_v);
    o->eps_v = (double *)malloc(sizeof(double) * (o->V > 0 ? o->V : 1));
    memcpy(o->eps_v, eps_v, sizeof(double) * o->V);
    o->e0 = e0;
    return 0;
}

void orc_set_options(orc_t *o, double eps_screen, int mode) { o->eps_screen = eps_screen; o->mode = mode; }

double orc_hmat_pub(const orc_t *o, const uint64_t *a, const uint64_t *b, int *phase, int *nexc) {
    return orc_hmat(o, a, b, phase, nexc);
}

int64_t orc_class_of(const orc_t *o, const uint64_t *d) { return class_of(o, d); }
double orc_ref_lookup(const orc_t *o, const uint64_t *d) { return ref_lookup(o, d); }

/* Neighbour list of one determinant (the set M(n)).  Writes at most cap
 * entries; returns the total count.  Dyall elements are written to hd_out
 * (0 where m has another virtual occupation). */
int64_t orc_neighbors(const orc_t *o, const uint64_t *det, int64_t cap, uint64_t *out_dets, int8_t *out_phase,
                      double *out_h, double *out_psi, double *out_hd, int64_t *out_cls) {
    nbr_list L = {0, 0, 0};
    enumerate(o, det, &L);
    int W2 = 2 * o->W;
    for (int64_t k = 0; k < L.n && k < cap; k++) {
        if (out_dets) memcpy(out_dets + k * W2, L.v[k].det, sizeof(uint64_t) * W2);
        if (out_phase) out_phase[k] = (int8_t)L.v[k].phase;
        if (out_h) out_h[k] = L.v[k].h;
        if (out_psi) out_psi[k] = L.v[k].psi;
        if (out_hd) out_hd[k] = L.v[k].hd;
        if (out_cls) out_cls[k] = L.v[k].cls;
    }
    int64_t n = L.n;
    free(L.v);
    return n;
}

/* Local energies of a batch of determinants (no move). */
/* sabs[i] = (|H_nn psi(n)| + sum_m |H_nm| A(m)) / |psi(n)| with A(m) the sum
 * of |terms| of psi(m); kappa[i] = A(n) / |psi(n)|.  Together they bound the
 * rounding any summation order can leave in E_L. */
int orc_eval(const orc_t *o, int64_t n, const uint64_t *dets, double *eloc, double *psi, double *gamma,
             double *eloc_d, int64_t *cls, double *sabs, double *kappa, int nthreads) {
    int W2 = 2 * o->W;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    #pragma omp parallel
    {
        nbr_list L = {0, 0, 0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; i++) {
            eval_t e;
            eval_walker(o, dets + i * W2, &L, &e);
            if (eloc) eloc[i] = e.eloc;
            if (psi) psi[i] = e.psi;
            if (gamma) gamma[i] = e.gamma;
            if (eloc_d) eloc_d[i] = e.eloc_d;
            if (cls) cls[i] = e.cls;
            if (sabs) sabs[i] = e.sabs;
            if (kappa) kappa[i] = e.kappa;
        }
        free(L.v);
    }
    return 0;
}

/* Continuous-time walk of W walkers for n_steps steps, starting at global
 * step index step0.  wid0 is the global id of the first walker.  After
 * burn_in (global step index), accumulates per walker
 *   wsum[w] += {t, t*E_L, t*[class 0]}
 * and per class l
 *   csum[l] += {t, t*E_L, t/c_l^2, t*E_D,L/c_l^2}
 * with t = 1/Gamma.  dets are updated in place, psi_out receives psi(n)
 * of the final walkers.  Returns the number of walker-steps whose rates
 * were all zero (such walkers stay put and accumulate nothing). */
int64_t orc_run(const orc_t *o, int64_t W, uint64_t *dets, double *psi_out, uint64_t seed, int64_t step0,
                int64_t n_steps, int64_t burn_in, int64_t wid0, double *wsum, double *csum, int nthreads) {
    int W2 = 2 * o->W;
    int64_t stuck = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int nt = omp_get_max_threads();
#else
    int nt = 1;
#endif
    double *part = (double *)calloc((size_t)nt * o->n_cls * 4, sizeof(double));
    #pragma omp parallel reduction(+:stuck)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *mycs = part + (size_t)tid * o->n_cls * 4;
        nbr_list L = {0, 0, 0};
        #pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < W; w++) {
            uint64_t *n = dets + w * W2;
            double last_psi = 0.0;
            for (int64_t st = step0; st < step0 + n_steps; st++) {
                eval_t e;
                eval_walker(o, n, &L, &e);
                last_psi = e.psi;
                if (!e.ok || !(e.gamma > 0.0)) { stuck++; continue; }
                double t = 1.0 / e.gamma;
                if (st >= burn_in) {
                    wsum[w * 3 + 0] += t;
                    wsum[w * 3 + 1] += t * e.eloc;
                    wsum[w * 3 + 2] += (e.cls == 0) ? t : 0.0;
                    double c = class_coeff(o, e.cls);
                    double *cs = mycs + e.cls * 4;
                    cs[0] += t;
                    cs[1] += t * e.eloc;
                    cs[2] += t / (c * c);
                    if (o->mode == 1 && e.cls != 0) cs[3] += t * e.eloc_d / (c * c);
                }
                int64_t k = select_next(o, &L, e.psi, seed, (uint32_t)(wid0 + w), (uint32_t)st);
                if (k < 0) { stuck++; continue; }
                memcpy(n, L.v[k].det, sizeof(uint64_t) * W2);
                last_psi = L.v[k].psi;
            }
            if (psi_out) psi_out[w] = last_psi;
        }
        free(L.v);
    }
    for (int t = 0; t < nt; t++)
        for (int64_t i = 0; i < o->n_cls * 4; i++) csum[i] += part[(size_t)t * o->n_cls * 4 + i];
    free(part);
    return stuck;
}

/* Hamiltonian over a list of determinants (COO, upper triangle incl.
 * diagonal); used to solve for the active-space ground state.  Returns the
 * number of nonzeros (entries beyond cap are counted, not written). */
int64_t orc_det_hamiltonian(const orc_t *o, int64_t n, const uint64_t *dets, int64_t cap, int64_t *rows,
                            int64_t *cols, double *vals) {
    int W2 = 2 * o->W;
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i; j < n; j++) {
            int ne;
            double h = orc_hmat(o, dets + i * W2, dets + j * W2, NULL, &ne);
            if (ne > 2 || h == 0.0) continue;
            if (nnz < cap) { rows[nnz] = i; cols[nnz] = j; vals[nnz] = h; }
            nnz++;
        }
    return nnz;
}

/* ------------------------------------------------------------------ */
/* properties of the reference phi0 ("SC-NEVPT2(s)": E_0^(0) and the   */
/* active one-particle density that enters the generalized Fock        */
/* operator of the semicanonical virtual orbitals)                     */
/* ------------------------------------------------------------------ */
/* E_0^(0) = <phi0|H|phi0> / <phi0|phi0>: every pair of reference
 * determinants through the generic Slater-Condon routine. */
double orc_reference_energy(const orc_t *o) {
    int W2 = 2 * o->W;
    nsum num = {0, 0}, den = {0, 0};
    for (int64_t i = 0; i < o->n_ref; i++) {
        const uint64_t *a = o->ref + i * W2;
        nadd(&den, o->ref_c[i] * o->ref_c[i]);
        for (int64_t j = 0; j < o->n_ref; j++) {
            int ph, ne;
            double h = orc_hmat(o, a, o->ref + j * W2, &ph, &ne);
            if (ne <= 2 && h != 0.0) nadd(&num, o->ref_c[i] * h * o->ref_c[j]);
        }
    }
    return nval(&num) / nval(&den);
}

/* Spin-summed active one-particle density of phi0, normalised:
 * gamma[t*A + u] = sum_sigma <phi0| a+_{t sigma} a_{u sigma} |phi0> / <phi0|phi0>,
 * t, u active (0..A-1).  The operator is applied to every reference
 * determinant with its Jordan-Wigner sign and the result looked up. */
void orc_reference_rdm1(const orc_t *o, double *gamma) {
    int A = o->A, W2 = 2 * o->W;
    nsum *acc = (nsum *)calloc((size_t)A * A, sizeof(nsum));
    nsum den = {0, 0};
    uint64_t d[2 * MAXW];
    for (int64_t i = 0; i < o->n_ref; i++) {
        const uint64_t *b = o->ref + i * W2;
        double cb = o->ref_c[i];
        nadd(&den, cb * cb);
        for (int sg = 0; sg < 2; sg++)
            for (int u = 0; u < A; u++) {
                int gu = o->C + u + sg * o->N;
                if (!bit(o, b, gu)) continue;
                for (int t = 0; t < A; t++) {
                    int gt = o->C + t + sg * o->N;
                    memcpy(d, b, sizeof(uint64_t) * W2);
                    int sign = (below(o, d, gu) & 1) ? -1 : 1;   /* a_u */
                    flip(o, d, gu);
                    if (bit(o, d, gt)) continue;                  /* a+_t on an occupied orbital */
                    if (below(o, d, gt) & 1) sign = -sign;       /* a+_t */
                    flip(o, d, gt);
                    double ca = ref_lookup(o, d);
                    if (ca != 0.0) nadd(&acc[t * A + u], ca * sign * cb);
                }
            }
    }
    double n = nval(&den);
    for (int k = 0; k < A * A; k++) gamma[k] = nval(&acc[k]) / n;
    free(acc);
}


/* ------------------------------------------------------------------ */
/* Algorithmic data volume of one walker-step (bench roofline figure)   */
/* ------------------------------------------------------------------ */
/* Counts the DISTINCT operands the local-energy sums of one walker-step
 * read, in the frozen-core formulation: two-electron integrals over
 * non-core orbitals (8-fold canonical index), entries of the core-folded
 * one-body operator (canonical pair) and reference determinants whose
 * coefficient enters a nonzero term.  Each element counts once however
 * often it is used. */
typedef struct { uint64_t *k; int64_t cap, n; } uset;
static void uset_add(uset *s, uint64_t key) {
    key += 1;  /* 0 marks a free slot */
    if (2 * (s->n + 1) > s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 1024;
        uint64_t *nk = (uint64_t *)calloc((size_t)nc, sizeof(uint64_t));
        for (int64_t i = 0; i < s->cap; i++)
            if (s->k[i]) {
                uint64_t h = (s->k[i] * 0x9E3779B97F4A7C15ull) >> 20;
                int64_t j = (int64_t)(h & (uint64_t)(nc - 1));
                while (nk[j]) j = (j + 1) & (nc - 1);
                nk[j] = s->k[i];
            }
        free(s->k);
        s->k = nk;
        s->cap = nc;
    }
    uint64_t h = (key * 0x9E3779B97F4A7C15ull) >> 20;
    int64_t j = (int64_t)(h & (uint64_t)(s->cap - 1));
    while (s->k[j]) { if (s->k[j] == key) return; j = (j + 1) & (s->cap - 1); }
    s->k[j] = key;
    s->n++;
}
static uint64_t pair_idx(uint64_t a, uint64_t b) { return a > b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }
static void count_eri(const orc_t *o, uset *si, int P, int Q, int R, int S) {
    if (spin(o, P) != spin(o, Q) || spin(o, R) != spin(o, S)) return;
    uint64_t pq = pair_idx((uint64_t)(orb(o, P) - o->C), (uint64_t)(orb(o, Q) - o->C));
    uint64_t rs = pair_idx((uint64_t)(orb(o, R) - o->C), (uint64_t)(orb(o, S) - o->C));
    uset_add(si, pair_idx(pq, rs));
}
/* operands of <a|H|b> (a != b, at most doubly excited) */
static void count_hmat(const orc_t *o, const uint64_t *a, const uint64_t *b, uset *si, uset *sh) {
    int N2 = 2 * o->N, rem[3], add[3], nr = 0, na = 0;
    for (int g = 0; g < N2; g++) {
        int x = bit(o, a, g), y = bit(o, b, g);
        if (y && !x) { if (nr < 3) rem[nr] = g; nr++; }
        if (x && !y) { if (na < 3) add[na] = g; na++; }
    }
    if (nr == 1) {
        int P = rem[0], Q = add[0];
        uset_add(sh, pair_idx((uint64_t)(orb(o, P) - o->C), (uint64_t)(orb(o, Q) - o->C)));
        for (int J = 0; J < N2; J++) {
            if (!bit(o, b, J) || J == P || is_core(o, J)) continue;
            count_eri(o, si, Q, P, J, J);
            count_eri(o, si, Q, J, J, P);
        }
    } else if (nr == 2) {
        count_eri(o, si, add[0], rem[0], add[1], rem[1]);
        count_eri(o, si, add[0], rem[1], add[1], rem[0]);
    }
}
/* out[0] distinct two-electron integrals, out[1] distinct one-body entries,
 * out[2] distinct reference determinants, out[3] |M(n)|, out[4] nonzero
 * overlap terms (with repetition) */
void orc_traffic(const orc_t *o, const uint64_t *n, int64_t out[5]) {
    nbr_list L = {0, 0, 0};
    enumerate(o, n, &L);
    uset si = {0, 0, 0}, sh = {0, 0, 0}, sr = {0, 0, 0};
    int64_t terms = 0;
    int W2 = 2 * o->W, N2 = 2 * o->N;
    /* diagonal */
    for (int i = 0; i < N2; i++) {
        if (!bit(o, n, i) || is_core(o, i)) continue;
        uset_add(&sh, pair_idx((uint64_t)(orb(o, i) - o->C), (uint64_t)(orb(o, i) - o->C)));
        for (int j = 0; j < N2; j++) {
            if (!bit(o, n, j) || is_core(o, j)) continue;
            count_eri(o, &si, i, i, j, j);
            count_eri(o, &si, i, j, j, i);
        }
    }
    uint64_t d[2 * MAXW];
    for (int64_t k = 0; k < L.n; k++) {
        const uint64_t *m = L.v[k].det;
        count_hmat(o, m, n, &si, &sh);
        int nv = n_virt_el(o, m);
        if (nv == 0) {
            if (ref_lookup(o, m) != 0.0) {
                /* reference index as key */
                uint64_t key = 0;
                for (int w = 0; w < W2; w++) key = key * 0x100000001B3ull ^ m[w];
                uset_add(&sr, key);
                terms++;
            }
            continue;
        }
        int vir[2], nvir = 0, occa[MAXE], nocca = 0, hol[MAXE], nhol = 0;
        for (int g = 0; g < N2; g++) {
            if (is_virt(o, g) && bit(o, m, g)) vir[nvir++] = g;
            if (is_act(o, g)) { if (bit(o, m, g)) occa[nocca++] = g; else hol[nhol++] = g; }
        }
#define VISIT()                                                               \
        do {                                                                  \
            if (ref_lookup(o, d) != 0.0) {                                    \
                uint64_t key = 0;                                             \
                for (int w = 0; w < W2; w++) key = key * 0x100000001B3ull ^ d[w]; \
                uset_add(&sr, key);                                           \
                count_hmat(o, m, d, &si, &sh);                                \
                terms++;                                                      \
            }                                                                 \
        } while (0)
        if (nv == 1) {
            int X = vir[0];
            for (int i = 0; i < nhol; i++) {
                int T = hol[i];
                if (spin(o, T) != spin(o, X)) continue;
                memcpy(d, m, sizeof(uint64_t) * W2); flip(o, d, X); flip(o, d, T);
                VISIT();
            }
            for (int r = 0; r < nocca; r++)
                for (int i = 0; i < nhol; i++)
                    for (int j = i + 1; j < nhol; j++) {
                        int R = occa[r], T = hol[i], S = hol[j];
                        if (spin(o, T) + spin(o, S) != spin(o, X) + spin(o, R)) continue;
                        memcpy(d, m, sizeof(uint64_t) * W2);
                        flip(o, d, X); flip(o, d, R); flip(o, d, T); flip(o, d, S);
                        VISIT();
                    }
        } else {
            for (int i = 0; i < nhol; i++)
                for (int j = i + 1; j < nhol; j++) {
                    int T = hol[i], S = hol[j];
                    if (spin(o, T) + spin(o, S) != spin(o, vir[0]) + spin(o, vir[1])) continue;
                    memcpy(d, m, sizeof(uint64_t) * W2);
                    flip(o, d, vir[0]); flip(o, d, vir[1]); flip(o, d, T); flip(o, d, S);
                    VISIT();
                }
        }
#undef VISIT
    }
    out[0] = si.n; out[1] = sh.n; out[2] = sr.n; out[3] = L.n; out[4] = terms;
    free(si.k); free(sh.k); free(sr.k); free(L.v);
}
